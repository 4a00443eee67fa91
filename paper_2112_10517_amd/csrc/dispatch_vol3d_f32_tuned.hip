// 3D stage-kernel instantiations, FP32 bulk precision, tile variants 1 and 2 (3 and 4 in their own units).
#include "dispatch_vol.hpp"

namespace esdg {

VolKernel stage_kernel_3d_f32_tuned(int N, int vf, int mesh, int variant) {
  if (variant == 1) return vol_pick<3, float, 1>(N, vf, mesh);
  if (variant == 2) return vol_pick<3, float, 2>(N, vf, mesh);
  if (variant == 3) return stage_kernel_3d_f32_nodes(N, vf, mesh);
  if (variant == 4) return stage_kernel_3d_f32_pairs(N, vf, mesh);
  return VolKernel{};
}

}  // namespace esdg
