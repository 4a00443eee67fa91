// 3D stage-kernel instantiations, FP64, default tile.
#include "dispatch_vol.hpp"

namespace esdg {

VolKernel stage_kernel_3d_f64(int N, int vf, int mesh, int variant) {
  if (variant == 0) return vol_pick<3, double, 0>(N, vf, mesh);
  return stage_kernel_3d_f64_tuned(N, vf, mesh, variant);
}

}  // namespace esdg
