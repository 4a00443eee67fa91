// 3D stage-kernel instantiations, FP32 bulk precision, tile variant 4 (pair layout, N = 8).
#include "dispatch_vol.hpp"

namespace esdg {

VolKernel stage_kernel_3d_f32_pairs(int N, int vf, int mesh) {
  return N == 8 ? vol_pick_n<3, float, 4, 8>(vf, mesh) : VolKernel{};
}

}  // namespace esdg
