// 3D stage-kernel instantiations, FP64, tile variant 4 (pair layout).
#include "dispatch_vol.hpp"

namespace esdg {

VolKernel stage_kernel_3d_f64_pairs(int N, int vf, int mesh) {
  return vol_pick<3, double, 4>(N, vf, mesh);
}

}  // namespace esdg
