// 3D stage-kernel instantiations.
#include "dispatch_vol.hpp"

namespace esdg {

VolKernel stage_kernel_3d(int prec, int N, int vf, int mesh) {
  if (prec == PREC_FP64) return vol_pick<3, double>(N, vf, mesh);
  return stage_kernel_3d_f32(N, vf, mesh);
}

}  // namespace esdg
