// 2D stage-kernel instantiations.
#include "dispatch_vol.hpp"

namespace esdg {

VolKernel stage_kernel_2d(int prec, int N, int vf, int mesh) {
  if (prec == PREC_FP64) return vol_pick<2, double>(N, vf, mesh);
  return stage_kernel_2d_f32(N, vf, mesh);
}

}  // namespace esdg
