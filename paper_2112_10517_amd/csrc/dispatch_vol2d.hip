// 2D stage-kernel instantiations, FP64 (2D tiles have a single variant).
#include "dispatch_vol.hpp"

namespace esdg {

VolKernel stage_kernel_2d_f64(int N, int vf, int mesh) { return vol_pick<2, double, 0>(N, vf, mesh); }

}  // namespace esdg
