// 2D stage-kernel instantiations, FP32 bulk precision.
#include "dispatch_vol.hpp"

namespace esdg {

VolKernel stage_kernel_2d_f32(int N, int vf, int mesh) { return vol_pick<2, float, 0>(N, vf, mesh); }

}  // namespace esdg
