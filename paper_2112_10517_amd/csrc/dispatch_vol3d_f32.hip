// 3D stage-kernel instantiations, FP32 bulk precision.
#include "dispatch_vol.hpp"

namespace esdg {

VolKernel stage_kernel_3d_f32(int N, int vf, int mesh) { return vol_pick<3, float>(N, vf, mesh); }

}  // namespace esdg
