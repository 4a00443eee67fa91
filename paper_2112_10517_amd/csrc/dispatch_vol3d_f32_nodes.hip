// 3D stage-kernel instantiations, FP32 bulk precision, tile variant 3 (node
// layout).
#include "dispatch_vol.hpp"

namespace esdg {

VolKernel stage_kernel_3d_f32_nodes(int N, int vf, int mesh) { return vol_pick<3, float, 3>(N, vf, mesh); }

}  // namespace esdg
