// 3D stage-kernel instantiations, FP64, tile variant 3 (node layout).
#include "dispatch_vol.hpp"

namespace esdg {

VolKernel stage_kernel_3d_f64_nodes(int N, int vf, int mesh) { return vol_pick<3, double, 3>(N, vf, mesh); }

}  // namespace esdg
