// Legendre-Gauss collocation kernels, FP32 bulk precision.
#include "dispatch_gauss.hpp"

namespace esdg {

VolKernel gauss_kernel_f32(int dim, int N, int vf, bool project) {
  return dim == 2 ? gauss_pick<2, float>(N, vf, project) : gauss_pick<3, float>(N, vf, project);
}

}  // namespace esdg
