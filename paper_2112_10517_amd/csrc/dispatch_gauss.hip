// Legendre-Gauss collocation kernels, FP64.
#include "dispatch_gauss.hpp"

namespace esdg {

VolKernel gauss_kernel_f64(int dim, int N, int vf, bool project) {
  return dim == 2 ? gauss_pick<2, double>(N, vf, project) : gauss_pick<3, double>(N, vf, project);
}

}  // namespace esdg
