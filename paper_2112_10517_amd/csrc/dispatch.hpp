// Lookup of kernel instantiations by runtime parameters.
#pragma once

namespace esdg {

enum Precision { PREC_FP64 = 0, PREC_FP32 = 1 };

struct VolKernel {
  const void* fn = nullptr;  // __global__ volume_kernel<...>
  int epb = 0;               // elements per 64-lane workgroup
};

VolKernel volume_kernel_2d(int prec, int N, int vf, int mesh);
VolKernel volume_kernel_3d(int prec, int N, int vf, int mesh);
const void* face_kernel_for(int prec, int dim, int sf, int mesh);
const void* reduce_partial_for(int prec, int dim, int mesh, int op);
const void* reduce_final_for(int op);
const void* convert_kernel_for(int to_fp64);  // elementwise precision casts
const void* set_scalar_kernel();              // scal[idx] = value

inline int elements_per_block(int dim, int N) {
  int L = 1;
  for (int d = 1; d < dim; ++d) L *= N;
  return 64 / L > 0 ? 64 / L : 1;
}

}  // namespace esdg
