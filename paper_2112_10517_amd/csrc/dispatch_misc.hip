// Reduction and utility kernel instantiations.
#include "dispatch.hpp"
#include "kernels.hpp"

namespace esdg {

namespace {

template <int DIM, typename Real>
const void* reduce_pick(int mesh, int op) {
  if (mesh == MESH_AFFINE) {
    switch (op) {
      case RED_TOTALS: return (const void*)&reduce_partial_kernel<DIM, MESH_AFFINE, RED_TOTALS, Real>;
      case RED_ENTROPY: return (const void*)&reduce_partial_kernel<DIM, MESH_AFFINE, RED_ENTROPY, Real>;
      case RED_MAXLAMBDA: return (const void*)&reduce_partial_kernel<DIM, MESH_AFFINE, RED_MAXLAMBDA, Real>;
    }
  } else {
    switch (op) {
      case RED_TOTALS: return (const void*)&reduce_partial_kernel<DIM, MESH_CURVED, RED_TOTALS, Real>;
      case RED_ENTROPY: return (const void*)&reduce_partial_kernel<DIM, MESH_CURVED, RED_ENTROPY, Real>;
      case RED_MAXLAMBDA: return (const void*)&reduce_partial_kernel<DIM, MESH_CURVED, RED_MAXLAMBDA, Real>;
    }
  }
  return nullptr;
}

__global__ void __launch_bounds__(256) to_fp64_kernel(const float* src, double* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}

__global__ void __launch_bounds__(256) to_fp32_kernel(const double* src, float* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

template <int DIM, typename Real, int MESH>
const void* face_pick(int N) {
  switch (N) {
    case 2: return (const void*)&face_kernel<DIM, 2, MESH, Real>;
    case 3: return (const void*)&face_kernel<DIM, 3, MESH, Real>;
    case 4: return (const void*)&face_kernel<DIM, 4, MESH, Real>;
    case 5: return (const void*)&face_kernel<DIM, 5, MESH, Real>;
    case 6: return (const void*)&face_kernel<DIM, 6, MESH, Real>;
    case 7: return (const void*)&face_kernel<DIM, 7, MESH, Real>;
    case 8: return (const void*)&face_kernel<DIM, 8, MESH, Real>;
  }
  return nullptr;
}

template <typename Real>
const void* face_pick_dim(int dim, int N, int mesh) {
  if (dim == 2) return mesh == MESH_AFFINE ? face_pick<2, Real, MESH_AFFINE>(N) : face_pick<2, Real, MESH_CURVED>(N);
  if (dim == 3) return mesh == MESH_AFFINE ? face_pick<3, Real, MESH_AFFINE>(N) : face_pick<3, Real, MESH_CURVED>(N);
  return nullptr;
}

}  // namespace

const void* face_kernel_for(int prec, int dim, int N, int mesh) {
  return prec == PREC_FP32 ? face_pick_dim<float>(dim, N, mesh) : face_pick_dim<double>(dim, N, mesh);
}

VolKernel stage_kernel_for(int prec, int dim, int N, int vf, int mesh, int variant) {
  if (variant < 0 || variant >= kTileVariants) return VolKernel{};
  if (dim == 2) {
    if (variant != 0) return VolKernel{};
    return prec == PREC_FP32 ? stage_kernel_2d_f32(N, vf, mesh) : stage_kernel_2d_f64(N, vf, mesh);
  }
  if (dim == 3) return prec == PREC_FP32 ? stage_kernel_3d_f32(N, vf, mesh, variant) : stage_kernel_3d_f64(N, vf, mesh, variant);
  return VolKernel{};
}

VolKernel gauss_kernel_for(int prec, int dim, int N, int vf, bool project) {
  if (dim != 2 && dim != 3) return VolKernel{};
  return prec == PREC_FP32 ? gauss_kernel_f32(dim, N, vf, project) : gauss_kernel_f64(dim, N, vf, project);
}

const void* reduce_partial_for(int prec, int dim, int mesh, int op) {
  if (prec == PREC_FP32) return dim == 2 ? reduce_pick<2, float>(mesh, op) : reduce_pick<3, float>(mesh, op);
  return dim == 2 ? reduce_pick<2, double>(mesh, op) : reduce_pick<3, double>(mesh, op);
}

const void* reduce_final_for(int op) {
  switch (op) {
    case RED_TOTALS: return (const void*)&reduce_final_kernel<RED_TOTALS>;
    case RED_ENTROPY: return (const void*)&reduce_final_kernel<RED_ENTROPY>;
    case RED_MAXLAMBDA: return (const void*)&reduce_final_kernel<RED_MAXLAMBDA>;
  }
  return nullptr;
}

const void* convert_kernel_for(int to_fp64) {
  return to_fp64 ? (const void*)&to_fp64_kernel : (const void*)&to_fp32_kernel;
}

}  // namespace esdg
