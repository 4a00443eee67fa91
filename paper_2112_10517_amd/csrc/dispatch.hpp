// Lookup of kernel instantiations by runtime parameters.
#pragma once

namespace esdg {

enum Precision { PREC_FP64 = 0, PREC_FP32 = 1 };

struct VolKernel {
  const void* fn = nullptr;  // __global__ stage_kernel<...>
  int epb = 0;               // elements per workgroup
  int threads = 0;           // lanes per workgroup
  bool faces_once = false;   // reads f* written by the face kernel when given one
  // the same stage with the prologue at raised wave priority (stage_kernel
  // with PRIO), for launches whose workgroups are all resident at once; NULL
  // if not built for this tile
  const void* fn_prio = nullptr;
};

// number of tile variants of the 3D stage kernel (2D has one)
constexpr int kTileVariants = 5;

// stage kernel for the given parameters and tile variant (fn == NULL if none)
VolKernel stage_kernel_for(int prec, int dim, int N, int vf, int mesh, int variant);
VolKernel stage_kernel_2d_f64(int N, int vf, int mesh);
VolKernel stage_kernel_2d_f32(int N, int vf, int mesh);
VolKernel stage_kernel_3d_f64(int N, int vf, int mesh, int variant);
VolKernel stage_kernel_3d_f32(int N, int vf, int mesh, int variant);
VolKernel stage_kernel_3d_f64_tuned(int N, int vf, int mesh, int variant);
VolKernel stage_kernel_3d_f32_tuned(int N, int vf, int mesh, int variant);
VolKernel stage_kernel_3d_f64_nodes(int N, int vf, int mesh);
VolKernel stage_kernel_3d_f32_nodes(int N, int vf, int mesh);
VolKernel stage_kernel_3d_f64_pairs(int N, int vf, int mesh);
VolKernel stage_kernel_3d_f32_pairs(int N, int vf, int mesh);
// Legendre-Gauss collocation (affine meshes): the stage kernel, or with
// project = true the entropy-projection kernel that precedes it
VolKernel gauss_kernel_for(int prec, int dim, int N, int vf, bool project);
VolKernel gauss_kernel_f64(int dim, int N, int vf, bool project);
VolKernel gauss_kernel_f32(int dim, int N, int vf, bool project);
const void* reduce_partial_for(int prec, int dim, int mesh, int op);
const void* reduce_final_for(int op);
const void* convert_kernel_for(int to_fp64);  // elementwise precision casts
// face fluxes once per face (LGL): face_kernel<dim, N, mesh, precision>
const void* face_kernel_for(int prec, int dim, int N, int mesh);

}  // namespace esdg
