// Legendre-Gauss collocation kernel instantiations (affine meshes, default
// tile) for one precision, included by the per-precision translation units.
#pragma once

#include "dispatch.hpp"
#include "kernels.hpp"

namespace esdg {

template <int DIM, typename Real, int N>
VolKernel gauss_stage_n(int vf) {
  constexpr int EPB = TileShape<DIM, N>::EPB0;
  using T = Tile<DIM, N, EPB>;
  VolKernel k;
  if (vf == VF_RANOCHA) k.fn = (const void*)&stage_kernel<DIM, N, VF_RANOCHA, MESH_AFFINE, Real, EPB, NODES_GAUSS>;
  else if (vf == VF_SHIMA) k.fn = (const void*)&stage_kernel<DIM, N, VF_SHIMA, MESH_AFFINE, Real, EPB, NODES_GAUSS>;
  else if (vf == VF_CENTRAL) k.fn = (const void*)&stage_kernel<DIM, N, VF_CENTRAL, MESH_AFFINE, Real, EPB, NODES_GAUSS>;
  else return VolKernel{};
  k.epb = T::EPB;
  k.threads = T::THREADS;
  return k;
}

template <int DIM, typename Real, int N>
VolKernel gauss_project_n() {
  using T = Tile<DIM, N>;
  VolKernel k;
  k.fn = (const void*)&gauss_project_kernel<DIM, N, Real>;
  k.epb = T::EPB;
  k.threads = T::THREADS;
  return k;
}

template <int DIM, typename Real>
VolKernel gauss_pick(int N, int vf, bool project) {
  switch (N) {
    case 2: return project ? gauss_project_n<DIM, Real, 2>() : gauss_stage_n<DIM, Real, 2>(vf);
    case 3: return project ? gauss_project_n<DIM, Real, 3>() : gauss_stage_n<DIM, Real, 3>(vf);
    case 4: return project ? gauss_project_n<DIM, Real, 4>() : gauss_stage_n<DIM, Real, 4>(vf);
    case 5: return project ? gauss_project_n<DIM, Real, 5>() : gauss_stage_n<DIM, Real, 5>(vf);
    case 6: return project ? gauss_project_n<DIM, Real, 6>() : gauss_stage_n<DIM, Real, 6>(vf);
    case 7: return project ? gauss_project_n<DIM, Real, 7>() : gauss_stage_n<DIM, Real, 7>(vf);
    case 8: return project ? gauss_project_n<DIM, Real, 8>() : gauss_stage_n<DIM, Real, 8>(vf);
    default: return VolKernel{};
  }
}

}  // namespace esdg
