// Stage-kernel instantiation table for one dimension (included by the
// per-dimension translation units so that they compile in parallel).
#pragma once

#include "dispatch.hpp"
#include "kernels.hpp"

namespace esdg {

template <int DIM, typename Real, int N>
VolKernel vol_pick_n(int vf, int mesh) {
  VolKernel k;
  k.epb = Tile<DIM, N>::EPB;
  k.threads = Tile<DIM, N>::THREADS;
  if (mesh == MESH_AFFINE) {
    if (vf == VF_RANOCHA) k.fn = (const void*)&stage_kernel<DIM, N, VF_RANOCHA, MESH_AFFINE, Real>;
    else if (vf == VF_SHIMA) k.fn = (const void*)&stage_kernel<DIM, N, VF_SHIMA, MESH_AFFINE, Real>;
    else if (vf == VF_CENTRAL) k.fn = (const void*)&stage_kernel<DIM, N, VF_CENTRAL, MESH_AFFINE, Real>;
  } else {
    if (vf == VF_RANOCHA) k.fn = (const void*)&stage_kernel<DIM, N, VF_RANOCHA, MESH_CURVED, Real>;
    else if (vf == VF_SHIMA) k.fn = (const void*)&stage_kernel<DIM, N, VF_SHIMA, MESH_CURVED, Real>;
    else if (vf == VF_CENTRAL) k.fn = (const void*)&stage_kernel<DIM, N, VF_CENTRAL, MESH_CURVED, Real>;
  }
  return k;
}

template <int DIM, typename Real>
VolKernel vol_pick(int N, int vf, int mesh) {
  switch (N) {
    case 2: return vol_pick_n<DIM, Real, 2>(vf, mesh);
    case 3: return vol_pick_n<DIM, Real, 3>(vf, mesh);
    case 4: return vol_pick_n<DIM, Real, 4>(vf, mesh);
    case 5: return vol_pick_n<DIM, Real, 5>(vf, mesh);
    case 6: return vol_pick_n<DIM, Real, 6>(vf, mesh);
    case 7: return vol_pick_n<DIM, Real, 7>(vf, mesh);
    case 8: return vol_pick_n<DIM, Real, 8>(vf, mesh);
    default: return VolKernel{};
  }
}

}  // namespace esdg
