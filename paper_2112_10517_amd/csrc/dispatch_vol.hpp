// Stage-kernel instantiation table for one dimension, precision and tile
// variant (included by the per-dimension translation units so that they
// compile in parallel).
#pragma once

#include "dispatch.hpp"
#include "kernels.hpp"

namespace esdg {

template <int DIM, typename Real, int N, int VF, int MESH, int V>
VolKernel vol_kernel() {
  constexpr int EPB = tile_epb(DIM, N, PrimCount<VF, DIM>::value, (int)sizeof(Real), V);
  // variant 3: node layout; variant 4: pair layout (at N = 7 one z-plane per
  // wave for the FP64 curved tiles, where it measured fastest)
  constexpr int LAY = V == 4 ? ((N == 7 && sizeof(Real) == 8 && MESH == MESH_CURVED) ? LAY_PLANES : LAY_PAIRS)
                             : (V == 3 ? LAY_NODES : LAY_LINES);
  using T = Tile<DIM, N, EPB, LAY>;
  VolKernel k;
  k.fn = (const void*)&stage_kernel<DIM, N, VF, MESH, Real, EPB, NODES_LGL, LAY>;
  k.epb = T::EPB;
  k.threads = T::THREADS;
  k.faces_once = FacesOnce<DIM, N, LAY>::value;
  // the priority twin of the default 3D line tiles (p <= 3, where launches of
  // one generation are common)
  if constexpr (DIM == 3 && N <= 4 && V == 0)
    k.fn_prio = (const void*)&stage_kernel<DIM, N, VF, MESH, Real, EPB, NODES_LGL, LAY, true>;
  return k;
}

template <int DIM, typename Real, int V, int N>
VolKernel vol_pick_n(int vf, int mesh) {
  if constexpr (V == 4 && DIM != 3) {
    return VolKernel{};  // the pair layout is 3D only
  } else {
  if (mesh == MESH_AFFINE) {
    if (vf == VF_RANOCHA) return vol_kernel<DIM, Real, N, VF_RANOCHA, MESH_AFFINE, V>();
    if (vf == VF_SHIMA) return vol_kernel<DIM, Real, N, VF_SHIMA, MESH_AFFINE, V>();
    if (vf == VF_CENTRAL) return vol_kernel<DIM, Real, N, VF_CENTRAL, MESH_AFFINE, V>();
  } else {
    if (vf == VF_RANOCHA) return vol_kernel<DIM, Real, N, VF_RANOCHA, MESH_CURVED, V>();
    if (vf == VF_SHIMA) return vol_kernel<DIM, Real, N, VF_SHIMA, MESH_CURVED, V>();
    if (vf == VF_CENTRAL) return vol_kernel<DIM, Real, N, VF_CENTRAL, MESH_CURVED, V>();
  }
  return VolKernel{};
  }
}

template <int DIM, typename Real, int V>
VolKernel vol_pick(int N, int vf, int mesh) {
  switch (N) {
    case 2: return vol_pick_n<DIM, Real, V, 2>(vf, mesh);
    case 3: return vol_pick_n<DIM, Real, V, 3>(vf, mesh);
    case 4: return vol_pick_n<DIM, Real, V, 4>(vf, mesh);
    case 5: return vol_pick_n<DIM, Real, V, 5>(vf, mesh);
    case 6: return vol_pick_n<DIM, Real, V, 6>(vf, mesh);
    case 7: return vol_pick_n<DIM, Real, V, 7>(vf, mesh);
    case 8: return vol_pick_n<DIM, Real, V, 8>(vf, mesh);
    default: return VolKernel{};
  }
}

}  // namespace esdg
