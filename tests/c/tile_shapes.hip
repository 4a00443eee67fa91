// Host-only listing of the stage kernel's workgroup shapes: for every 3D
// degree, precision, volume flux and tile variant, the elements per
// workgroup, lanes, nodes per lane and the LDS the kernel declares for it
// (the same __shared__ arrays as stage_kernel).  tests/test_tiles_cpu.py
// checks them against the hardware limits.
#include <cstdio>

#include "kernels.hpp"

using namespace esdg;

template <int N, typename Real, int VF, int MESH, int V>
void one(const char* prec) {
  constexpr int DIM = 3;
  constexpr int NP = PrimCount<VF, DIM>::value;
  constexpr int EPB = tile_epb(DIM, N, NP, (int)sizeof(Real), V);
  constexpr int LAY = V == 4 ? ((N == 7 && sizeof(Real) == 8 && MESH == MESH_CURVED) ? LAY_PLANES : LAY_PAIRS)
                             : (V == 3 ? LAY_NODES : LAY_LINES);
  using T = Tile<DIM, N, EPB, LAY>;
  constexpr bool NODEL = LAY != LAY_LINES;
  constexpr bool CNODE = NODEL && MESH == MESH_CURVED;
  constexpr long rb = sizeof(Real);
  constexpr long NNL = T::NN + (LAY == LAY_PAIRS && N == 8 ? (T::NN / 64) * 8 : 0);  // padded rows (pairs, N = 8)
  constexpr long lds = (long)EPB * NP * NNL * rb                         // s_prim (s_acc aliases it)
                       + (long)EPB * T::NV * T::NFACE * rb               // s_face
                       + (long)EPB * 2 * DIM * 4                         // s_nbr
                       + (DtInLds<N, Real>::value ? N * N : 1) * rb      // s_dt
                       + (NODEL ? (LAY != LAY_NODES ? N * N : N * (N - 1)) : 1) * rb  // s_dts
                       + (CNODE ? (long)EPB * 2 * DIM * NNL : 1) * rb     // s_nrm
                       + (LAY == LAY_PAIRS && !T::PLANE ? (long)EPB * T::NV * T::NN : 1) * rb;  // s_vol (packed lines)
  std::printf("N %d prec %s vf %d mesh %d variant %d epb %d epb0 %d threads %d npt %d fpt %d nn %d lds %ld waves %d\n", N,
              prec, VF, MESH, V, EPB, TileShape<DIM, N>::EPB0, T::THREADS, T::NPT, T::FPT, T::NN, lds,
              StageWaves<DIM, N, MESH, Real, EPB, LAY>::value);
}

template <int N, typename Real, int VF, int MESH>
void variants(const char* prec) {
  one<N, Real, VF, MESH, 0>(prec);
  one<N, Real, VF, MESH, 1>(prec);
  one<N, Real, VF, MESH, 2>(prec);
  one<N, Real, VF, MESH, 3>(prec);
  one<N, Real, VF, MESH, 4>(prec);
}

template <int N>
void degree() {
  variants<N, double, VF_RANOCHA, MESH_CURVED>("fp64");
  variants<N, double, VF_SHIMA, MESH_AFFINE>("fp64");
  variants<N, float, VF_RANOCHA, MESH_CURVED>("fp32");
  variants<N, float, VF_SHIMA, MESH_AFFINE>("fp32");
}

int main() {
  degree<2>();
  degree<3>();
  degree<4>();
  degree<5>();
  degree<6>();
  degree<7>();
  degree<8>();
  return 0;
}
