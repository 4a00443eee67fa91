// Device kernels of the flux-differencing LGL-DGSEM (gfx950, wave64).
//
// One launch per right-hand side or RK stage, stage_kernel<DIM,N,VF,MESH>:
// a workgroup owns EPB elements (Tile<DIM,N>) and
//   prologue  loads u coalesced and computes the primitive variables,
//             log(rho), beta = rho/p and log(beta) once per node into LDS
//             (Sec. 7.1/7.2 precomputation);
//   lines     one lane per (direction, element, line): the lane evaluates the
//             N(N-1)/2 pairs i<k of its line once each, with the two-point
//             volume flux in the direction of the averaged contravariant
//             vectors (Sec. 2.3 rearranged form; skew-symmetric D~ with zero
//             diagonal, Sec. 2.2), accumulating D~_ik F and D~_ki F in
//             registers; all directions run concurrently and are summed per
//             node in a fixed order (deterministic, no atomics);
//   surface   one lane per face node evaluates f*(u_L, u_R, n_face) from the
//             conservative traces of both elements; both elements of a face
//             evaluate it with identical inputs, so f* is bitwise shared and
//             the surface terms telescope exactly (computing it on each side
//             avoids a launch and a round trip of f* through HBM);
//   epilogue  lifting (+f*/w_p, -f*/w_0), scaling by -1/J and the fused RK
//             stage update.
// MFMA is not used: the volume term is an element-wise two-point flux
// followed by a row-sum, not a dense contraction.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace esdg {

enum VolFlux { VF_RANOCHA = 0, VF_SHIMA = 1, VF_CENTRAL = 3 };
enum SurfFlux { SF_RANOCHA = 0, SF_SHIMA = 1, SF_LLF = 2, SF_CENTRAL = 3 };
enum MeshKind { MESH_AFFINE = 0, MESH_CURVED = 1 };
// RK4 stages (classical scheme in low-storage form) and the stages of the
// 2N-storage scheme (du <- A du + dt k; u <- u + B du; A = coef_a, B = coef_b)
enum StageMode {
  MODE_RHS = 0,
  MODE_RK_FIRST = 1,
  MODE_RK_MID = 2,
  MODE_RK_LAST = 3,
  MODE_LS_FIRST = 4,
  MODE_LS_MID = 5,
  MODE_LS_LAST = 6
};
enum RedOp { RED_TOTALS = 0, RED_ENTROPY = 1, RED_MAXLAMBDA = 2 };

constexpr int kDevMaxN = 8;
constexpr int kLamSlots = 64;  // CFL maxima are spread over this many slots (atomic contention)

template <typename Real>
struct StageOps {
  Real Dt[kDevMaxN * kDevMaxN];  // LGL: D~; Gauss: T = M^-1 (M D - (M D)^T); row-major
  Real inv_w0, inv_wp;           // 1/w_0, 1/w_p
  Real gamma, inv_gm1;           // gamma, 1/(gamma-1)
  // Gauss collocation: Lagrange basis at -1 / +1 (R) and M^-1 R^T B, and R
  // in FP64 for the entropy projection
  Real rL[kDevMaxN], rR[kDevMaxN], cL[kDevMaxN], cR[kDevMaxN];
  double r64[2][kDevMaxN];
};

enum NodeKind { NODES_LGL = 0, NODES_GAUSS = 1 };

// One problem of a launch (device memory).  A launch covers the tiles of one
// or more problems of equal degree, flux, mesh kind and precision; a problem
// computes the same values whether it runs alone or with others.
template <typename Real>
struct ProbDesc {
  Real* buf[5];              // U (state), Y, Y2 (stage states), R (RK accumulator), DU (RHS): [E][nv][nn]
  const Real* metric;        // curved: [E][dim*dim+1][nn] (Ja^n_m, then 1/J)
  const Real* nface;         // curved: [dim][E][dim][nf] normal of the + face of each element
  unsigned long long* lam;   // CFL: 2 x kLamSlots slots by step parity (bit patterns of non-negative doubles)
  double* time;              // time of the state, 2 slots by step parity
  int* flag;                 // non-physical state flag (host-mapped memory; kernels store 1)
  Real* faceb;               // Gauss: entropy-projected face states [E][2 dim][dim+4][nf] (rho, v, p, log rho, log beta)
  double t_end;              // a step never passes t_end: dt = min(dt, t_end - t)
  int E, n0, n1, n2;         // elements, per direction
  int tile0;                 // first tile of this problem in the launch
  int pad;
  Real scale[3];             // affine: 2/h_n ; curved: 1
};

template <typename Real>
struct StageArgs {
  const ProbDesc<Real>* probs;  // problems of the launch, ordered by tile0
  const int* tile_prob;         // problem index of every tile; NULL for a single problem
  Real* out_ext;        // RHS mode of a single problem: output; else NULL (buf[out_idx])
  // face fluxes evaluated once per face: f* of every element's + faces,
  // [E][DIM][NV][NF], written by face_kernel before the stage launch; NULL:
  // every element evaluates the fluxes of its own faces (both sides of a face)
  Real* fstar;
  int in_idx, out_idx;  // ProbDesc::buf indices of the stage input and output
  int mode;             // StageMode
  int surf;             // SurfFlux
  Real coef_b, coef_a;  // RK: acc += b dt k ; y = u0 + a dt k
  // time step: fixed (cfl <= 0) or dt = cfl 2 / (N lam) with lam the largest
  // sum over directions of wave speeds of the step's start state, the maximum
  // over the problem's kLamSlots slots of parity par; then clipped to t_end
  double dt_fixed, cfl;
  double gamma64;       // gamma in FP64 (the CFL wave speeds are FP64 in both precisions)
  int par;              // step parity: time and CFL slots of the step's start state
  int lam_update;       // LAST stage: atomic max of the new state's value into parity 1 - par
  StageOps<Real> ops;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Global-memory view of a pointer read from a descriptor: accesses through it
// compile to global_* instructions.  Through the generic pointer they would be
// flat_* instructions, which also count against the LDS wait counter, so every
// LDS wait would wait for the outstanding global loads as well.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* as_global(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

template <int B, int K>
struct Pow { static constexpr int value = B * Pow<B, K - 1>::value; };
template <int B>
struct Pow<B, 0> { static constexpr int value = 1; };

// Series cutoff of the log means: u = ((a+ - a-)/(a+ + a-))^2 < eps, eps =
// 1e-4 in FP64 (Sec. 3.1) and 2e-2 in FP32; tested as |a+ - a-| < sqrt(eps)
// (a+ + a-) (both arguments positive)
template <typename Real> struct LogMeanCut;
template <> struct LogMeanCut<double> { static constexpr double value = 1.0e-2; };
template <> struct LogMeanCut<float> { static constexpr float value = 0.14142135623730950f; };

__device__ __forceinline__ double dev_log(double x) { return log(x); }
__device__ __forceinline__ float dev_log(float x) { return logf(x); }
__device__ __forceinline__ double dev_exp(double x) { return exp(x); }
__device__ __forceinline__ float dev_exp(float x) { return expf(x); }

// Reciprocal: hardware estimate refined by Newton's iteration r <- r(2 - q r)
// written as two fused multiply-adds (two steps in FP64; the FP32 estimate
// is used as is).
__device__ __forceinline__ double dev_rcp(double q) {
  double r = __builtin_amdgcn_rcp(q);
  double e = fma(-q, r, 1.0);
  r = fma(r, e, r);
  e = fma(-q, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float dev_rcp(float q) {
  return __builtin_amdgcn_rcpf(q);  // 1 ulp: below the FP32 parity bar, no refinement
}

// Primitive variables at one node, with log(rho), beta = rho/p and log(beta)
// when the volume flux needs log means.
template <typename Real>
struct Prim {
  Real rho, v0, v1, v2, p, lr, b, lb;
};

// ---------------------------------------------------------------------------
// two-point volume fluxes in direction n (Sec. 3.2), from primitive values
// ---------------------------------------------------------------------------

// a b + c with one rounding
__device__ __forceinline__ double mad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float mad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// The two-point flux code below compiles with contraction off and states
// every fused multiply-add explicitly: left to the compiler, which products
// get fused depends on the code around an inlined call, and the kernel
// layouts (which inline the flux into different loops) must give the same
// bits.

// Log mean and inverse log mean (Sec. 3.1, Algorithms 2 and 3) with the
// node logarithms precomputed (Sec. 7.2).  The branch of the algorithms,
// u = ((a+ - a-)/(a+ + a-))^2 < eps, is decided without a division as
// |a+ - a-| < sqrt(eps) (a+ + a-); each mean then costs one reciprocal:
//   LM : series (a- + a+)(1/2 - u/6 - 2u^2/45 - 22u^3/945)  [the division-free
//        variant of Algorithm 2 given in Sec. 3.1]   or   (a+ - a-) / (la+ - la-)
//   ILM: series (2 + 2u/3 + 2u^2/5 + 2u^3/7)/(a- + a+)   or   (la+ - la-)/(a+ - a-)
// Swapping the two arguments (and their logarithms) flips the sign of d and
// of the log difference together, so both means are bitwise symmetric.
template <typename Real>
__device__ __forceinline__ Real log_mean_pre(Real am, Real ap, Real lam, Real lap) {
#pragma clang fp contract(off)
  const Real s = am + ap, d = ap - am;
  const bool series = fabs(d) < LogMeanCut<Real>::value * s;
  const Real r = dev_rcp(series ? s : (lap - lam));
  const Real f = d * r;
  const Real u = f * f;
  Real poly;
  {
    // Horner's scheme with fused multiply-adds formed within the expression
    // (the fmuladd form keeps the register use of the stage kernels low,
    // where explicit fma calls make them spill)
#pragma clang fp contract(on)
    poly = Real(0.5) + u * (Real(-1.0 / 6.0) + u * (Real(-2.0 / 45.0) + u * Real(-22.0 / 945.0)));
  }
  return series ? s * poly : f;
}

// SEL: pick the series polynomial or the log difference, then multiply once
// (the same product as the two-branch form, so the same bits).  The compiler
// makes a branch of the two-branch form (the log difference, and its LDS
// load, on one side).  The FP64 node and pair loops run branch-free with SEL
// (1.5-2.5% faster at p = 6-7); in FP32, where the series branch covers
// nearly every pair, and in the line tiles, the branch measured as fast or
// faster, at fewer registers.
template <typename Real, bool SEL = false>
__device__ __forceinline__ Real inv_log_mean_pre(Real am, Real ap, Real lam, Real lap) {
#pragma clang fp contract(off)
  const Real s = am + ap, d = ap - am;
  const bool series = fabs(d) < LogMeanCut<Real>::value * s;
  const Real r = dev_rcp(series ? s : d);
  const Real f = d * r;
  const Real u = f * f;
  Real poly;
  {
#pragma clang fp contract(on)  // as in log_mean_pre
    poly = Real(2) + u * (Real(2.0 / 3.0) + u * (Real(2.0 / 5.0) + u * Real(2.0 / 7.0)));
  }
  if (SEL) return r * (series ? poly : lap - lam);
  return series ? r * poly : (lap - lam) * r;
}

// v . n of one state
template <int DIM, typename Real>
__device__ __forceinline__ Real dot_n(Real v0, Real v1, Real v2, Real nx, Real ny, Real nz) {
#pragma clang fp contract(off)
  Real r = v0 * nx;
  if (DIM > 1) r = mad(v1, ny, r);
  if (DIM > 2) r = mad(v2, nz, r);
  return r;
}

// Directional volume flux f(u_i, u_k, n) into F[0..DIM+1].  NX/NY/NZ are the
// normal components (compile-time constants for the affine mesh).  Every
// expression is symmetric in the two states down to the rounding (sums and
// products of the two sides commute, fused products pair a value of one side
// with the same value of the other, mixed products p_a (v.n)_b + p_b (v.n)_a
// are rounded before their sum), so f(u_a, u_b, n) and f(u_b, u_a, n) are
// bitwise equal: a kernel may evaluate a pair from either end and get the
// bits of the other.
template <int VF, int DIM, typename Real, bool SEL = false>
__device__ __forceinline__ void volume_flux(const Prim<Real>& a, const Prim<Real>& b, Real nx, Real ny,
                                            Real nz, Real inv_gm1, Real* F) {
#pragma clang fp contract(off)
  const Real vna = dot_n<DIM>(a.v0, a.v1, a.v2, nx, ny, nz);
  const Real vnb = dot_n<DIM>(b.v0, b.v1, b.v2, nx, ny, nz);
  const Real vn_avg = Real(0.5) * (vna + vnb);
  const Real p_avg = Real(0.5) * (a.p + b.p);
  const Real vv = dot_n<DIM>(a.v0, a.v1, a.v2, b.v0, b.v1, b.v2);
  const Real pvn = Real(0.5) * (b.p * vna + a.p * vnb);  // ((p; v.n))
  if (VF == VF_CENTRAL) {
    // (f(u_a) + f(u_b)).n / 2 with f written in primitive variables
    const Real ka = a.rho * vna, kb = b.rho * vnb;
    F[0] = Real(0.5) * (ka + kb);
    F[1] = mad(p_avg, nx, Real(0.5) * (ka * a.v0 + kb * b.v0));
    if (DIM > 1) F[2] = mad(p_avg, ny, Real(0.5) * (ka * a.v1 + kb * b.v1));
    if (DIM > 2) F[3] = mad(p_avg, nz, Real(0.5) * (ka * a.v2 + kb * b.v2));
    const Real va2 = dot_n<DIM>(a.v0, a.v1, a.v2, a.v0, a.v1, a.v2);
    const Real vb2 = dot_n<DIM>(b.v0, b.v1, b.v2, b.v0, b.v1, b.v2);
    const Real ea = mad(a.p, inv_gm1, Real(0.5) * a.rho * va2) + a.p;
    const Real eb = mad(b.p, inv_gm1, Real(0.5) * b.rho * vb2) + b.p;
    F[DIM + 1] = Real(0.5) * (ea * vna + eb * vnb);
    return;
  }
  Real frho, fe_int;
  if (VF == VF_RANOCHA) {
    frho = log_mean_pre(a.rho, b.rho, a.lr, b.lr) * vn_avg;
    // Sec. 3.2 writes 1/{{rho/p}}_log as p_a p_b / {{rho_a p_b, rho_b p_a}}_log;
    // the log mean is homogeneous of degree one, so that is 1/{{beta}}_log
    // with beta = rho/p taken once per node
    const Real ilm = inv_log_mean_pre<Real, SEL>(a.b, b.b, a.lb, b.lb);
    fe_int = frho * ilm * inv_gm1;
  } else {  // Shima et al.
    frho = Real(0.5) * (a.rho + b.rho) * vn_avg;
    fe_int = p_avg * vn_avg * inv_gm1;
  }
  const Real hf = Real(0.5) * frho;
  F[0] = frho;
  F[1] = mad(hf, a.v0 + b.v0, p_avg * nx);
  if (DIM > 1) F[2] = mad(hf, a.v1 + b.v1, p_avg * ny);
  if (DIM > 2) F[3] = mad(hf, a.v2 + b.v2, p_avg * nz);
  F[DIM + 1] = mad(hf, vv, fe_int) + pvn;
}

// ---------------------------------------------------------------------------
// surface flux from conservative traces
// ---------------------------------------------------------------------------

template <int DIM, typename Real>
__device__ __forceinline__ void cons_to_prim(const Real* u, Real gm1, Prim<Real>& P) {
  P.rho = u[0];
  const Real ir = dev_rcp(P.rho);
  P.v0 = u[1] * ir;
  P.v1 = DIM > 1 ? u[2] * ir : Real(0);
  P.v2 = DIM > 2 ? u[3] * ir : Real(0);
  P.p = gm1 * (u[DIM + 1] - Real(0.5) * (u[1] * P.v0 + (DIM > 1 ? u[2] * P.v1 : Real(0)) +
                                          (DIM > 2 ? u[3] * P.v2 : Real(0))));
  P.lr = P.b = P.lb = Real(0);
}

// f*(u_L, u_R, n) of kind sf (runtime, uniform across the launch)
template <int DIM, typename Real>
__device__ __forceinline__ void surface_flux(int sf, const Real* uL, const Real* uR, Real nx, Real ny, Real nz,
                                             Real gamma, Real inv_gm1, Real* F) {
  const Real gm1 = gamma - Real(1);
  Prim<Real> PL, PR;
  cons_to_prim<DIM>(uL, gm1, PL);
  cons_to_prim<DIM>(uR, gm1, PR);
  if (sf == SF_RANOCHA) {
    PL.lr = dev_log(PL.rho);
    PL.b = PL.rho * dev_rcp(PL.p);
    PL.lb = dev_log(PL.b);
    PR.lr = dev_log(PR.rho);
    PR.b = PR.rho * dev_rcp(PR.p);
    PR.lb = dev_log(PR.b);
    volume_flux<VF_RANOCHA, DIM>(PL, PR, nx, ny, nz, inv_gm1, F);
  } else if (sf == SF_SHIMA) {
    volume_flux<VF_SHIMA, DIM>(PL, PR, nx, ny, nz, inv_gm1, F);
  } else {
    volume_flux<VF_CENTRAL, DIM>(PL, PR, nx, ny, nz, inv_gm1, F);
    if (sf == SF_LLF) {
      const Real vnL = PL.v0 * nx + PL.v1 * ny + PL.v2 * nz;
      const Real vnR = PR.v0 * nx + PR.v1 * ny + PR.v2 * nz;
      const Real cL = sqrt(gamma * PL.p * dev_rcp(PL.rho)), cR = sqrt(gamma * PR.p * dev_rcp(PR.rho));
      const Real nn = sqrt(nx * nx + ny * ny + nz * nz);
      const Real lam = fmax(fabs(vnL), fabs(vnR)) + fmax(cL, cR) * nn;
#pragma unroll
      for (int v = 0; v < DIM + 2; ++v) F[v] -= Real(0.5) * lam * (uR[v] - uL[v]);
    }
  }
}

// f*(u_L, u_R, n) of kind sf from primitive states with their logarithms
// (Gauss collocation: the face states are entropy projections, Sec. 6)
template <int DIM, typename Real>
__device__ __forceinline__ void surface_flux_prim(int sf, const Prim<Real>& PL, const Prim<Real>& PR, Real nx,
                                                  Real ny, Real nz, Real gamma, Real inv_gm1, Real* F) {
  if (sf == SF_RANOCHA) {
    volume_flux<VF_RANOCHA, DIM>(PL, PR, nx, ny, nz, inv_gm1, F);
  } else if (sf == SF_SHIMA) {
    volume_flux<VF_SHIMA, DIM>(PL, PR, nx, ny, nz, inv_gm1, F);
  } else {
    volume_flux<VF_CENTRAL, DIM>(PL, PR, nx, ny, nz, inv_gm1, F);
    if (sf == SF_LLF) {
      const Real vnL = PL.v0 * nx + PL.v1 * ny + PL.v2 * nz;
      const Real vnR = PR.v0 * nx + PR.v1 * ny + PR.v2 * nz;
      const Real cL = sqrt(gamma * PL.p * dev_rcp(PL.rho)), cR = sqrt(gamma * PR.p * dev_rcp(PR.rho));
      const Real nn = sqrt(nx * nx + ny * ny + nz * nz);
      const Real lam = fmax(fabs(vnL), fabs(vnR)) + fmax(cL, cR) * nn;
      const Real h = Real(0.5) * lam;
      F[0] -= h * (PR.rho - PL.rho);
      F[1] -= h * (PR.rho * PR.v0 - PL.rho * PL.v0);
      if (DIM > 1) F[DIM > 1 ? 2 : 0] -= h * (PR.rho * PR.v1 - PL.rho * PL.v1);
      if (DIM > 2) F[DIM > 2 ? 3 : 0] -= h * (PR.rho * PR.v2 - PL.rho * PL.v2);
      const Real eL = PL.p * inv_gm1 + Real(0.5) * PL.rho * (PL.v0 * PL.v0 + PL.v1 * PL.v1 + PL.v2 * PL.v2);
      const Real eR = PR.p * inv_gm1 + Real(0.5) * PR.rho * (PR.v0 * PR.v0 + PR.v1 * PR.v1 + PR.v2 * PR.v2);
      F[DIM + 1] -= h * (eR - eL);
    }
  }
}

// ---------------------------------------------------------------------------
// fused stage kernel
// ---------------------------------------------------------------------------

// Tile of one workgroup: EPB elements.  The line phase gives one lane to each
// (direction, element, line); the lanes of one direction fill whole waves, so
// a wave never diverges on the direction.  Node and face-node work is spread
// over all lanes of the workgroup.
template <int DIM, int N>
struct TileShape {
  static constexpr int NN = Pow<N, DIM>::value;   // nodes per element
  static constexpr int L = NN / N;                // lines per direction
  static constexpr int EPB0 = (64 / L) > 0 ? 64 / L : 1;  // default elements per block: one wave per direction
};

// Work layout of the volume term.  LAY_LINES: one lane per (direction,
// element, line) evaluates each i<k pair of its line once and scatters to
// both nodes.  LAY_NODES: one lane per node sweeps its N-1 partners along
// each direction in turn and accumulates its own row only; every pair is
// evaluated from both ends (twice the flux evaluations), in exchange for a
// register footprint of one node instead of one line, hence more waves per
// SIMD at high degree.  Both layouts add the same terms in the same order, so
// they give the same bits.  LAY_PAIRS (3D): one lane per node as in
// LAY_NODES, but the lanes of a line evaluate each pair once in a rotation
// schedule and hand the flux to the partner lane with a cross-lane permute
// (pair_fluxes); half the flux evaluations of LAY_NODES, the same values up to
// the order of the sums.  At N = 8 a wave holds one z-plane of the element,
// so the x- and y-lines lie in one wave; below, floor(64/N) whole lines of
// one direction are packed per wave and the directions' sums merged in LDS.
// LAY_PLANES (N = 7): the pair layout with one z-plane (49 nodes) per wave
// and lanes 49 .. 63 idle, no merge buffer; faster than packed lines for the
// FP64 curved tiles only.
enum Layout { LAY_LINES = 0, LAY_NODES = 1, LAY_PAIRS = 2, LAY_PLANES = 3 };

template <int DIM, int N, int EPB_ = TileShape<DIM, N>::EPB0, int LAY_ = LAY_LINES>
struct Tile {
  static constexpr int NN = Pow<N, DIM>::value;   // nodes per element
  static constexpr int NF = NN / N;               // nodes per face
  static constexpr int L = NN / N;                // lines per direction
  static constexpr int NFACE = 2 * DIM * NF;      // face nodes per element
  static constexpr int EPB = EPB_;                // elements per block
  static constexpr int LAY = LAY_;
  // lanes per direction (line layout); the node and pair layouts have one
  // group of lanes: one per node, in the pair layout with packed lines also
  // enough for the lines of one direction packed floor(64/N) to a wave, and
  // in the plane layouts N waves of 64 lanes
  static constexpr int NODE_LANES = ((EPB * NN + 63) / 64) * 64;
  static constexpr int LPW = 64 / N;  // pair layout: whole lines per wave
  static constexpr int PAIR_LANES = ((EPB * L + LPW - 1) / LPW) * 64;
  // pair layout, one element per workgroup, wave w = z-plane w (lanes
  // 0 .. N^2-1 of each wave hold the plane's nodes)
  static constexpr bool PLANE = DIM == 3 && ((LAY == LAY_PAIRS && N == 8) || (LAY == LAY_PLANES && N * N <= 64));
  static constexpr int LANES_DIR = LAY == LAY_LINES ? ((EPB * L + 63) / 64) * 64
                                   : (PLANE ? N * 64
                                            : (LAY != LAY_NODES && PAIR_LANES > NODE_LANES ? PAIR_LANES : NODE_LANES));
  static constexpr int THREADS = LAY == LAY_LINES ? DIM * LANES_DIR : LANES_DIR;
  static constexpr int NPT = (EPB * NN + THREADS - 1) / THREADS;     // nodes per lane
  static constexpr int FPT = (EPB * NFACE + THREADS - 1) / THREADS;  // face nodes per lane
  static constexpr int NV = DIM + 2;
  // waves per SIMD the register allocation must allow: every workgroup of a
  // typical launch resident at once (3 x 64-lane waves per SIMD for N <= 4);
  // node layout: two workgroups of up to 8 waves per CU
  static constexpr int WPE = LAY != LAY_LINES ? 4 : (N <= 4 ? 3 : (N <= 6 ? 2 : 1));
  static_assert(LAY == LAY_LINES || NPT == 1, "node layout: one node per lane");
  static_assert(!PLANE || EPB == 1, "plane layout: one element (N waves) per block");
  static_assert(LAY != LAY_PLANES || PLANE, "LAY_PLANES: 3D, N = 7 or 8");
};

// Lane slot q (= tid + r THREADS) holds node q of the tile (element-major),
// except in the plane layout: there lane l of wave w holds node l + N^2 w of
// the one element and the lanes l >= N^2 hold none (false).
template <int N>
__device__ __forceinline__ bool plane_node(int q, int& i) {
  const int w = q >> 6, l = q & 63;
  i = l + w * (N * N);
  return l < N * N && w < N;
}

// LDS budget of one workgroup of a tile variant (two workgroups fit a CU)
constexpr int kTileLdsCap = 80 * 1024;

// Elements per workgroup of tile variant `variant` (0: one wave per
// direction; 1: the fewest elements that fill >= 90% of the lanes of whole
// waves; 2: twice the default), falling back to the default when the LDS of
// the variant would exceed kTileLdsCap.  Every variant computes the same
// values; only the speed differs.
constexpr int tile_epb(int dim, int N, int np, int rbytes, int variant) {
  int nn = 1;
  for (int j = 0; j < dim; ++j) nn *= N;
  const int L = nn / N, nv = dim + 2, nface = 2 * dim * L;
  const int epb0 = 64 / L > 0 ? 64 / L : 1;
  const int per = (np * nn + nv * nface) * rbytes + 2 * dim * 4;  // primitives (volume sums alias them), face fluxes
  if (variant == 1) {
    for (int e = epb0; e <= 32; ++e) {
      const int lanes = (e * L + 63) / 64 * 64;
      if (10 * e * L >= 9 * lanes) return e * per <= kTileLdsCap ? e : epb0;
    }
    return epb0;
  }
  if (variant == 2) return 2 * epb0 * per <= kTileLdsCap ? 2 * epb0 : epb0;
  // pair layout (3D): from N = 6 one element (at N = 8, and at N = 7 in the
  // LAY_PLANES tiles, a wave per z-plane); below, the elements that fill
  // whole waves best with one lane per node and with floor(64/N) lines per
  // wave
  if (variant == 4) return N >= 6 ? 1 : (N == 5 ? 2 : (N == 4 ? 4 : (N == 3 ? 7 : 16)));
  if (variant == 3) {
    // node layout (LDS: primitives, two direction buffers of halved
    // contravariant vectors, face fluxes): the smallest tile of at least 128
    // lanes (and at most 1024, within the LDS budget) that keeps >= 80% of its
    // lanes busy -- small workgroups pack more of them per CU (measured: p = 5
    // FP64 one element 7% faster than two); else the one that leaves the
    // fewest lanes idle
    const int pn = ((np + 2 * dim) * nn + nv * nface) * rbytes + 2 * dim * 4;
    int best = 1;
    long best_num = 0, best_den = 1;
    for (int e = 1; e <= 32 && e * nn <= 1024; ++e) {
      const int lanes = (e * nn + 63) / 64 * 64;
      if ((lanes < 128 && (e + 1) * nn <= 1024) || (e > 1 && e * pn > kTileLdsCap)) continue;
      if (5 * e * nn >= 4 * lanes) return e;
      if ((long)e * nn * best_den > best_num * (long)lanes) {
        best = e;
        best_num = (long)e * nn;
        best_den = lanes;
      }
    }
    return best;
  }
  return epb0;
}

// D~ is a scalar operand of the pair loop (N^2 values in scalar registers)
// except for N = 8: in FP64 its 128 scalar registers exceed a wave's, and
// the code generated at -O2/-O3 for the spilled operands gave wrong volume
// sums (correct at -O1 and with D~ in LDS); in FP32 its 64 registers left
// the line tiles 15-30 scalar registers short, and one of them gave wrong
// sums after an unrelated change.  N = 8 tiles read D~ from LDS (no scalar
// spills).
template <int N, typename Real>
struct DtInLds { static constexpr bool value = N >= 8; };

template <int VF, int DIM>
struct PrimCount { static constexpr int value = (VF == VF_RANOCHA) ? DIM + 5 : DIM + 2; };

// node of face node f (other digits, lowest direction first) with digit `pos` in direction dir
template <int N>
__device__ __forceinline__ int face_node(int dir, int f, int pos) {
  const int sa = dir == 0 ? 1 : (dir == 1 ? N : N * N);
  return (f % sa) + pos * sa + (f / sa) * sa * N;
}

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of tiles so that neighbouring elements (whose traces a
// tile reads) are processed by the same XCD and hit its L2.
__device__ __forceinline__ int xcd_tile(int b, int G) {
  const int q = G >> 3;
  return b < (q << 3) ? (b & 7) * q + (b >> 3) : b;
}

// CFL wave-speed sum of one node, sum_n (|v.Ja^n| + c |Ja^n|) / J (affine:
// sum_n (|v_n| + c) 2/h_n), from its conservative state, evaluated in FP64
// for both state precisions (the time step is an FP64 reduction).  me points
// at the node's first metric entry (stride nn between entries; curved
// meshes).  The last RK stage and the CFL reduction both use this one
// expression, so the step size of a state is the same whichever of them
// computed it.
template <int DIM, int MESH, typename Real, typename MP>
__device__ __forceinline__ double cfl_rate(const Real (&ur)[DIM + 2], MP me, int64_t nn, Real rinvj_r,
                                           const Real* scale, double gamma) {
  double u[DIM + 2];
#pragma unroll
  for (int v = 0; v < DIM + 2; ++v) u[v] = (double)ur[v];
  const double gm1 = gamma - 1.0;
  const double rho = u[0], ir = dev_rcp(rho);
  const double w0 = u[1] * ir;
  const double w1 = DIM > 1 ? u[DIM > 1 ? 2 : 1] * ir : 0.0;
  const double w2 = DIM > 2 ? u[DIM > 2 ? 3 : 1] * ir : 0.0;
  const double pr = gm1 * (u[DIM + 1] - 0.5 * rho * (w0 * w0 + w1 * w1 + w2 * w2));
  const double c = sqrt(gamma * pr * ir);
  double lam = 0.0;
  if (MESH == MESH_CURVED) {
#pragma unroll
    for (int n = 0; n < DIM; ++n) {
      const double j0 = (double)me[(n * DIM) * nn];
      const double j1 = DIM > 1 ? (double)me[(n * DIM + (DIM > 1 ? 1 : 0)) * nn] : 0.0;
      const double j2 = DIM > 2 ? (double)me[(n * DIM + (DIM > 2 ? 2 : 0)) * nn] : 0.0;
      lam += fabs(w0 * j0 + w1 * j1 + w2 * j2) + c * sqrt(j0 * j0 + j1 * j1 + j2 * j2);
    }
    lam *= (double)rinvj_r;
  } else {
    lam = (fabs(w0) + c) * (double)scale[0];
    if (DIM > 1) lam += (fabs(w1) + c) * (double)scale[DIM > 1 ? 1 : 0];
    if (DIM > 2) lam += (fabs(w2) + c) * (double)scale[DIM > 2 ? 2 : 0];
  }
  return lam;
}

// primitive state from (rho, v_1..v_d, p, log rho, log beta) stored as dim+4 values
template <int DIM, typename Real>
__device__ __forceinline__ Prim<Real> unpack_prim(const Real* f) {
  Prim<Real> P;
  P.rho = f[0];
  P.v0 = f[1];
  P.v1 = DIM > 1 ? f[DIM > 1 ? 2 : 1] : Real(0);
  P.v2 = DIM > 2 ? f[DIM > 2 ? 3 : 1] : Real(0);
  P.p = f[DIM + 1];
  P.lr = f[DIM + 2];
  P.b = P.rho * dev_rcp(P.p);
  P.lb = f[DIM + 3];
  return P;
}

// The i<k pairs of one line in direction DIR: the lane loads the line's
// primitive variables (LDS) and averaged contravariant vectors, evaluates each
// two-point flux once and scatters D~_ik F to node i and D~_ki F to node k in
// registers (skew-symmetric D~ with zero diagonal, Sec. 2.2; all indices are
// compile-time constants).
//
// Gauss collocation (NODES_GAUSS, affine): the line is the volume block of
// the hybridised operator and its two face points carry the entropy-projected
// states fo[0] (end at -1) and fo[1] (end at +1); fn holds the neighbours'
// states at the same points.  Besides the volume pairs (T in the D~ slot) the
// lane evaluates f(u_k, u~_f) for every node k and both ends, adds
// M^-1 R^T B (f(u_k, u~_f) - sum_j R_fj f(u_j, u~_f) + f*_f), i.e. the
// face-point rows of 2 Q_h lifted by R^T and the surface term of Sec. 6.
template <int DIR, int DIM, int N, int VF, int MESH, typename Real, int NODES = NODES_LGL>
__device__ __forceinline__ void line_fluxes(const Real (*sp)[Pow<N, DIM>::value], const Real (&nrm)[N][3], int base,
                                            const StageOps<Real>& ops, const Real* s_dt, Real scale,
                                            Real (&A)[N][DIM + 2], const Real (*fo)[DIM + 4] = nullptr,
                                            const Real (*fn)[DIM + 4] = nullptr, int surf = 0) {
  // contraction off: the affine scaling below must not fuse with the caller's
  // sum over directions (the layouts sum them in different places)
#pragma clang fp contract(off)
  constexpr int NV = DIM + 2;
  constexpr int NP = PrimCount<VF, DIM>::value;
  constexpr int stride = Pow<N, DIR>::value;
  Prim<Real> P[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int q = base + k * stride;
    P[k].rho = sp[0][q];
    P[k].v0 = sp[1][q];
    P[k].v1 = DIM > 1 ? sp[DIM > 1 ? 2 : 0][q] : Real(0);
    P[k].v2 = DIM > 2 ? sp[DIM > 2 ? 3 : 0][q] : Real(0);
    P[k].p = sp[DIM + 1][q];
    P[k].lr = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 2 : 0][q] : Real(0);
    P[k].b = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 3 : 0][q] : Real(0);
    P[k].lb = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 4 : 0][q] : Real(0);
  }
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int v = 0; v < NV; ++v) A[k][v] = Real(0);
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int k = i + 1; k < N; ++k) {
      Real F[NV];
      if (MESH == MESH_CURVED) {
        // nrm holds half the contravariant vectors: the sum is the pair average
        volume_flux<VF, DIM>(P[i], P[k], nrm[i][0] + nrm[k][0], nrm[i][1] + nrm[k][1], nrm[i][2] + nrm[k][2],
                             ops.inv_gm1, F);
      } else {
        volume_flux<VF, DIM>(P[i], P[k], DIR == 0 ? Real(1) : Real(0), DIR == 1 ? Real(1) : Real(0),
                             DIR == 2 ? Real(1) : Real(0), ops.inv_gm1, F);
      }
      const Real dik = DtInLds<N, Real>::value ? s_dt[i * N + k] : ops.Dt[i * N + k];
      const Real dki = DtInLds<N, Real>::value ? s_dt[k * N + i] : ops.Dt[k * N + i];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        A[i][v] = mad(dik, F[v], A[i][v]);
        A[k][v] = mad(dki, F[v], A[k][v]);
      }
    }
  }
  if constexpr (NODES == NODES_GAUSS) {
    const Real nx = DIR == 0 ? Real(1) : Real(0), ny = DIR == 1 ? Real(1) : Real(0), nz = DIR == 2 ? Real(1) : Real(0);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const Prim<Real> Pf = unpack_prim<DIM>(fo[s]), Pn = unpack_prim<DIM>(fn[s]);
      Real Fs[NV], G[NV];
      // f* oriented along +DIR: at the -1 end the neighbour is on the left
      if (s) surface_flux_prim<DIM>(surf, Pf, Pn, nx, ny, nz, ops.gamma, ops.inv_gm1, Fs);
      else surface_flux_prim<DIM>(surf, Pn, Pf, nx, ny, nz, ops.gamma, ops.inv_gm1, Fs);
#pragma unroll
      for (int v = 0; v < NV; ++v) G[v] = Real(0);
#pragma unroll
      for (int k = 0; k < N; ++k) {
        Real F[NV];
        volume_flux<VF, DIM>(P[k], Pf, nx, ny, nz, ops.inv_gm1, F);
        const Real c = s ? ops.cR[k] : ops.cL[k], r = s ? ops.rR[k] : ops.rL[k];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          A[k][v] = mad(c, F[v], A[k][v]);
          G[v] = mad(r, F[v], G[v]);
        }
      }
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const Real c = s ? ops.cR[k] : ops.cL[k];
#pragma unroll
        for (int v = 0; v < NV; ++v) A[k][v] = mad(c, Fs[v] - G[v], A[k][v]);
      }
    }
  }
  if (MESH == MESH_AFFINE) {
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
      for (int v = 0; v < NV; ++v) A[k][v] *= scale;
  }
}

// The partners of one node along direction DIR (node layout): the lane reads
// each partner's primitive variables and halved contravariant vector from
// LDS, evaluates f(u_i, u_k) (bitwise the pair's flux, see volume_flux) and
// accumulates D~_ik F in increasing k, the order in which the line layout's
// pair loop reaches node i.  sn holds the halved contravariant vectors of
// direction DIR of the element ([DIM][NN]); no is the node's own.  s_dts is
// D~ without its diagonal, row id holding D~_ik for k = j + (j >= id),
// j = 0..N-2: the sweep's j-th coefficient is one load at a lane-constant
// base, and the partner's node index one select and one add.
template <int DIR, int DIM, int N, int VF, int MESH, typename Real, int RL>
__device__ __forceinline__ void node_fluxes(const Real (*sp)[RL], const Real (*sn)[RL],
                                            const Prim<Real>& Po, const Real (&no)[3], int i, int id,
                                            const Real* s_dts, Real scale, Real inv_gm1, Real (&A)[DIM + 2]) {
#pragma clang fp contract(off)  // as in line_fluxes
  constexpr int NV = DIM + 2;
  constexpr int NP = PrimCount<VF, DIM>::value;
  constexpr int stride = Pow<N, DIR>::value;
  const int q_lo = i - id * stride;  // partner k = j for j < id
  const int q_hi = q_lo + stride;    // partner k = j + 1 from j = id on
  const Real* drow = s_dts + id * (N - 1);
#pragma unroll
  for (int v = 0; v < NV; ++v) A[v] = Real(0);
  // a rolled loop: unrolled, the partners' loads are hoisted ahead of the
  // fluxes and the registers spill
#pragma unroll 1
  for (int j = 0; j < N - 1; ++j) {
    const int q = (j >= id ? q_hi : q_lo) + j * stride;
    Prim<Real> Pk;
    Pk.rho = sp[0][q];
    Pk.v0 = sp[1][q];
    Pk.v1 = DIM > 1 ? sp[DIM > 1 ? 2 : 0][q] : Real(0);
    Pk.v2 = DIM > 2 ? sp[DIM > 2 ? 3 : 0][q] : Real(0);
    Pk.p = sp[DIM + 1][q];
    Pk.lr = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 2 : 0][q] : Real(0);
    Pk.b = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 3 : 0][q] : Real(0);
    Pk.lb = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 4 : 0][q] : Real(0);
    Real F[NV];
    if (MESH == MESH_CURVED) {
      volume_flux<VF, DIM, Real, sizeof(Real) == 8>(Po, Pk, no[0] + sn[0][q], DIM > 1 ? no[1] + sn[DIM > 1 ? 1 : 0][q] : Real(0),
                           DIM > 2 ? no[2] + sn[DIM > 2 ? 2 : 0][q] : Real(0), inv_gm1, F);
    } else {
      volume_flux<VF, DIM, Real, sizeof(Real) == 8>(Po, Pk, DIR == 0 ? Real(1) : Real(0), DIR == 1 ? Real(1) : Real(0),
                           DIR == 2 ? Real(1) : Real(0), inv_gm1, F);
    }
    const Real dik = drow[j];
#pragma unroll
    for (int v = 0; v < NV; ++v) A[v] = mad(dik, F[v], A[v]);
  }
  if (MESH == MESH_AFFINE) {
#pragma unroll
    for (int v = 0; v < NV; ++v) A[v] *= scale;
  }
}

// LDS slot of node q when every 64-node block of a row is followed by PAD
// unused entries (PAD = 0: the node index itself)
template <int PAD>
__device__ __forceinline__ int lds_node(int q) { return PAD ? q + (q >> 6) * PAD : q; }

// Cross-lane copy of one value within a wave: the lane receives `x` of wave
// lane `src` (ds_bpermute, which reads the VGPRs of the other lanes through
// the LDS crossbar without using LDS memory; every lane of the wave active).
__device__ __forceinline__ float lane_pull(int src, float x) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(x)));
}
__device__ __forceinline__ double lane_pull(int src, double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// The pairs of one line in direction DIR, each evaluated once (pair layout).
// The N lanes of a line lie in one wave, lane stride LS apart; the lane at
// line position a owns node i (node stride N^DIR along the line).  Round d =
// 1 .. ceil(N/2)-1 pairs every lane with the position b = a+d (mod N): the
// lane evaluates f(u_a, u_b) once, adds D~_ab F to its own row, and takes
// from the lane at c = a-d (mod N), which has just evaluated the pair (c, a),
// its F for D~_ac F.  For even N the last round d = N/2 pairs a with a+N/2
// from both ends (no exchange; the same cost as leaving half the lanes
// idle).  Each pair is thus evaluated once apart from the N/2 pairs of the
// last round: N/2 evaluations per lane and direction instead of N-1.  The
// flux is bitwise symmetric (volume_flux) and the averaged normal a sum of
// the two halves, so both lanes of a pair see the same F.  s_rot holds
// D~_{a,a+d} at [d-1][a] and s_rot + (N/2) N holds D~_{a,a-d} at [d-1][a].
// The sum runs in the order of the rounds (own, then received), not in
// increasing k as in the other layouts: the same values up to rounding.
// Rows of sp and sn have RL entries, node q at lds_node<PAD>(q).
template <int DIR, int DIM, int N, int LS, int VF, int MESH, typename Real, int RL, int PAD>
__device__ __forceinline__ void pair_fluxes(const Real (*sp)[RL], const Real (*sn)[RL], const Prim<Real>& Po,
                                            const Real (&no)[3], int i, int a, int lane, const Real* s_rot, Real scale,
                                            Real inv_gm1, Real (&A)[DIM + 2]) {
#pragma clang fp contract(off)  // as in line_fluxes
  constexpr int NV = DIM + 2;
  constexpr int NP = PrimCount<VF, DIM>::value;
  constexpr int stride = Pow<N, DIR>::value;
  constexpr int H = N / 2;                 // rounds with exchange: 1 .. (N-1)/2; even N adds round H
  constexpr bool POW2 = (N & (N - 1)) == 0;
  // LDS distance of consecutive nodes of the line: the padded rows (N = 8)
  // add PAD per 64-node z-plane, which only the z-lines cross
  static_assert(PAD == 0 || N == 8, "padded LDS rows: 64-node z-planes");
  constexpr int LSTEP = (PAD && DIR == 2) ? stride + PAD : stride;
  const int node0 = i - a * stride;        // node at line position 0
  const int lbase = lds_node<PAD>(node0);  // its LDS slot
  const int lane0 = lane - a * LS;         // its lane
  const Real* rot_own = s_rot + a;         // D~_{a,a+d} at (d-1) N
  const Real* rot_in = s_rot + H * N + a;  // D~_{a,a-d} at (d-1) N
#pragma unroll
  for (int v = 0; v < NV; ++v) A[v] = Real(0);
#pragma unroll 1
  for (int d = 1; d <= H; ++d) {
    const int b = POW2 ? ((a + d) & (N - 1)) : (a + d < N ? a + d : a + d - N);
    const int q = lbase + b * LSTEP;
    Prim<Real> Pk;
    Pk.rho = sp[0][q];
    Pk.v0 = sp[1][q];
    Pk.v1 = DIM > 1 ? sp[DIM > 1 ? 2 : 0][q] : Real(0);
    Pk.v2 = DIM > 2 ? sp[DIM > 2 ? 3 : 0][q] : Real(0);
    Pk.p = sp[DIM + 1][q];
    Pk.lr = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 2 : 0][q] : Real(0);
    Pk.b = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 3 : 0][q] : Real(0);
    Pk.lb = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 4 : 0][q] : Real(0);
    Real F[NV];
    if (MESH == MESH_CURVED) {
      volume_flux<VF, DIM, Real, sizeof(Real) == 8>(Po, Pk, no[0] + sn[0][q], DIM > 1 ? no[1] + sn[DIM > 1 ? 1 : 0][q] : Real(0),
                           DIM > 2 ? no[2] + sn[DIM > 2 ? 2 : 0][q] : Real(0), inv_gm1, F);
    } else {
      volume_flux<VF, DIM, Real, sizeof(Real) == 8>(Po, Pk, DIR == 0 ? Real(1) : Real(0), DIR == 1 ? Real(1) : Real(0),
                           DIR == 2 ? Real(1) : Real(0), inv_gm1, F);
    }
    const Real dab = rot_own[(d - 1) * N];
#pragma unroll
    for (int v = 0; v < NV; ++v) A[v] = mad(dab, F[v], A[v]);
    if (2 * d < N) {  // uniform across the wave
      const int src = lane0 + (POW2 ? ((a - d) & (N - 1)) : (a >= d ? a - d : a - d + N)) * LS;
      const Real dac = rot_in[(d - 1) * N];
#pragma unroll
      for (int v = 0; v < NV; ++v) A[v] = mad(dac, lane_pull(src, F[v]), A[v]);
    }
  }
  if (MESH == MESH_AFFINE) {
#pragma unroll
    for (int v = 0; v < NV; ++v) A[v] *= scale;
  }
}

// Stage kernels built with the once-per-face reading of f* (a runtime
// branch): 3D tiles whose register allocation it leaves unchanged, i.e. the
// node and pair layouts and the line layout up to N = 5 (in the line tiles
// above, and in 2D, it adds spills).
template <int DIM, int N, int LAY>
struct FacesOnce { static constexpr bool value = DIM == 3 && (LAY != LAY_LINES || N <= 5); };

// Waves per SIMD the register allocation of a tile must allow: the tile's
// default, except for the FP64 node tiles up to N = 5, whose prologue (two or
// three face nodes per lane) spills at four waves (three measured 3% faster
// at p = 4).
template <int DIM, int N, int MESH, typename Real, int EPB_, int LAY = LAY_LINES>
struct StageWaves {
  static constexpr int value = (LAY != LAY_LINES && sizeof(Real) == 8 && N <= 5) ? 3 : Tile<DIM, N, EPB_, LAY>::WPE;
};

// PRIO, the one-generation form: the prologue and the surface fluxes run at
// raised wave priority, and the RK4 stage results are stored with the
// nontemporal hint.  The host launches this form only where all the
// launch's workgroups are resident at once (one generation, more than one
// workgroup per compute unit): the workgroups dispatched last then set up
// their tiles ahead of the volume work of those dispatched first, which
// shortens the launch's tail, and the results stream out without displacing
// the inputs from the caches.  With workgroups queued behind the resident
// ones, or one per compute unit, the same priority measured slower and the
// hint gained nothing or lost.
template <int DIM, int N, int VF, int MESH, typename Real, int EPB_, int NODES = NODES_LGL, int LAY = LAY_LINES,
          bool PRIO = false>
__global__ void __launch_bounds__((Tile<DIM, N, EPB_, LAY>::THREADS))
__attribute__((amdgpu_waves_per_eu(StageWaves<DIM, N, MESH, Real, EPB_, LAY>::value))) stage_kernel(StageArgs<Real> a) {
  static_assert(NODES == NODES_LGL || MESH == MESH_AFFINE, "Gauss collocation is built for affine meshes");
  static_assert(LAY == LAY_LINES || (NODES == NODES_LGL && DIM == 3), "node layout: 3D LGL");
  static_assert(!Tile<DIM, N, EPB_, LAY>::PLANE || EPB_ == 1, "plane layouts: one element per block");
  using T = Tile<DIM, N, EPB_, LAY>;
  constexpr bool NODEL = LAY != LAY_LINES;  // one lane per node (node and pair layouts)
  constexpr bool PAIRS = LAY == LAY_PAIRS || LAY == LAY_PLANES;
  constexpr bool PG = PAIRS && !T::PLANE;   // pair layout with lines packed per wave (N < 7)
  // plane layout with idle lanes (N = 7: lane l of wave w holds node l + N^2 w);
  // at N = 8 the plane layout's node of lane slot q is q itself
  constexpr bool PMAP = T::PLANE && N * N < 64;
  constexpr bool CNODE = NODEL && MESH == MESH_CURVED;
  constexpr bool FONCE = FacesOnce<DIM, N, LAY>::value && NODES == NODES_LGL;  // may read f* (a.fstar)
  constexpr int NN = T::NN, NF = T::NF, L = T::L, EPB = T::EPB, NV = T::NV, NFACE = T::NFACE;
  constexpr int THREADS = T::THREADS, NPT = T::NPT, FPT = T::FPT, LANES_DIR = T::LANES_DIR;
  constexpr int NP = PrimCount<VF, DIM>::value;
  constexpr int NM = DIM * DIM + 1;
  // node-indexed LDS rows; the pair layout at N = 8 pads each 64-node z-plane by
  // LPAD entries, so that its z-lines (one node per plane, read by 8 lanes
  // at once) fall on different banks
  constexpr int LPAD = PAIRS && N == 8 ? 8 : 0;
  constexpr int NNL = NN + (NN / 64) * LPAD;
  __shared__ Real s_prim[EPB][NP][NNL];     // primitive variables (and logs)
  // volume term, summed over directions in order (line layout): reuses the
  // primitives' LDS, which every lane has read into registers by then
  static_assert(NV <= NP, "volume sums fit in the primitives' LDS");
  Real(*s_acc)[NV][NNL] = reinterpret_cast<Real(*)[NV][NNL]>(&s_prim[0][0][0]);
  __shared__ Real s_face[EPB][NV][NFACE];  // surface fluxes of the element's faces
  __shared__ int s_nbr[EPB][2 * DIM];      // neighbour across face (2 dir + side), side 1 = +
  __shared__ Real s_dt[DtInLds<N, Real>::value ? N * N : 1];  // D~ when it stays out of scalar registers
  __shared__ Real s_dts[NODEL ? (PAIRS ? N * N : N * (N - 1)) : 1];  // node layout: D~ rows without the diagonal;
                                                   // pair layout: D~_{a,a+d}, then D~_{a,a-d} (pair_fluxes)
  // node layout, curved: halved contravariant vectors of two directions
  // (directions 0 and 1, then 2 in the first buffer)
  __shared__ Real s_nrm[CNODE ? EPB : 1][2][DIM][CNODE ? NNL : 1];
  // pair layout with packed lines: the volume sums of the nodes, merged
  // direction by direction (the lanes of a direction are not the nodes' own)
  __shared__ Real s_vol[PG ? EPB : 1][NV][PG ? NN : 1];

  const int tid = threadIdx.x;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int pi = a.tile_prob ? a.tile_prob[tile] : 0;
  const ProbDesc<Real>& P = a.probs[pi];
  const auto uin = as_global((const Real*)P.buf[a.in_idx]);
  const auto out = as_global(a.out_ext ? a.out_ext : P.buf[a.out_idx]);
  const auto racc_buf = as_global(P.buf[3]);
  const auto u0 = as_global((const Real*)P.buf[0]);
  const auto metric = as_global(P.metric);
  const auto nface = as_global(P.nface);
  const int E = P.E, n0 = P.n0, n1 = P.n1, n2 = P.n2;
  const int e0 = (tile - P.tile0) * EPB;
  const bool cfl_mode = a.cfl > 0.0;
  const auto lam_in = as_global((const unsigned long long*)P.lam + a.par * kLamSlots);
  unsigned long long* lam_next = P.lam + (1 - a.par) * kLamSlots;
  const bool first_stage = a.mode == MODE_RK_FIRST || a.mode == MODE_LS_FIRST;
  const bool last_stage = a.mode == MODE_RK_LAST || a.mode == MODE_LS_LAST;
  const bool lam_out = last_stage && cfl_mode && a.lam_update;
  const Real gm1 = a.ops.gamma - Real(1);
  if (tid < EPB) {
    const int e = e0 + tid;
    const int ex = e % n0, ey = (e / n0) % n1, ez = e / (n0 * n1);
    const int exm = ex == 0 ? n0 - 1 : ex - 1, exp_ = ex == n0 - 1 ? 0 : ex + 1;
    s_nbr[tid][0] = exm + n0 * (ey + n1 * ez);
    s_nbr[tid][1] = exp_ + n0 * (ey + n1 * ez);
    if (DIM > 1) {
      const int eym = ey == 0 ? n1 - 1 : ey - 1, eyp = ey == n1 - 1 ? 0 : ey + 1;
      s_nbr[tid][DIM > 1 ? 2 : 0] = ex + n0 * (eym + n1 * ez);
      s_nbr[tid][DIM > 1 ? 3 : 0] = ex + n0 * (eyp + n1 * ez);
    }
    if (DIM > 2) {
      const int ezm = ez == 0 ? n2 - 1 : ez - 1, ezp = ez == n2 - 1 ? 0 : ez + 1;
      s_nbr[tid][DIM > 2 ? 4 : 0] = ex + n0 * (ey + n1 * ezm);
      s_nbr[tid][DIM > 2 ? 5 : 0] = ex + n0 * (ey + n1 * ezp);
    }
  }

  // the lane's line: direction (wave-uniform), element and line index
  const int ldir = tid / LANES_DIR;
  const int lrem = tid - ldir * LANES_DIR;
  const int lel = lrem / L;
  const int lline = lrem - lel * L;
  const bool lactive = lel < EPB && e0 + lel < E;
  const int stride = ldir == 0 ? 1 : (ldir == 1 ? N : N * N);
  const int lbase = (lline % stride) + (lline / stride) * stride * N;

  // ---- every global load the block needs before its stores is issued here:
  // own state and 1/J per node, the line's contravariant vectors, the face
  // traces and normals.  Indices of lanes without work are clamped to
  // element 0 so that every address stays in bounds.
  Real uo[NPT][NV], rinvj[NPT];
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int q = tid + r * THREADS;
    int el = q / NN, i = q - el * NN;
    bool ok = q < EPB * NN && e0 + el < E;
    if constexpr (PMAP) {
      el = 0;
      ok = plane_node<N>(q, i) && e0 < E;
    }
    const size_t o = ok ? (size_t)(e0 + el) * (NV * NN) + i : 0;
#pragma unroll
    for (int v = 0; v < NV; ++v) uo[r][v] = uin[o + (size_t)v * NN];
    rinvj[r] = MESH == MESH_CURVED ? metric[(ok ? (size_t)(e0 + el) * (NM * NN) + i : 0) + (size_t)(NM - 1) * NN]
                                   : Real(1);
  }
  Real nrm[N][3];
  // node layout, curved: the node's halved contravariant vectors of
  // directions 0 and 1 (direction 2 is loaded after their sweeps)
  Real hm[2][DIM];
  int pnode = 0;
  const bool pok = PMAP && plane_node<N>(tid, pnode) && e0 < E;  // plane layout: the lane's node
  const auto me_node =
      metric + (PMAP ? (CNODE && pok ? (size_t)e0 * (NM * NN) + pnode : 0)
                         : ((CNODE && tid < EPB * NN && e0 + tid / NN < E)
                                ? (size_t)(e0 + tid / NN) * (NM * NN) + (tid - (tid / NN) * NN)
                                : 0));
  if constexpr (CNODE) {
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int m = 0; m < DIM; ++m) hm[n][m] = Real(0.5) * me_node[(n * DIM + m) * NN];
  }
  if (MESH == MESH_CURVED && !NODEL) {
    const auto me = metric + (size_t)(lactive ? e0 + lel : 0) * (NM * NN);
#pragma unroll
    for (int k = 0; k < N; ++k)
#pragma unroll
      for (int m = 0; m < 3; ++m) nrm[k][m] = m < DIM ? Real(0.5) * me[(ldir * DIM + m) * NN + lbase + k * stride] : Real(0);
  }
  if (DtInLds<N, Real>::value)
    for (int t = tid; t < N * N; t += THREADS) s_dt[t] = a.ops.Dt[t];
  if (NODEL && !PAIRS)
    for (int t = tid; t < N * (N - 1); t += THREADS) {
      const int r = t / (N - 1), j = t - r * (N - 1);
      s_dts[t] = a.ops.Dt[r * N + j + (j >= r ? 1 : 0)];
    }
  if (PAIRS)
    for (int t = tid; t < 2 * (N / 2) * N; t += THREADS) {
      const int hh = t / ((N / 2) * N), rr = t - hh * (N / 2) * N;
      const int d = rr / N + 1, ap = rr - (d - 1) * N;
      const int k = hh ? (ap - d + N) % N : (ap + d) % N;
      s_dts[t] = a.ops.Dt[ap * N + k];
    }
  __syncthreads();  // s_nbr, s_dt
  Real tL[FPT][NV], tR[FPT][NV], tn[FPT][3];
  constexpr int NPF = DIM + 4;
  Real fo[2][NPF], fnb[2][NPF];  // Gauss: own / neighbours' projected states at the line's ends
  if constexpr (NODES == NODES_GAUSS) {
    const auto fb = as_global((const Real*)P.faceb);
    const int e = lactive ? e0 + lel : 0;
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const int fc = 2 * ldir + sd;
      const int en = lactive ? s_nbr[lel][fc] : 0;
#pragma unroll
      for (int c = 0; c < NPF; ++c) {
        fo[sd][c] = fb[(((size_t)e * (2 * DIM) + fc) * NPF + c) * NF + lline];
        fnb[sd][c] = fb[(((size_t)en * (2 * DIM) + (fc ^ 1)) * NPF + c) * NF + lline];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < FPT && NODES == NODES_LGL; ++r) {
    const int t = tid + r * THREADS;
    const int el = t / NFACE, rr = t - el * NFACE;
    const bool ok = t < EPB * NFACE && e0 + el < E;
    const int fc = rr / NF, f = rr - fc * NF, dir = fc >> 1, side = fc & 1;
    const int e = ok ? e0 + el : 0;
    const int en = ok ? s_nbr[el][fc] : 0;
    const int eL = side ? e : en, eR = side ? en : e;
    if (FONCE && a.fstar) {  // the face's flux, from the + face of its left element
      const auto fs = as_global((const Real*)a.fstar) + ((size_t)eL * DIM + dir) * (NV * NF) + f;
#pragma unroll
      for (int v = 0; v < NV; ++v) tL[r][v] = fs[v * NF];
      continue;
    }
    const int qL = face_node<N>(dir, f, N - 1), qR = face_node<N>(dir, f, 0);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      tL[r][v] = uin[(size_t)eL * (NV * NN) + v * NN + qL];
      tR[r][v] = uin[(size_t)eR * (NV * NN) + v * NN + qR];
    }
    if (MESH == MESH_CURVED) {
      const auto nf = nface + ((size_t)dir * E + eL) * (DIM * NF) + f;
      tn[r][0] = nf[0];
      tn[r][1] = DIM > 1 ? nf[NF] : Real(0);
      tn[r][2] = DIM > 2 ? nf[2 * NF] : Real(0);
    } else {
      tn[r][0] = dir == 0 ? Real(1) : Real(0);
      tn[r][1] = dir == 1 ? Real(1) : Real(0);
      tn[r][2] = dir == 2 ? Real(1) : Real(0);
    }
  }

  if constexpr (PRIO) __builtin_amdgcn_s_setprio(2);
  // ---- prologue: primitive variables and logs once per node into LDS
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int q = tid + r * THREADS;
    int el = q / NN, i = q - el * NN;
    if constexpr (PMAP) {
      el = 0;
      if (!(plane_node<N>(q, i) && e0 < E)) continue;
    } else if (!(q < EPB * NN && e0 + el < E)) {
      continue;
    }
    const Real rho = uo[r][0];
    const Real inv_rho = dev_rcp(rho);
    const Real m0 = uo[r][1];
    const Real m1 = DIM > 1 ? uo[r][DIM > 1 ? 2 : 1] : Real(0);
    const Real m2 = DIM > 2 ? uo[r][DIM > 2 ? 3 : 1] : Real(0);
    const Real E_ = uo[r][DIM + 1];
    const Real v0 = m0 * inv_rho, v1 = m1 * inv_rho, v2 = m2 * inv_rho;
    const Real p = gm1 * (E_ - Real(0.5) * (m0 * v0 + m1 * v1 + m2 * v2));
    if (!(rho > Real(0)) || !(p > Real(0)) || !isfinite(E_) || !isfinite(m0 + m1 + m2)) *(volatile int*)P.flag = 1;
    const int li = lds_node<LPAD>(i);
    s_prim[el][0][li] = rho;
    s_prim[el][1][li] = v0;
    if (DIM > 1) s_prim[el][DIM > 1 ? 2 : 0][li] = v1;
    if (DIM > 2) s_prim[el][DIM > 2 ? 3 : 0][li] = v2;
    s_prim[el][DIM + 1][li] = p;
    if (NP > DIM + 2) {
      const Real beta = rho * dev_rcp(p);
      s_prim[el][(NP > DIM + 2) ? DIM + 2 : 0][li] = dev_log(rho);
      s_prim[el][(NP > DIM + 2) ? DIM + 3 : 0][li] = beta;
      s_prim[el][(NP > DIM + 2) ? DIM + 4 : 0][li] = dev_log(beta);
    }
    if constexpr (CNODE) {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int m = 0; m < DIM; ++m) s_nrm[el][b][m][li] = hm[b][m];
    }
  }

  // ---- surface fluxes of the element's faces (LGL; Gauss lines handle their own ends)
#pragma unroll
  for (int r = 0; r < FPT && NODES == NODES_LGL; ++r) {
    const int t = tid + r * THREADS;
    const int el = t / NFACE, rr = t - el * NFACE;
    if (!(t < EPB * NFACE && e0 + el < E)) continue;
    Real F[NV];
    if (FONCE && a.fstar) {
#pragma unroll
      for (int v = 0; v < NV; ++v) F[v] = tL[r][v];
    } else {
      surface_flux<DIM>(a.surf, tL[r], tR[r], tn[r][0], tn[r][1], tn[r][2], a.ops.gamma, a.ops.inv_gm1, F);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) s_face[el][v][rr] = F[v];
  }
  __syncthreads();
  if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);

  // ---- volume term, node layout: each lane sweeps the partners of its node,
  // direction by direction, and sums the directions in the line layout's order
  Real Sn[NV];
  if constexpr (PG) {
    // pair layout with packed lines: lane x of a wave takes position x % N of line
    // x / N (floor(64/N) whole lines per wave, element-major); per direction
    // the lines' pairs are evaluated once (pair_fluxes, lanes of a line
    // consecutive) and the sums are merged per node in LDS: direction 0
    // writes, 1 adds, 2 adds, the order of the other layouts
    const int lane = tid & 63, slot = lane / N, pos = lane - slot * N;
    const int line = (tid >> 6) * T::LPW + slot;
    const bool lok = slot < T::LPW && line < EPB * N * N && e0 + line / (N * N) < E;
    const int lel = lok ? line / (N * N) : 0, lix = lok ? line - lel * N * N : 0;  // idle lanes: line 0
    const int c1 = lix % N, c2 = lix / N;
    const Real(*sp)[NNL] = s_prim[lel];
    const Real(*sn0)[NNL] = reinterpret_cast<const Real(*)[NNL]>(&s_nrm[CNODE ? lel : 0][0][0][0]);
    const Real(*sn1)[NNL] = reinterpret_cast<const Real(*)[NNL]>(&s_nrm[CNODE ? lel : 0][1][0][0]);
    Real Ad[NV];
    auto sweep = [&](auto dir_c, const Real(*sn)[NNL], int q, Real scale) {
      constexpr int DIR = decltype(dir_c)::value;
      Prim<Real> Pq;
      Pq.rho = sp[0][q];
      Pq.v0 = sp[1][q];
      Pq.v1 = sp[2][q];
      Pq.v2 = sp[3][q];
      Pq.p = sp[4][q];
      Pq.lr = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 2 : 0][q] : Real(0);
      Pq.b = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 3 : 0][q] : Real(0);
      Pq.lb = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 4 : 0][q] : Real(0);
      Real nq[3] = {Real(0), Real(0), Real(0)};
      if constexpr (CNODE) { nq[0] = sn[0][q]; nq[1] = sn[1][q]; nq[2] = sn[2][q]; }
      pair_fluxes<DIR, DIM, N, 1, VF, MESH, Real, NNL, 0>(sp, sn, Pq, nq, q, pos, lane, s_dts, scale, a.ops.inv_gm1,
                                                           Ad);
    };
    const int q0 = pos + N * c1 + N * N * c2, q1 = c1 + N * pos + N * N * c2, q2 = c1 + N * c2 + N * N * pos;
    sweep(std::integral_constant<int, 0>(), sn0, q0, P.scale[0]);
    if (lok)
#pragma unroll
      for (int v = 0; v < NV; ++v) s_vol[lel][v][q0] = Ad[v];
    sweep(std::integral_constant<int, 1>(), sn1, q1, P.scale[1]);
    __syncthreads();  // direction 0's sums written; its vectors (first buffer) read
    if (lok)
#pragma unroll
      for (int v = 0; v < NV; ++v) s_vol[lel][v][q1] += Ad[v];
    if constexpr (CNODE) {
      // direction 2 replaces direction 0 in the first buffer (node owners)
      if (tid < EPB * NN && e0 + tid / NN < E) {
        const int el = tid / NN, i = tid - el * NN;
#pragma unroll
        for (int m = 0; m < DIM; ++m) s_nrm[el][0][m][i] = Real(0.5) * me_node[(2 * DIM + m) * NN];
      }
    }
    __syncthreads();
    sweep(std::integral_constant<int, 2>(), sn0, q2, P.scale[2]);
    if (lok)
#pragma unroll
      for (int v = 0; v < NV; ++v) s_vol[lel][v][q2] += Ad[v];
    __syncthreads();
    if (tid < EPB * NN) {
      const int el = tid / NN, i = tid - el * NN;
#pragma unroll
      for (int v = 0; v < NV; ++v) Sn[v] = s_vol[el][v][i];
    }
  }
  if constexpr (NODEL && !PG) {
    const bool ok = PMAP ? pok : (tid < EPB * NN && e0 + tid / NN < E);
    const int el = (ok && !PMAP) ? tid / NN : 0;
    const int i = ok ? (PMAP ? pnode : tid - el * NN) : 0;  // idle lanes repeat node 0
    const Real(*sp)[NNL] = s_prim[el];
    const int ix = i % N, iy = (i / N) % N, iz = i / (N * N);
    const int li = lds_node<LPAD>(i);
    Prim<Real> Po;
    Po.rho = sp[0][li];
    Po.v0 = sp[1][li];
    Po.v1 = sp[2][li];
    Po.v2 = sp[3][li];
    Po.p = sp[4][li];
    Po.lr = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 2 : 0][li] : Real(0);
    Po.b = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 3 : 0][li] : Real(0);
    Po.lb = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 4 : 0][li] : Real(0);
    Real no[3] = {Real(0), Real(0), Real(0)};
    Real Ad[NV];
    // the two direction buffers (never read on affine meshes); the node's own
    // vectors are read back from them rather than held in registers
    const Real(*sn0)[NNL] = reinterpret_cast<const Real(*)[NNL]>(&s_nrm[CNODE ? el : 0][0][0][0]);
    const Real(*sn1)[NNL] = reinterpret_cast<const Real(*)[NNL]>(&s_nrm[CNODE ? el : 0][1][0][0]);
    if constexpr (CNODE) { no[0] = sn0[0][li]; no[1] = sn0[1][li]; no[2] = sn0[2][li]; }
    const int lane = tid & 63;
    // pair layout: a wave is one z-plane of the element (lanes x + N y), so
    // the lines of directions 0 and 1 lie in one wave (lane strides 1 and N)
    if constexpr (PAIRS)
      pair_fluxes<0, DIM, N, 1, VF, MESH, Real, NNL, LPAD>(sp, sn0, Po, no, i, ix, lane, s_dts, P.scale[0],
                                                           a.ops.inv_gm1, Ad);
    else
      node_fluxes<0, DIM, N, VF, MESH, Real>(sp, sn0, Po, no, i, ix, s_dts, P.scale[0], a.ops.inv_gm1, Ad);
#pragma unroll
    for (int v = 0; v < NV; ++v) Sn[v] = Ad[v];
    if constexpr (CNODE) { no[0] = sn1[0][li]; no[1] = sn1[1][li]; no[2] = sn1[2][li]; }
    if constexpr (PAIRS)
      pair_fluxes<1, DIM, N, N, VF, MESH, Real, NNL, LPAD>(sp, sn1, Po, no, i, iy, lane, s_dts, P.scale[1],
                                                           a.ops.inv_gm1, Ad);
    else
      node_fluxes<1, DIM, N, VF, MESH, Real>(sp, sn1, Po, no, i, iy, s_dts, P.scale[1], a.ops.inv_gm1, Ad);
#pragma unroll
    for (int v = 0; v < NV; ++v) Sn[v] += Ad[v];
    if constexpr (CNODE) {
      // direction 2 replaces direction 0 in the first buffer
#pragma unroll
      for (int m = 0; m < DIM; ++m) no[m] = Real(0.5) * me_node[(2 * DIM + m) * NN];
      __syncthreads();
      if (ok)
#pragma unroll
        for (int m = 0; m < DIM; ++m) s_nrm[el][0][m][li] = no[m];
      __syncthreads();
    }
    if constexpr (PAIRS) {
      // direction 2: the lanes are re-mapped so that a wave holds one
      // y-plane (lane x + N z of wave y takes node (x, y, z)), which puts
      // each z-line in one wave at lane stride N; the sums go back to the
      // nodes' own lanes through the primitives' LDS.  Lanes N^2 .. 63 (N = 7)
      // take node (x, y, 0) and store nothing.
      const bool ok2 = lane < N * N;
      const int z2 = ok2 ? lane / N : 0;
      const int i2 = (lane % N) + N * (tid / 64) + N * N * z2;
      const int l2 = lds_node<LPAD>(i2);
      Prim<Real> P2;
      P2.rho = sp[0][l2];
      P2.v0 = sp[1][l2];
      P2.v1 = sp[2][l2];
      P2.v2 = sp[3][l2];
      P2.p = sp[4][l2];
      P2.lr = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 2 : 0][l2] : Real(0);
      P2.b = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 3 : 0][l2] : Real(0);
      P2.lb = NP > DIM + 2 ? sp[(NP > DIM + 2) ? DIM + 4 : 0][l2] : Real(0);
      Real n2[3] = {Real(0), Real(0), Real(0)};
      if constexpr (CNODE) { n2[0] = sn0[0][l2]; n2[1] = sn0[1][l2]; n2[2] = sn0[2][l2]; }
      pair_fluxes<2, DIM, N, N, VF, MESH, Real, NNL, LPAD>(sp, sn0, P2, n2, i2, z2, lane, s_dts, P.scale[2],
                                                           a.ops.inv_gm1, Ad);
      __syncthreads();  // every lane has read the primitives
      if (ok2)
#pragma unroll
        for (int v = 0; v < NV; ++v) s_acc[0][v][l2] = Ad[v];
      __syncthreads();
#pragma unroll
      for (int v = 0; v < NV; ++v) Sn[v] += s_acc[0][v][li];
    } else {
      node_fluxes<2, DIM, N, VF, MESH, Real>(sp, sn0, Po, no, i, iz, s_dts, P.scale[2], a.ops.inv_gm1, Ad);
#pragma unroll
      for (int v = 0; v < NV; ++v) Sn[v] += Ad[v];
    }
  }

  // ---- volume term, line layout: each lane sweeps the pairs of its line
  Real A[N][NV];
  if constexpr (!NODEL) {
    const Real(*sp)[NN] = s_prim[lactive ? lel : 0];
    const Real sc = P.scale[ldir];
    if (ldir == 0) line_fluxes<0, DIM, N, VF, MESH, Real, NODES>(sp, nrm, lbase, a.ops, s_dt, sc, A, fo, fnb, a.surf);
    else if (DIM > 1 && ldir == 1)
      line_fluxes<(DIM > 1 ? 1 : 0), DIM, N, VF, MESH, Real, NODES>(sp, nrm, lbase, a.ops, s_dt, sc, A, fo, fnb, a.surf);
    else if (DIM > 2)
      line_fluxes<(DIM > 2 ? 2 : 0), DIM, N, VF, MESH, Real, NODES>(sp, nrm, lbase, a.ops, s_dt, sc, A, fo, fnb, a.surf);
  }
  // RK registers of the owned nodes, in flight while the line sums are merged
  Real ru0[NPT][NV], racc[NPT][NV];
  const bool need_u0 = a.mode == MODE_RK_MID;
  const bool need_acc =
      a.mode == MODE_RK_MID || a.mode == MODE_RK_LAST || a.mode == MODE_LS_MID || a.mode == MODE_LS_LAST;
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int q = tid + r * THREADS;
    int el = q / NN, i = q - el * NN;
    bool ok = q < EPB * NN && e0 + el < E;
    if constexpr (PMAP) {
      el = 0;
      ok = plane_node<N>(q, i) && e0 < E;
    }
    const size_t o = ok ? (size_t)(e0 + el) * (NV * NN) + i : 0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      ru0[r][v] = need_u0 ? u0[o + (size_t)v * NN] : Real(0);
      racc[r][v] = need_acc ? racc_buf[o + (size_t)v * NN] : Real(0);
    }
  }
  // fixed summation order over directions: dir 0 writes, then dir 1, dir 2 add
  if constexpr (!NODEL) __syncthreads();  // every line's primitives are read
#pragma unroll
  for (int d = 0; d < (NODEL ? 0 : DIM); ++d) {
    if (ldir == d && lactive) {
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const int q = lbase + k * stride;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          if (d == 0) s_acc[lel][v][q] = A[k][v];
          else s_acc[lel][v][q] += A[k][v];
        }
      }
    }
    __syncthreads();
  }

  // ---- epilogue: lifting, -1/J, stage update
  double dt = a.dt_fixed;
  if (a.mode == MODE_RHS) dt = 0.0;
  if (a.mode != MODE_RHS && cfl_mode) {
    // every wave folds the slots: lane l reads slot l, then a max over the wave
    double lam = __longlong_as_double((long long)lam_in[tid & (kLamSlots - 1)]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(lam, off, 64);
      if (!(o <= lam)) lam = o;
    }
    dt = a.cfl * 2.0 / ((double)N * lam);
  }
  if (a.mode != MODE_RHS) {
    const auto time = as_global(P.time);
    const double t0 = time[a.par];
    const double rem = P.t_end - t0;
    if (dt > rem) dt = rem > 0.0 ? rem : 0.0;  // a NaN dt stays NaN
    if (e0 == 0 && first_stage && cfl_mode && tid < kLamSlots) lam_next[tid] = 0ull;
    if (e0 == 0 && last_stage && tid == 0) time[1 - a.par] = t0 + dt;
  }
  double lam_max = 0.0;  // CFL wave-speed sum of the new state (LAST stage)
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int q = tid + r * THREADS;
    int el = q / NN, i = q - el * NN;
    if constexpr (PMAP) {
      el = 0;
      if (!(plane_node<N>(q, i) && e0 < E)) continue;
    } else if (!(q < EPB * NN && e0 + el < E)) {
      continue;
    }
    const int ee = e0 + el;
    const int ix = i % N;
    const int iy = DIM > 1 ? (i / N) % N : 0;
    const int iz = DIM > 2 ? i / (N * N) : 0;
    Real S[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) S[v] = NODEL ? Sn[v] : s_acc[NODEL ? 0 : el][v][NODEL ? 0 : i];
#pragma unroll
    for (int dir = 0; dir < DIM && NODES == NODES_LGL; ++dir) {
      const int id = dir == 0 ? ix : (dir == 1 ? iy : iz);
      if (id != 0 && id != N - 1) continue;
      const int f = dir == 0 ? (iy + N * iz) : (dir == 1 ? (ix + N * iz) : (ix + N * iy));
      const Real sc = MESH == MESH_AFFINE ? P.scale[dir] : Real(1);
      if (id == N - 1) {
        const Real w = sc * a.ops.inv_wp;
#pragma unroll
        for (int v = 0; v < NV; ++v) S[v] += w * s_face[el][v][(2 * dir + 1) * NF + f];
      }
      if (id == 0) {
        const Real w = sc * a.ops.inv_w0;
#pragma unroll
        for (int v = 0; v < NV; ++v) S[v] -= w * s_face[el][v][(2 * dir) * NF + f];
      }
    }
    const Real mul = -rinvj[r];
    const size_t base = (size_t)ee * (NV * NN) + i;
    Real unew[NV] = {};
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const Real k = mul * S[v];
      const size_t o = base + (size_t)v * NN;
      if (a.mode == MODE_RHS) {
        out[o] = k;
      } else if (a.mode == MODE_RK_FIRST) {
        // the stage input is read again (an L2 hit) rather than kept live in
        // registers through the line phase
        const Real u_in = uin[o];
        if constexpr (PRIO) {
          __builtin_nontemporal_store(u_in + a.coef_b * (Real)dt * k, racc_buf + o);
          __builtin_nontemporal_store(u_in + a.coef_a * (Real)dt * k, out + o);
        } else {
          racc_buf[o] = u_in + a.coef_b * (Real)dt * k;
          out[o] = u_in + a.coef_a * (Real)dt * k;
        }
      } else if (a.mode == MODE_RK_MID) {
        if constexpr (PRIO) {
          __builtin_nontemporal_store(racc[r][v] + a.coef_b * (Real)dt * k, racc_buf + o);
          __builtin_nontemporal_store(ru0[r][v] + a.coef_a * (Real)dt * k, out + o);
        } else {
          racc_buf[o] = racc[r][v] + a.coef_b * (Real)dt * k;
          out[o] = ru0[r][v] + a.coef_a * (Real)dt * k;
        }
      } else if (a.mode >= MODE_LS_FIRST) {
        // 2N storage: the accumulator holds du
        const Real d = a.mode == MODE_LS_FIRST ? (Real)dt * k : a.coef_a * racc[r][v] + (Real)dt * k;
        racc_buf[o] = d;
        unew[v] = uin[o] + a.coef_b * d;
        out[o] = unew[v];
      } else {
        unew[v] = racc[r][v] + a.coef_b * (Real)dt * k;
        if constexpr (PRIO) __builtin_nontemporal_store(unew[v], out + o);
        else out[o] = unew[v];
      }
    }
    if (lam_out) {
      // CFL wave-speed sum of the new state at this node
      const auto me = MESH == MESH_CURVED ? metric + (size_t)ee * (NM * NN) + i : metric;
      const double ld = cfl_rate<DIM, MESH, Real>(unew, me, (int64_t)NN, rinvj[r], P.scale, a.gamma64);
      if (!(ld <= lam_max)) lam_max = ld;  // a NaN wins and poisons dt (flagged anyway)
    }
  }
  if (lam_out) {
    // max over the wave, then one atomic per wave: max is exact, so the
    // result does not depend on the order of the atomics
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(lam_max, off, 64);
      if (!(o <= lam_max)) lam_max = o;
    }
    if ((tid & 63) == 0)
      atomicMax(lam_next + (blockIdx.x & (kLamSlots - 1)), (unsigned long long)__double_as_longlong(lam_max));
  }
}

// ---------------------------------------------------------------------------
// Gauss collocation: entropy projection to the face points (Sec. 6)
// ---------------------------------------------------------------------------

// u~ = u(R w(u)) at every face point of the tile's elements: entropy
// variables w = ((gamma - s)/(gamma-1) - beta|v|^2/2, beta v, -beta),
// beta = rho/p, s = ln p - gamma ln rho, at the nodes (LDS); their values at
// the element ends along each line (rows of R); back to primitive variables
// with beta = -w_E, v = w_m/beta, s = gamma - (gamma-1)(w_0 + beta|v|^2/2),
// ln p = (s + gamma ln beta)/(1 - gamma), ln rho = ln beta + ln p.  Written
// to faceb as (rho, v, p, ln rho, ln beta) per face point; launched before each
// Gauss stage on the same tiles and descriptors.  The projection is evaluated
// in FP64 for both precisions: the map back from w cancels digits (ln p from
// s and ln beta), which FP32 would expose at ~1e-6 relative.
template <int DIM, int N, typename Real>
__global__ void __launch_bounds__((Tile<DIM, N>::THREADS)) gauss_project_kernel(StageArgs<Real> a) {
  using T = Tile<DIM, N>;
  constexpr int NN = T::NN, NF = T::NF, EPB = T::EPB, NV = T::NV, NFACE = T::NFACE;
  constexpr int THREADS = T::THREADS, NPT = T::NPT, FPT = T::FPT;
  constexpr int NPF = DIM + 4;
  __shared__ double s_w[EPB][NV][NN];
  const int tid = threadIdx.x;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int pi = a.tile_prob ? a.tile_prob[tile] : 0;
  const ProbDesc<Real>& P = a.probs[pi];
  const auto uin = as_global((const Real*)P.buf[a.in_idx]);
  const auto fb = as_global(P.faceb);
  const int E = P.E;
  const int e0 = (tile - P.tile0) * EPB;
  const double g = (double)a.ops.gamma, gm1 = g - 1.0, inv_gm1 = 1.0 / gm1;
#pragma unroll
  for (int r = 0; r < NPT; ++r) {
    const int q = tid + r * THREADS;
    const int el = q / NN, i = q - el * NN;
    if (!(q < EPB * NN && e0 + el < E)) continue;
    const size_t o = (size_t)(e0 + el) * (NV * NN) + i;
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = (double)uin[o + (size_t)v * NN];
    const double ir = dev_rcp(u[0]);
    double kin = 0.0;
#pragma unroll
    for (int m = 0; m < DIM; ++m) kin += u[1 + m] * u[1 + m];
    kin *= ir;  // rho |v|^2
    const double p = gm1 * (u[DIM + 1] - 0.5 * kin);
    const double beta = u[0] * dev_rcp(p);
    const double s = log(p) - g * log(u[0]);
    s_w[el][0][i] = (g - s) * inv_gm1 - 0.5 * beta * (kin * ir);
#pragma unroll
    for (int m = 0; m < DIM; ++m) s_w[el][1 + m][i] = beta * (u[1 + m] * ir);
    s_w[el][DIM + 1][i] = -beta;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < FPT; ++r) {
    const int t = tid + r * THREADS;
    const int el = t / NFACE, rr = t - el * NFACE;
    if (!(t < EPB * NFACE && e0 + el < E)) continue;
    const int fc = rr / NF, f = rr - fc * NF, dir = fc >> 1, side = fc & 1;
    double w[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) w[v] = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const double rk = a.ops.r64[side][k];
      const int q = face_node<N>(dir, f, k);
#pragma unroll
      for (int v = 0; v < NV; ++v) w[v] += rk * s_w[el][v][q];
    }
    const double beta = -w[DIM + 1], ib = dev_rcp(beta);
    double vel[3] = {0.0, 0.0, 0.0}, v2 = 0.0;
#pragma unroll
    for (int m = 0; m < DIM; ++m) {
      vel[m] = w[1 + m] * ib;
      v2 += vel[m] * vel[m];
    }
    const double s = g - gm1 * (w[0] + 0.5 * beta * v2);
    const double lb = log(beta);
    const double lp = (s + g * lb) / (1.0 - g);
    const double lr = lb + lp;
    const double rho = exp(lr), p = exp(lp);
    if (!(beta > 0.0) || !isfinite(rho + p)) *(volatile int*)P.flag = 1;
    const size_t o = (((size_t)(e0 + el) * (2 * DIM) + fc) * NPF) * NF + f;
    fb[o] = (Real)rho;
#pragma unroll
    for (int m = 0; m < DIM; ++m) fb[o + (size_t)(1 + m) * NF] = (Real)vel[m];
    fb[o + (size_t)(DIM + 1) * NF] = (Real)p;
    fb[o + (size_t)(DIM + 2) * NF] = (Real)lr;
    fb[o + (size_t)(DIM + 3) * NF] = (Real)lb;
  }
}

// ---------------------------------------------------------------------------
// FP64 reductions (fixed order: per-block tree, then one block over partials)
// ---------------------------------------------------------------------------

template <typename Real>
struct RedArgs {
  const Real* u;        // state
  const Real* du;       // RHS (RED_ENTROPY)
  const Real* metric;   // curved metrics (1/J and Ja)
  double* partial;      // [blocks][K]
  int64_t E;
  int N, dim, nn;
  double J_affine, inv_half_h[3];
  double w[kDevMaxN];
  double gamma;
  Real scale[3];        // 2/h_n of the affine box in the state's precision (CFL)
};

constexpr int kRedThreads = 256;

template <int DIM, int MESH, int OP, typename Real>
__global__ void __launch_bounds__(kRedThreads) reduce_partial_kernel(RedArgs<Real> a, int64_t per_block) {
  constexpr int NV = DIM + 2;
  constexpr int K = OP == RED_TOTALS ? NV : 1;
  __shared__ double sh[K][kRedThreads];
  double accv[K];
#pragma unroll
  for (int k = 0; k < K; ++k) accv[k] = 0.0;
  const int nn = a.nn, N = a.N;
  const int64_t total = a.E * nn;
  const int64_t start = (int64_t)blockIdx.x * per_block;
  const int64_t stop = start + per_block < total ? start + per_block : total;
  const int NM = DIM * DIM + 1;
  const double gm1 = a.gamma - 1.0;
  for (int64_t g = start + threadIdx.x; g < stop; g += kRedThreads) {
    const int64_t e = g / nn;
    const int i = (int)(g - e * nn);
    double W = a.w[i % N];
    if (DIM > 1) W *= a.w[(i / N) % N];
    if (DIM > 2) W *= a.w[i / (N * N)];
    const double J = MESH == MESH_CURVED ? 1.0 / (double)a.metric[(e * NM + DIM * DIM) * nn + i] : a.J_affine;
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = (double)a.u[(e * NV + v) * nn + i];
    if (OP == RED_TOTALS) {
#pragma unroll
      for (int v = 0; v < NV; ++v) accv[v] += J * W * u[v];
    } else {
      const double rho = u[0], ir = 1.0 / rho;
      double v2 = 0.0, mv = 0.0;
      double vel[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int m = 0; m < DIM; ++m) {
        vel[m] = u[1 + m] * ir;
        v2 += vel[m] * vel[m];
        mv += u[1 + m] * vel[m];
      }
      const double p = gm1 * (u[DIM + 1] - 0.5 * mv);
      if (OP == RED_ENTROPY) {
        // w = ((gamma - s)/(gamma-1) - rho|v|^2/(2p), rho v/p, -rho/p), s = ln p - gamma ln rho
        const double s = log(p) - a.gamma * log(rho);
        const double beta = rho / p;
        double dot = ((a.gamma - s) / gm1 - 0.5 * beta * v2) * (double)a.du[(e * NV) * nn + i];
#pragma unroll
        for (int m = 0; m < DIM; ++m) dot += beta * vel[m] * (double)a.du[(e * NV + 1 + m) * nn + i];
        dot -= beta * (double)a.du[(e * NV + DIM + 1) * nn + i];
        accv[0] += J * W * dot;
      } else {
        // the expression of the last RK stage, in the state's precision
        Real ur[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) ur[v] = a.u[(e * NV + v) * nn + i];
        const Real* me = MESH == MESH_CURVED ? a.metric + e * NM * nn + i : a.metric;
        const Real rinvj = MESH == MESH_CURVED ? a.metric[(e * NM + DIM * DIM) * nn + i] : Real(1);
        const double lam = cfl_rate<DIM, MESH, Real>(ur, me, (int64_t)nn, rinvj, a.scale, a.gamma);
        if (!(lam <= accv[0])) accv[0] = lam;  // NaN propagates
      }
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) sh[k][threadIdx.x] = accv[k];
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (OP == RED_MAXLAMBDA) {
          const double o = sh[k][threadIdx.x + s];
          if (!(o <= sh[k][threadIdx.x])) sh[k][threadIdx.x] = o;
        } else {
          sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        }
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < K) a.partial[(int64_t)blockIdx.x * K + threadIdx.x] = sh[threadIdx.x][0];
}

// Final pass: one block folds the partials in index order.  For
// RED_MAXLAMBDA it turns lam_max into dt = cfl*2/(N lam_max) (out[0]) and, if
// lam_slot is given, stores lam_max in its first slot (bit pattern of the
// double) and zero in the other kLamSlots - 1.
template <int OP>
__global__ void __launch_bounds__(kRedThreads) reduce_final_kernel(const double* partial, int blocks, int K,
                                                                     double* out, double cfl, int N,
                                                                     unsigned long long* lam_slot) {
  __shared__ double sh[kRedThreads];
  for (int k = 0; k < K; ++k) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < blocks; b += kRedThreads) {
      const double v = partial[(int64_t)b * K + k];
      if (OP == RED_MAXLAMBDA) {
        if (!(v <= acc)) acc = v;
      } else {
        acc += v;
      }
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        if (OP == RED_MAXLAMBDA) {
          const double o = sh[threadIdx.x + s];
          if (!(o <= sh[threadIdx.x])) sh[threadIdx.x] = o;
        } else {
          sh[threadIdx.x] += sh[threadIdx.x + s];
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      if (OP == RED_MAXLAMBDA) out[k] = cfl * 2.0 / ((double)N * sh[0]);
      else out[k] = sh[0];
    }
    if (OP == RED_MAXLAMBDA && lam_slot && threadIdx.x < kLamSlots)
      lam_slot[threadIdx.x] = threadIdx.x == 0 ? (unsigned long long)__double_as_longlong(sh[0]) : 0ull;
    __syncthreads();
  }
}


// ---------------------------------------------------------------------------
// face fluxes once per face (LGL, one problem): the organisation Sec. 2.4
// names as the usual efficient one on CPUs (and Sec. 6 reports for the LGL
// solver it times); an option beside the fused default, which evaluates each
// face from both of its elements inside the stage kernel
// ---------------------------------------------------------------------------

constexpr int kFaceThreads = 256;

// One lane per node of an element's + face in each direction: f*(u_L, u_R, n)
// with u_L the element's trace at position N-1, u_R the + neighbour's at 0
// and n the normal of the element's + face, the inputs (and so the bits) the
// stage kernel uses when it evaluates the face from either side.  Writes
// a.fstar[e][dir][v][f] from the stage input buf[in_idx] of a.probs[0].
template <int DIM, int N, int MESH, typename Real>
__global__ void __launch_bounds__(kFaceThreads) face_kernel(StageArgs<Real> a) {
  constexpr int NV = DIM + 2, NF = Pow<N, DIM - 1>::value, NN = Pow<N, DIM>::value;
  const ProbDesc<Real>& P = a.probs[0];
  const int E = P.E, n0 = P.n0, n1 = P.n1, n2 = P.n2;
  const int64_t g = (int64_t)blockIdx.x * kFaceThreads + threadIdx.x;
  if (g >= (int64_t)E * DIM * NF) return;
  const int e = (int)(g / (DIM * NF));
  const int rem = (int)(g - (int64_t)e * (DIM * NF));
  const int dir = rem / NF, f = rem - dir * NF;
  const int ex = e % n0, ey = (e / n0) % n1, ez = e / (n0 * n1);
  int en;
  if (dir == 0) en = (ex == n0 - 1 ? 0 : ex + 1) + n0 * (ey + n1 * ez);
  else if (dir == 1) en = ex + n0 * ((ey == n1 - 1 ? 0 : ey + 1) + n1 * ez);
  else en = ex + n0 * (ey + n1 * (ez == n2 - 1 ? 0 : ez + 1));
  const auto uin = as_global((const Real*)P.buf[a.in_idx]);
  const int qL = face_node<N>(dir, f, N - 1), qR = face_node<N>(dir, f, 0);
  Real tL[NV], tR[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    tL[v] = uin[(size_t)e * (NV * NN) + v * NN + qL];
    tR[v] = uin[(size_t)en * (NV * NN) + v * NN + qR];
  }
  Real nx, ny, nz;
  if (MESH == MESH_CURVED) {
    const auto nf = as_global(P.nface) + ((size_t)dir * E + e) * (DIM * NF) + f;
    nx = nf[0];
    ny = DIM > 1 ? nf[NF] : Real(0);
    nz = DIM > 2 ? nf[2 * NF] : Real(0);
  } else {
    nx = dir == 0 ? Real(1) : Real(0);
    ny = dir == 1 ? Real(1) : Real(0);
    nz = dir == 2 ? Real(1) : Real(0);
  }
  Real F[NV];
  surface_flux<DIM>(a.surf, tL, tR, nx, ny, nz, a.ops.gamma, a.ops.inv_gm1, F);
  const auto out = as_global(a.fstar) + ((size_t)e * DIM + dir) * (NV * NF) + f;
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v * NF] = F[v];
}

}  // namespace esdg
