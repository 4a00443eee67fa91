// Device kernels of the flux-differencing LGL-DGSEM (gfx950, wave64).
//
// Per right-hand side (or RK stage) two launches:
//   face_kernel   one thread per face node: gathers the two traces and writes
//                 the surface flux f* once per face (Sec. 2.4 remark on
//                 computing surface fluxes once per surface);
//   volume_kernel one 64-lane workgroup per tile of EPB elements:
//                 prologue  coalesced load of u, primitive variables and
//                           log(rho), log(p) once per node into LDS
//                           (Sec. 7.1/7.2 precomputation);
//                 sweeps    per direction, one lane per line, each lane
//                           evaluating the i<k pairs of its line once and
//                           scattering D~_ik F to node i and D~_ki F to node k
//                           (skew-symmetric D~, Sec. 2.2; tensor-product
//                           sparsity, Sec. 2.3), accumulated in LDS in a fixed
//                           direction order (deterministic, no atomics);
//                 epilogue  lifting of the face fluxes (+f*/w_p, -f*/w_0),
//                           scaling by -1/J and the fused RK stage update.
// MFMA is not used: the volume term is an element-wise two-point flux
// followed by a row-sum, not a dense contraction.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace esdg {

enum VolFlux { VF_RANOCHA = 0, VF_SHIMA = 1, VF_CENTRAL = 3 };
enum SurfFlux { SF_RANOCHA = 0, SF_SHIMA = 1, SF_LLF = 2, SF_CENTRAL = 3 };
enum MeshKind { MESH_AFFINE = 0, MESH_CURVED = 1 };
enum StageMode { MODE_RHS = 0, MODE_RK_FIRST = 1, MODE_RK_MID = 2, MODE_RK_LAST = 3 };
enum RedOp { RED_TOTALS = 0, RED_ENTROPY = 1, RED_MAXLAMBDA = 2 };

constexpr int kDevMaxN = 8;

template <typename Real>
struct LineOps {
  Real Dt[kDevMaxN * kDevMaxN];  // D~ row-major
  Real inv_w0, inv_wp;           // 1/w_0, 1/w_p
  Real scale[3];                 // affine: 2/h_n ; curved: 1
  Real gamma, inv_gm1;           // gamma, 1/(gamma-1)
};

template <typename Real>
struct VolArgs {
  const Real* uin;     // stage input state [E][nv][nn]
  const Real* metric;  // curved: [E][dim*dim+1][nn] (Ja^n_m, then 1/J)
  const Real* fstar;   // [dim][E][nv][nf] surface fluxes of + faces
  Real* out;           // MODE_RHS: du; RK: stage output y (FIRST, MID) or state (LAST)
  Real* acc;           // RK accumulator
  const Real* u0;      // RK state at the start of the step (MID)
  const double* dt;    // device scalar time step
  int* flag;           // non-physical state flag
  int64_t E;
  int n0, n1, n2;      // elements per direction
  int mode;
  Real coef_b, coef_a; // RK: acc += b dt k ; y = u0 + a dt k
  LineOps<Real> ops;
};

template <typename Real>
struct FaceArgs {
  const Real* u;       // [E][nv][nn]
  const Real* nface;   // curved: [dim][E][dim][nf]
  Real* fstar;         // [dim][E][nv][nf]
  int64_t E;
  int n0, n1, n2;
  int N;
  Real gamma, inv_gm1;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

template <int B, int K>
struct Pow { static constexpr int value = B * Pow<B, K - 1>::value; };
template <int B>
struct Pow<B, 0> { static constexpr int value = 1; };

template <typename Real> struct LogMeanEps;
template <> struct LogMeanEps<double> { static constexpr double value = 1.0e-4; };
template <> struct LogMeanEps<float> { static constexpr float value = 2.0e-2f; };

__device__ __forceinline__ double dev_log(double x) { return log(x); }
__device__ __forceinline__ float dev_log(float x) { return __logf(x); }

// Primitive variables at one node, with log(rho) and log(p) when the volume
// flux needs log means.
template <typename Real>
struct Prim {
  Real rho, v0, v1, v2, p, lr, lp;
};

// ---------------------------------------------------------------------------
// two-point volume fluxes in direction n (Sec. 3.2), from primitive values
// ---------------------------------------------------------------------------

// Log mean and inverse log mean (Sec. 3.1, Algorithms 2 and 3) with the
// node logarithms precomputed (Sec. 7.2).  The branch of the algorithms,
// u = ((a+ - a-)/(a+ + a-))^2 < eps, is decided without a division as
// (a+ - a-)^2 < eps (a+ + a-)^2; each mean then costs one reciprocal:
//   LM : series (a- + a+)(1/2 - u/6 - 2u^2/45 - 22u^3/945)  [the division-free
//        variant of Algorithm 2 given in Sec. 3.1]   or   (a+ - a-) / (la+ - la-)
//   ILM: series (2 + 2u/3 + 2u^2/5 + 2u^3/7)/(a- + a+)   or   (la+ - la-)/(a+ - a-)
template <typename Real>
__device__ __forceinline__ Real log_mean_pre(Real am, Real ap, Real lam, Real lap) {
  const Real s = am + ap, d = ap - am;
  const bool series = d * d < LogMeanEps<Real>::value * (s * s);
  const Real r = Real(1) / (series ? s : (lap - lam));
  const Real f = d * r;
  const Real u = f * f;
  const Real poly = Real(0.5) + u * (Real(-1.0 / 6.0) + u * (Real(-2.0 / 45.0) + u * Real(-22.0 / 945.0)));
  return series ? s * poly : f;
}

template <typename Real>
__device__ __forceinline__ Real inv_log_mean_pre(Real am, Real ap, Real lam, Real lap) {
  const Real s = am + ap, d = ap - am;
  const bool series = d * d < LogMeanEps<Real>::value * (s * s);
  const Real r = Real(1) / (series ? s : d);
  const Real f = d * r;
  const Real u = f * f;
  const Real poly = Real(2) + u * (Real(2.0 / 3.0) + u * (Real(2.0 / 5.0) + u * Real(2.0 / 7.0)));
  return series ? r * poly : (lap - lam) * r;
}

// Directional volume flux f(u_i, u_k, n) into F[0..DIM+1].  NX/NY/NZ are the
// normal components (compile-time constants for the affine mesh).
template <int VF, int DIM, typename Real>
__device__ __forceinline__ void volume_flux(const Prim<Real>& a, const Prim<Real>& b, Real nx, Real ny,
                                            Real nz, Real inv_gm1, Real* F) {
  const Real vna = a.v0 * nx + (DIM > 1 ? a.v1 * ny : Real(0)) + (DIM > 2 ? a.v2 * nz : Real(0));
  const Real vnb = b.v0 * nx + (DIM > 1 ? b.v1 * ny : Real(0)) + (DIM > 2 ? b.v2 * nz : Real(0));
  const Real vn_avg = Real(0.5) * (vna + vnb);
  const Real p_avg = Real(0.5) * (a.p + b.p);
  const Real vv = a.v0 * b.v0 + (DIM > 1 ? a.v1 * b.v1 : Real(0)) + (DIM > 2 ? a.v2 * b.v2 : Real(0));
  const Real pvn = Real(0.5) * (b.p * vna + a.p * vnb);  // ((p; v.n))
  if (VF == VF_CENTRAL) {
    // (f(u_a) + f(u_b)).n / 2 with f written in primitive variables
    const Real ka = a.rho * vna, kb = b.rho * vnb;
    F[0] = Real(0.5) * (ka + kb);
    F[1] = Real(0.5) * (ka * a.v0 + kb * b.v0) + p_avg * nx;
    if (DIM > 1) F[2] = Real(0.5) * (ka * a.v1 + kb * b.v1) + p_avg * ny;
    if (DIM > 2) F[3] = Real(0.5) * (ka * a.v2 + kb * b.v2) + p_avg * nz;
    const Real va2 = a.v0 * a.v0 + (DIM > 1 ? a.v1 * a.v1 : Real(0)) + (DIM > 2 ? a.v2 * a.v2 : Real(0));
    const Real vb2 = b.v0 * b.v0 + (DIM > 1 ? b.v1 * b.v1 : Real(0)) + (DIM > 2 ? b.v2 * b.v2 : Real(0));
    const Real ea = a.p * inv_gm1 + Real(0.5) * a.rho * va2 + a.p;
    const Real eb = b.p * inv_gm1 + Real(0.5) * b.rho * vb2 + b.p;
    F[DIM + 1] = Real(0.5) * (ea * vna + eb * vnb);
    return;
  }
  Real frho, fe_int;
  if (VF == VF_RANOCHA) {
    frho = log_mean_pre(a.rho, b.rho, a.lr, b.lr) * vn_avg;
    // 1/{{rho/p}}_log = p_a p_b / {{rho_a p_b, rho_b p_a}}_log (Sec. 3.2)
    const Real ilm = inv_log_mean_pre(a.rho * b.p, b.rho * a.p, a.lr + b.lp, b.lr + a.lp);
    fe_int = frho * (a.p * b.p) * ilm * inv_gm1;
  } else {  // Shima et al.
    frho = Real(0.5) * (a.rho + b.rho) * vn_avg;
    fe_int = p_avg * vn_avg * inv_gm1;
  }
  F[0] = frho;
  F[1] = frho * Real(0.5) * (a.v0 + b.v0) + p_avg * nx;
  if (DIM > 1) F[2] = frho * Real(0.5) * (a.v1 + b.v1) + p_avg * ny;
  if (DIM > 2) F[3] = frho * Real(0.5) * (a.v2 + b.v2) + p_avg * nz;
  F[DIM + 1] = Real(0.5) * frho * vv + fe_int + pvn;
}

// ---------------------------------------------------------------------------
// volume kernel
// ---------------------------------------------------------------------------

template <int DIM, int N>
struct Tile {
  static constexpr int NN = Pow<N, DIM>::value;      // nodes per element
  static constexpr int L = NN / N;                    // lines per direction
  static constexpr int EPB = (64 / L) > 0 ? 64 / L : 1;  // elements per block
  static constexpr int THREADS = 64;
  static constexpr int NV = DIM + 2;
};

template <int VF, int DIM>
struct PrimCount { static constexpr int value = (VF == VF_RANOCHA) ? DIM + 4 : DIM + 2; };

// one direction of the flux-differencing sweep for one line
template <int DIR, int DIM, int N, int VF, int MESH, typename Real>
__device__ __forceinline__ void line_sweep(const Real* __restrict__ sp, Real* __restrict__ sa,
                                           const Real* __restrict__ metric_e, int line, bool first,
                                           const LineOps<Real>& ops) {
  using T = Tile<DIM, N>;
  constexpr int NN = T::NN;
  constexpr int NV = T::NV;
  constexpr int NP = PrimCount<VF, DIM>::value;
  constexpr int stride = Pow<N, DIR>::value;
  // base node of the line: remove the DIR digit
  const int lo_part = line % stride;
  const int hi_part = line / stride;
  const int base = lo_part + hi_part * stride * N;

  Prim<Real> P[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int q = base + k * stride;
    P[k].rho = sp[0 * NN + q];
    P[k].v0 = sp[1 * NN + q];
    P[k].v1 = DIM > 1 ? sp[2 * NN + q] : Real(0);
    P[k].v2 = DIM > 2 ? sp[3 * NN + q] : Real(0);
    P[k].p = sp[(DIM + 1) * NN + q];
    if (NP > DIM + 2) {
      P[k].lr = sp[(DIM + 2) * NN + q];
      P[k].lp = sp[(DIM + 3) * NN + q];
    } else {
      P[k].lr = P[k].lp = Real(0);
    }
  }
  Real nrm[N][3];
  if (MESH == MESH_CURVED) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const int q = base + k * stride;
#pragma unroll
      for (int m = 0; m < 3; ++m) nrm[k][m] = m < DIM ? metric_e[(DIR * DIM + m) * NN + q] : Real(0);
    }
  }
  Real A[N][NV];
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
        const Real nx = Real(0.5) * (nrm[i][0] + nrm[k][0]);
        const Real ny = Real(0.5) * (nrm[i][1] + nrm[k][1]);
        const Real nz = Real(0.5) * (nrm[i][2] + nrm[k][2]);
        volume_flux<VF, DIM>(P[i], P[k], nx, ny, nz, ops.inv_gm1, F);
      } else {
        volume_flux<VF, DIM>(P[i], P[k], DIR == 0 ? Real(1) : Real(0), DIR == 1 ? Real(1) : Real(0),
                             DIR == 2 ? Real(1) : Real(0), ops.inv_gm1, F);
      }
      const Real dik = ops.Dt[i * N + k], dki = ops.Dt[k * N + i];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        A[i][v] += dik * F[v];
        A[k][v] += dki * F[v];
      }
    }
  }
  const Real sc = MESH == MESH_AFFINE ? ops.scale[DIR] : Real(1);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int q = base + k * stride;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const Real val = MESH == MESH_AFFINE ? sc * A[k][v] : A[k][v];
      if (first) sa[v * NN + q] = val;
      else sa[v * NN + q] += val;
    }
  }
}

template <int DIM, int N, int VF, int MESH, typename Real>
__global__ void __launch_bounds__(64) volume_kernel(VolArgs<Real> a) {
  using T = Tile<DIM, N>;
  constexpr int NN = T::NN, L = T::L, EPB = T::EPB, NV = T::NV;
  constexpr int NP = PrimCount<VF, DIM>::value;
  constexpr int NF = NN / N;
  constexpr int NM = DIM * DIM + 1;
  __shared__ Real s_prim[EPB][NP * NN];
  __shared__ Real s_acc[EPB][NV * NN];

  const int tid = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * EPB;
  const Real gm1 = a.ops.gamma - Real(1);

  // prologue: primitive variables (and logs) once per node
  for (int q = tid; q < EPB * NN; q += T::THREADS) {
    const int el = q / NN, i = q - el * NN;
    const int64_t e = e0 + el;
    if (e >= a.E) continue;
    const Real* ue = a.uin + e * NV * NN;
    const Real rho = ue[i];
    const Real inv_rho = Real(1) / rho;
    const Real m0 = ue[NN + i];
    const Real m1 = DIM > 1 ? ue[2 * NN + i] : Real(0);
    const Real m2 = DIM > 2 ? ue[3 * NN + i] : Real(0);
    const Real E_ = ue[(DIM + 1) * NN + i];
    const Real v0 = m0 * inv_rho, v1 = m1 * inv_rho, v2 = m2 * inv_rho;
    const Real p = gm1 * (E_ - Real(0.5) * (m0 * v0 + m1 * v1 + m2 * v2));
    if (!(rho > Real(0)) || !(p > Real(0)) || !isfinite(E_) || !isfinite(m0 + m1 + m2)) atomicOr(a.flag, 1);
    Real* sp = s_prim[el];
    sp[0 * NN + i] = rho;
    sp[1 * NN + i] = v0;
    if (DIM > 1) sp[2 * NN + i] = v1;
    if (DIM > 2) sp[3 * NN + i] = v2;
    sp[(DIM + 1) * NN + i] = p;
    if (NP > DIM + 2) {
      sp[(DIM + 2) * NN + i] = dev_log(rho);
      sp[(DIM + 3) * NN + i] = dev_log(p);
    }
  }
  __syncthreads();

  // flux-differencing sweeps, one direction after the other
  const int el = tid / L, line = tid - el * L;
  const int64_t e = e0 + el;
  const bool active = (tid < EPB * L) && (e < a.E);
  const Real* me = MESH == MESH_CURVED && active ? a.metric + e * NM * NN : nullptr;
  if (active) line_sweep<0, DIM, N, VF, MESH>(s_prim[el], s_acc[el], me, line, true, a.ops);
  __syncthreads();
  if (DIM > 1) {
    if (active) line_sweep<(DIM > 1 ? 1 : 0), DIM, N, VF, MESH>(s_prim[el], s_acc[el], me, line, false, a.ops);
    __syncthreads();
  }
  if (DIM > 2) {
    if (active) line_sweep<(DIM > 2 ? 2 : 0), DIM, N, VF, MESH>(s_prim[el], s_acc[el], me, line, false, a.ops);
    __syncthreads();
  }

  // epilogue: lifting, -1/J, stage update
  const double dt = (a.mode == MODE_RHS) ? 0.0 : *a.dt;
  for (int q = tid; q < EPB * NN; q += T::THREADS) {
    const int el2 = q / NN, i = q - el2 * NN;
    const int64_t ee = e0 + el2;
    if (ee >= a.E) continue;
    const int ix = i % N;
    const int iy = DIM > 1 ? (i / N) % N : 0;
    const int iz = DIM > 2 ? i / (N * N) : 0;
    const int64_t ex = ee % a.n0;
    const int64_t ey = (ee / a.n0) % a.n1;
    const int64_t ez = ee / ((int64_t)a.n0 * a.n1);
    Real S[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) S[v] = s_acc[el2][v * NN + i];
#pragma unroll
    for (int dir = 0; dir < DIM; ++dir) {
      const int id = dir == 0 ? ix : (dir == 1 ? iy : iz);
      if (id != 0 && id != N - 1) continue;
      // face node index: the other node indices, lowest direction first
      const int f = dir == 0 ? (iy + N * iz) : (dir == 1 ? (ix + N * iz) : (ix + N * iy));
      const Real sc = MESH == MESH_AFFINE ? a.ops.scale[dir] : Real(1);
      if (id == N - 1) {
        const Real* fs = a.fstar + ((int64_t)dir * a.E + ee) * NV * NF;
        const Real w = sc * a.ops.inv_wp;
#pragma unroll
        for (int v = 0; v < NV; ++v) S[v] += w * fs[v * NF + f];
      }
      if (id == 0) {
        int64_t mx = ex, my = ey, mz = ez;
        if (dir == 0) mx = (ex + a.n0 - 1) % a.n0;
        if (dir == 1) my = (ey + a.n1 - 1) % a.n1;
        if (dir == 2) mz = (ez + a.n2 - 1) % a.n2;
        const int64_t em = mx + (int64_t)a.n0 * (my + (int64_t)a.n1 * mz);
        const Real* fs = a.fstar + ((int64_t)dir * a.E + em) * NV * NF;
        const Real w = sc * a.ops.inv_w0;
#pragma unroll
        for (int v = 0; v < NV; ++v) S[v] -= w * fs[v * NF + f];
      }
    }
    const Real mul = MESH == MESH_CURVED ? -a.metric[(ee * NM + DIM * DIM) * NN + i] : Real(-1);
    const int64_t base = ee * NV * NN + i;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const Real k = mul * S[v];
      const int64_t o = base + (int64_t)v * NN;
      if (a.mode == MODE_RHS) {
        a.out[o] = k;
      } else if (a.mode == MODE_RK_FIRST) {
        const Real u0 = a.uin[o];
        a.acc[o] = u0 + a.coef_b * (Real)dt * k;
        a.out[o] = u0 + a.coef_a * (Real)dt * k;
      } else if (a.mode == MODE_RK_MID) {
        a.acc[o] = a.acc[o] + a.coef_b * (Real)dt * k;
        a.out[o] = a.u0[o] + a.coef_a * (Real)dt * k;
      } else {
        a.out[o] = a.acc[o] + a.coef_b * (Real)dt * k;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// surface flux kernel (one thread per face node)
// ---------------------------------------------------------------------------

template <int DIM, typename Real>
__device__ __forceinline__ void cons_to_prim(const Real* u, Real gm1, Prim<Real>& P) {
  P.rho = u[0];
  const Real ir = Real(1) / P.rho;
  P.v0 = u[1] * ir;
  P.v1 = DIM > 1 ? u[2] * ir : Real(0);
  P.v2 = DIM > 2 ? u[3] * ir : Real(0);
  P.p = gm1 * (u[DIM + 1] - Real(0.5) * (u[1] * P.v0 + (DIM > 1 ? u[2] * P.v1 : Real(0)) +
                                          (DIM > 2 ? u[3] * P.v2 : Real(0))));
  P.lr = P.lp = Real(0);
}

template <int DIM, int SF, int MESH, typename Real>
__global__ void __launch_bounds__(256) face_kernel(FaceArgs<Real> a) {
  constexpr int NV = DIM + 2;
  const int N = a.N;
  const int NF = DIM == 3 ? N * N : N;
  const int NN = NF * N;
  const int64_t total = (int64_t)DIM * a.E * NF;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  const int dir = (int)(gid / (a.E * NF));
  const int64_t rem = gid - (int64_t)dir * a.E * NF;
  const int64_t e = rem / NF;
  const int f = (int)(rem - e * NF);
  // node indices of face node f on the + face (L) and - face (R)
  const int sa = dir == 0 ? 1 : (dir == 1 ? N : N * N);
  const int lo_part = f % sa, hi_part = f / sa;
  const int qL = lo_part + (N - 1) * sa + hi_part * sa * N;
  const int qR = lo_part + hi_part * sa * N;
  int64_t ex = e % a.n0, ey = (e / a.n0) % a.n1, ez = e / ((int64_t)a.n0 * a.n1);
  if (dir == 0) ex = (ex + 1) % a.n0;
  if (dir == 1) ey = (ey + 1) % a.n1;
  if (dir == 2) ez = (ez + 1) % a.n2;
  const int64_t eR = ex + (int64_t)a.n0 * (ey + (int64_t)a.n1 * ez);
  Real uL[NV], uR[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    uL[v] = a.u[(e * NV + v) * NN + qL];
    uR[v] = a.u[(eR * NV + v) * NN + qR];
  }
  Real nx, ny, nz;
  if (MESH == MESH_CURVED) {
    const Real* nf = a.nface + ((int64_t)dir * a.E + e) * DIM * NF + f;
    nx = nf[0];
    ny = DIM > 1 ? nf[NF] : Real(0);
    nz = DIM > 2 ? nf[2 * NF] : Real(0);
  } else {
    nx = dir == 0 ? Real(1) : Real(0);
    ny = dir == 1 ? Real(1) : Real(0);
    nz = dir == 2 ? Real(1) : Real(0);
  }
  const Real gm1 = a.gamma - Real(1);
  Prim<Real> PL, PR;
  cons_to_prim<DIM>(uL, gm1, PL);
  cons_to_prim<DIM>(uR, gm1, PR);
  Real F[NV];
  if (SF == SF_RANOCHA) {
    PL.lr = dev_log(PL.rho);
    PL.lp = dev_log(PL.p);
    PR.lr = dev_log(PR.rho);
    PR.lp = dev_log(PR.p);
    volume_flux<VF_RANOCHA, DIM>(PL, PR, nx, ny, nz, a.inv_gm1, F);
  } else if (SF == SF_SHIMA) {
    volume_flux<VF_SHIMA, DIM>(PL, PR, nx, ny, nz, a.inv_gm1, F);
  } else {
    volume_flux<VF_CENTRAL, DIM>(PL, PR, nx, ny, nz, a.inv_gm1, F);
    if (SF == SF_LLF) {
      const Real vnL = PL.v0 * nx + PL.v1 * ny + PL.v2 * nz;
      const Real vnR = PR.v0 * nx + PR.v1 * ny + PR.v2 * nz;
      const Real cL = sqrt(a.gamma * PL.p / PL.rho), cR = sqrt(a.gamma * PR.p / PR.rho);
      const Real nn = sqrt(nx * nx + ny * ny + nz * nz);
      const Real lam = fmax(fabs(vnL), fabs(vnR)) + fmax(cL, cR) * nn;
#pragma unroll
      for (int v = 0; v < NV; ++v) F[v] -= Real(0.5) * lam * (uR[v] - uL[v]);
    }
  }
  Real* out = a.fstar + ((int64_t)dir * a.E + e) * NV * NF + f;
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v * NF] = F[v];
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
        const double c = sqrt(a.gamma * p / rho);
        double lam = 0.0;
#pragma unroll
        for (int n = 0; n < DIM; ++n) {
          if (MESH == MESH_CURVED) {
            double vn = 0.0, an = 0.0;
#pragma unroll
            for (int m = 0; m < DIM; ++m) {
              const double jm = (double)a.metric[(e * NM + n * DIM + m) * nn + i];
              vn += vel[m] * jm;
              an += jm * jm;
            }
            lam += fabs(vn) + c * sqrt(an);
          } else {
            lam += (fabs(vel[n]) + c) * a.inv_half_h[n] * a.J_affine;
          }
        }
        lam /= J;
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
// RED_MAXLAMBDA it also turns lam_max into dt = cfl*2/(N lam_max), stores it
// in scal[0] and, if advance_t, adds it to scal[1].
template <int OP>
__global__ void __launch_bounds__(kRedThreads) reduce_final_kernel(const double* partial, int blocks, int K,
                                                                     double* out, double cfl, int N,
                                                                     double* scal, int advance_t) {
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
      if (OP == RED_MAXLAMBDA) {
        const double lam = sh[0];
        const double dt = cfl * 2.0 / ((double)N * lam);
        out[k] = dt;
        if (scal) {
          scal[0] = dt;
          if (advance_t) scal[1] += dt;
        }
      } else {
        out[k] = sh[0];
      }
    }
    __syncthreads();
  }
}

}  // namespace esdg
