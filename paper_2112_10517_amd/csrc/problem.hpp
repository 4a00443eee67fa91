// Internal state of a problem handle and the launch helpers shared by the
// single-problem entry points and the batch entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "esdg.h"
#include "dispatch.hpp"
#include "host_ops.hpp"
#include "kernels.hpp"

namespace esdg {

struct TimedLaunch {
  int kind;
  hipEvent_t start, stop;
};

}  // namespace esdg

struct esdg_problem {
  esdg::MeshSpec spec;
  esdg::Operators ops;
  esdg::Geometry geo;
  int dim = 3, p = 3, N = 4, nn = 64, nv = 5, nf = 16;
  int64_t E = 0;
  int vf = esdg::VF_RANOCHA, sf = esdg::SF_LLF, prec = esdg::PREC_FP64, mesh = esdg::MESH_AFFINE;
  int nodes = esdg::NODES_LGL;
  int integrator = ESDG_RK4;  // esdg_integrator of esdg_step
  double gamma = 1.4;
  hipStream_t stream = nullptr;
  int device = 0;
  size_t rsize = 8;  // bytes per internal real

  // device buffers (internal precision unless noted)
  void* U = nullptr;          // state
  void* Y = nullptr;          // RK stage state
  void* Y2 = nullptr;         // second RK stage state (stage inputs and outputs alternate)
  void* R = nullptr;          // RK accumulator
  void* DU = nullptr;         // right-hand side
  double* STAGE64 = nullptr;  // FP32 mode: FP64 staging of states crossing the ABI
  void* METRIC = nullptr;     // curved metrics
  void* NFACE = nullptr;      // curved face normals
  double* PARTIAL = nullptr;  // reduction partials (FP64)
  double* SCAL = nullptr;     // FP64 scalars: [0..1] time by step parity, [2..7] results
  unsigned long long* LAM = nullptr;  // CFL slots: 2 x kLamSlots by step parity (bit patterns of doubles)
  void* DESC = nullptr;               // ProbDesc<Real> of this problem (device)
  int* FLAG = nullptr;                // non-physical flag: device address of FLAG_H
  int* FLAG_H = nullptr;              // the flag in host-mapped pinned memory (kernels store 1)
  void* FACEB = nullptr;              // Gauss: entropy-projected face states
  void* FSTAR = nullptr;              // ESDG_FACES_ONCE: f* of every element's + faces [E][dim][nv][nf]
  int red_blocks = 1;
  int64_t red_per_block = 256;

  bool have_state = false;
  // step parity: the time and the CFL value of the current state live in
  // slot `par` of SCAL[0..1] and LAM; every step flips it.  The CFL value is
  // valid until the state changes other than through a CFL-mode step.
  int par = 0;
  bool lam_valid = false;
  bool timing = false;
  std::vector<esdg::TimedLaunch> launches;
  std::string err;
};

namespace esdg {

// Record an error message in *dst (if given) and in the calling thread's slot.
esdg_status report(std::string* dst, esdg_status st, const char* fmt, ...);
esdg_status fail(esdg_problem* P, esdg_status st, const char* fmt, ...);

#define ESDG_TRY(x)                   \
  do {                                \
    esdg_status s_ = (x);             \
    if (s_ != ESDG_OK) return s_;     \
  } while (0)

#define ESDG_HIP(errp, call)                                                                          \
  do {                                                                                                \
    hipError_t e_ = (call);                                                                           \
    if (e_ != hipSuccess)                                                                             \
      return ::esdg::report((errp), ESDG_EDEVICE, "%s: %s", #call, hipGetErrorString(e_));            \
  } while (0)

// Runs f, turning C++ exceptions into status codes so that none crosses the
// C ABI: host allocation failures become ESDG_ENOMEM, others ESDG_EDEVICE.
template <typename F>
esdg_status guarded(std::string* err, F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return report(err, ESDG_ENOMEM, "host memory exhausted");
  } catch (const std::exception& e) {
    return report(err, ESDG_EDEVICE, "%s", e.what());
  }
}

// Where and how a kernel is launched: stream, optional event bracketing, error slot.
struct Launcher {
  hipStream_t stream = nullptr;
  std::vector<TimedLaunch>* timed = nullptr;  // NULL: untimed
  std::string* err = nullptr;
};

inline Launcher launcher_of(esdg_problem* P) {
  Launcher L;
  L.stream = P->stream;
  L.timed = P->timing ? &P->launches : nullptr;
  L.err = &P->err;
  return L;
}

esdg_status launch_kernel(const Launcher& L, int kind, const void* fn, dim3 grid, dim3 block, void** args);

// Time stepping of one stage launch: fixed dt, or CFL from the lam slots.
struct StepCtl {
  double dt_fixed = 0.0, cfl = 0.0;
  int par = 0, lam_update = 0;
};

enum { BUF_U = 0, BUF_Y = 1, BUF_Y2 = 2, BUF_R = 3, BUF_DU = 4 };

inline unsigned long long* lam_slot(esdg_problem* P, int k) { return P->LAM + k * kLamSlots; }

// The non-physical flag of a problem lives in host-mapped pinned memory: a
// kernel that meets rho <= 0, p <= 0 or a non-finite state stores 1 into it,
// and the host reads it without waiting for the stream (a raised flag is
// seen once the kernel that stored it has run).  Only the host clears it.
inline bool flag_raised(const esdg_problem* P) { return __atomic_load_n(P->FLAG_H, __ATOMIC_ACQUIRE) != 0; }
inline void flag_clear(esdg_problem* P) { __atomic_store_n(P->FLAG_H, 0, __ATOMIC_RELEASE); }

// Tile variant of the stage kernel currently chosen for P's parameters
// (process-wide table, written by the autotuner) and its version counter.
int tile_variant_of(const esdg_problem* P);
int tile_table_version();
VolKernel pick_stage_kernel(const esdg_problem* P);
// stage kernel of tile variant v for P's parameters (fn == NULL if none) and
// the table update that makes v the variant in use for them
VolKernel kernel_of_variant(const esdg_problem* P, int v);
void set_tile_variant(const esdg_problem* P, int v);

template <typename Real>
StageOps<Real> stage_ops(const esdg_problem* P) {
  StageOps<Real> o{};
  for (int i = 0; i < P->N * P->N; ++i) o.Dt[i] = (Real)P->ops.Dt[i];
  o.inv_w0 = (Real)(1.0 / P->ops.w[0]);
  o.inv_wp = (Real)(1.0 / P->ops.w[P->N - 1]);
  o.gamma = (Real)P->gamma;
  o.inv_gm1 = (Real)(1.0 / (P->gamma - 1.0));
  for (int i = 0; i < P->N; ++i) {
    o.rL[i] = (Real)P->ops.rL[i];
    o.rR[i] = (Real)P->ops.rR[i];
    o.cL[i] = (Real)P->ops.cL[i];
    o.cR[i] = (Real)P->ops.cR[i];
    o.r64[0][i] = P->ops.rL[i];
    o.r64[1][i] = P->ops.rR[i];
  }
  return o;
}

// descriptor of problem P as the tile0-th tile of a launch
template <typename Real>
ProbDesc<Real> prob_desc(const esdg_problem* P, int tile0, double t_end) {
  ProbDesc<Real> d{};
  d.buf[BUF_U] = (Real*)P->U;
  d.buf[BUF_Y] = (Real*)P->Y;
  d.buf[BUF_Y2] = (Real*)P->Y2;
  d.buf[BUF_R] = (Real*)P->R;
  d.buf[BUF_DU] = (Real*)P->DU;
  d.metric = (const Real*)P->METRIC;
  d.nface = (const Real*)P->NFACE;
  d.lam = P->LAM;
  d.time = P->SCAL;
  d.flag = P->FLAG;
  d.faceb = (Real*)P->FACEB;
  d.t_end = t_end;
  d.E = (int)P->E;
  d.n0 = P->spec.n[0];
  d.n1 = P->spec.n[1];
  d.n2 = P->dim == 3 ? P->spec.n[2] : 1;
  d.tile0 = tile0;
  for (int j = 0; j < 3; ++j) d.scale[j] = (Real)(P->mesh == MESH_AFFINE ? P->geo.inv_half_h[j] : 1.0);
  return d;
}

// Whether a launch of `blocks` workgroups of kernel fn (`threads` lanes each)
// is one generation of more than one workgroup per compute unit on the
// current device: all resident at once, by the runtime's occupancy query
// (cached per device and kernel).  False if the query fails.
bool one_generation(const void* fn, int threads, int64_t blocks);

// Legendre-Gauss problems: the entropy-projection kernel that must precede
// every stage launch (same tiles and descriptors); fn == NULL for LGL
VolKernel pick_projection_kernel(const esdg_problem* P);

// One fused stage launch of kernel k over `tiles` tiles of the problems whose
// descriptors (device memory) are `probs`, all with the parameters of `rep`:
// right-hand side of buf[in_idx] (surface and volume terms) and, for the RK
// modes, the stage update into buf[out_idx] / R; RHS mode writes buf[out_idx]
// or out_ext.  Gauss problems first run the entropy projection of buf[in_idx];
// a problem in once-per-face mode stepped by itself first runs the face
// kernel on buf[in_idx] (batch launches evaluate faces in the stage kernel).

template <typename Real>
esdg_status run_stage_on(const esdg_problem* rep, const Launcher& L, const VolKernel& k, const void* probs,
                         const int* tile_prob, int64_t tiles, int in_idx, int out_idx, void* out_ext, int mode,
                         double coef_b, double coef_a, const StepCtl& ctl) {
  if (!k.fn) return report(L.err, ESDG_EINVAL, "no stage kernel for dim=%d p=%d flux=%d", rep->dim, rep->p, rep->vf);
  const VolKernel proj = pick_projection_kernel(rep);
  if (rep->nodes == NODES_GAUSS && (!proj.fn || proj.epb != k.epb))
    return report(L.err, ESDG_EINVAL, "no projection kernel for dim=%d p=%d", rep->dim, rep->p);
  StageArgs<Real> a{};
  a.probs = (const ProbDesc<Real>*)probs;
  a.tile_prob = tile_prob;
  a.out_ext = (Real*)out_ext;
  a.in_idx = in_idx;
  a.out_idx = out_idx;
  a.mode = mode;
  a.surf = rep->sf;
  a.coef_b = (Real)coef_b;
  a.coef_a = (Real)coef_a;
  a.dt_fixed = ctl.dt_fixed;
  a.cfl = ctl.cfl;
  a.gamma64 = rep->gamma;
  a.par = ctl.par;
  a.lam_update = ctl.lam_update;
  a.ops = stage_ops<Real>(rep);
  void* args[] = {&a};
  if (proj.fn) ESDG_TRY(launch_kernel(L, ESDG_KERNEL_PROJECT, proj.fn, dim3((unsigned)tiles), dim3(proj.threads), args));
  if (rep->FSTAR && probs == rep->DESC) {
    // once-per-face mode of a problem stepped by itself: the face kernel
    // writes f* of every face, the stage kernel reads it
    const void* fk = face_kernel_for(rep->prec, rep->dim, rep->N, rep->mesh);
    if (!fk || !k.faces_once)
      return report(L.err, ESDG_EINVAL,
                    "once-per-face mode needs a 3D node or pair tile, or a line tile up to p = 4 (dim=%d p=%d)",
                    rep->dim, rep->p);
    a.fstar = (Real*)rep->FSTAR;
    const int64_t lanes = rep->E * rep->dim * rep->nf;
    ESDG_TRY(launch_kernel(L, ESDG_KERNEL_FACE, fk, dim3((unsigned)((lanes + kFaceThreads - 1) / kFaceThreads)),
                           dim3(kFaceThreads), args));
  }
  const void* fn = k.fn_prio && one_generation(k.fn_prio, k.threads, tiles) ? k.fn_prio : k.fn;
  return launch_kernel(L, ESDG_KERNEL_STAGE, fn, dim3((unsigned)tiles), dim3(k.threads), args);
}

// FP64 reduction of op over P's state (and DU for the entropy rate) on L's
// stream; the result lands in SCAL[2..] (dt for RED_MAXLAMBDA, whose lam_max
// also goes to `slot` if given).
esdg_status run_reduce(esdg_problem* P, const Launcher& L, int op, double cfl, unsigned long long* slot);

// elementwise precision conversion of P's state-sized arrays on L's stream
esdg_status convert_state(esdg_problem* P, const Launcher& L, const void* src, void* dst, int to_fp64);

// copy slot `from` of P's time and CFL slots to slot 1 - from (L's stream)
esdg_status copy_parity(esdg_problem* P, const Launcher& L, int from);

inline size_t state_count(const esdg_problem* P) { return (size_t)P->E * P->nv * P->nn; }

// Coefficients of the five-stage, fourth-order 2N-storage scheme of Carpenter
// and Kennedy (1994): du <- A_i du + dt RHS(u), u <- u + B_i du, A_1 = 0.
constexpr int kCkStages = 5;
constexpr double kCkA[kCkStages] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                                    -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
constexpr double kCkB[kCkStages] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                                    1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                                    2277821191437.0 / 14882151754819.0};

// The stage launches of one step of P's integrator: (input buffer, output
// buffer, mode, coef_b, coef_a) in order; the last one writes BUF_U.
struct StagePlan {
  int in, out, mode;
  double b, a;
};
inline int step_plan(int integrator, StagePlan* s) {
  if (integrator == ESDG_CK45) {
    const int bufs[kCkStages + 1] = {BUF_U, BUF_Y, BUF_Y2, BUF_Y, BUF_Y2, BUF_U};
    for (int i = 0; i < kCkStages; ++i)
      s[i] = StagePlan{bufs[i], bufs[i + 1], i == 0 ? MODE_LS_FIRST : (i == kCkStages - 1 ? MODE_LS_LAST : MODE_LS_MID),
                       kCkB[i], kCkA[i]};
    return kCkStages;
  }
  // classical RK4 (a = 1/2, 1/2, 1; b = 1/6, 1/3, 1/3, 1/6) in low-storage form
  s[0] = StagePlan{BUF_U, BUF_Y, MODE_RK_FIRST, 1.0 / 6.0, 0.5};
  s[1] = StagePlan{BUF_Y, BUF_Y2, MODE_RK_MID, 1.0 / 3.0, 0.5};
  s[2] = StagePlan{BUF_Y2, BUF_Y, MODE_RK_MID, 1.0 / 3.0, 1.0};
  s[3] = StagePlan{BUF_Y, BUF_U, MODE_RK_LAST, 1.0 / 6.0, 0.0};
  return 4;
}

}  // namespace esdg
