// C ABI of the library (include/esdg.h): problem handles, device buffers,
// launch sequencing and error reporting.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "esdg.h"
#include "dispatch.hpp"
#include "host_ops.hpp"
#include "kernels.hpp"

using namespace esdg;

namespace {

thread_local std::string g_thread_error;

struct TimedLaunch {
  int kind;
  hipEvent_t start, stop;
};

}  // namespace

struct esdg_problem {
  MeshSpec spec;
  Operators ops;
  Geometry geo;
  int dim = 3, p = 3, N = 4, nn = 64, nv = 5, nf = 16;
  int64_t E = 0;
  int vf = VF_RANOCHA, sf = SF_LLF, prec = PREC_FP64, mesh = MESH_AFFINE;
  double gamma = 1.4;
  hipStream_t stream = nullptr;
  int device = 0;
  size_t rsize = 8;  // bytes per internal real

  // device buffers (internal precision unless noted)
  void* U = nullptr;       // state
  void* Y = nullptr;       // RK stage state
  void* R = nullptr;       // RK accumulator
  void* DU = nullptr;      // right-hand side scratch
  double* STAGE64 = nullptr;  // FP32 mode: FP64 staging of states crossing the ABI
  void* Y2 = nullptr;      // second RK stage state (stage inputs and outputs alternate)
  void* METRIC = nullptr;  // curved metrics
  void* NFACE = nullptr;   // curved face normals
  double* PARTIAL = nullptr;  // reduction partials (FP64)
  double* SCAL = nullptr;     // FP64 scalars: [1] t, [2..7] results
  unsigned long long* LAM = nullptr;  // CFL slots: 2 x kLamSlots (bit patterns of doubles)
  void* DESC = nullptr;               // ProbDesc<Real> of this problem (device)
  int* FLAG = nullptr;        // non-physical flag
  int red_blocks = 1;
  int64_t red_per_block = 256;

  bool have_state = false;
  // CFL: the largest wave-speed sum of the current state lives in one of two
  // device slots (bit pattern of a double); valid until the state changes
  // other than through esdg_step in CFL mode
  bool lam_valid = false;
  int lam_cur = 0;
  bool timing = false;
  std::vector<TimedLaunch> launches;
  std::string err;
};

namespace {

esdg_status fail(esdg_problem* P, esdg_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (P) P->err = buf;
  g_thread_error = buf;
  return st;
}

#define HIPCHECK(P, call)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return fail((P), ESDG_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

size_t state_count(const esdg_problem* P) { return (size_t)P->E * P->nv * P->nn; }

template <typename Real>
StageOps<Real> stage_ops(const esdg_problem* P) {
  StageOps<Real> o{};
  for (int i = 0; i < P->N * P->N; ++i) o.Dt[i] = (Real)P->ops.Dt[i];
  o.inv_w0 = (Real)(1.0 / P->ops.w[0]);
  o.inv_wp = (Real)(1.0 / P->ops.w[P->N - 1]);
  o.gamma = (Real)P->gamma;
  o.inv_gm1 = (Real)(1.0 / (P->gamma - 1.0));
  return o;
}

// descriptor of problem P as the first (tile0) tile of a launch
template <typename Real>
ProbDesc<Real> prob_desc(const esdg_problem* P, int tile0) {
  ProbDesc<Real> d{};
  d.buf[0] = (Real*)P->U;
  d.buf[1] = (Real*)P->Y;
  d.buf[2] = (Real*)P->Y2;
  d.buf[3] = (Real*)P->R;
  d.metric = (const Real*)P->METRIC;
  d.nface = (const Real*)P->NFACE;
  d.lam = P->LAM;
  d.t_acc = P->SCAL + 1;
  d.flag = P->FLAG;
  d.E = (int)P->E;
  d.n0 = P->spec.n[0];
  d.n1 = P->spec.n[1];
  d.n2 = P->dim == 3 ? P->spec.n[2] : 1;
  d.tile0 = tile0;
  for (int j = 0; j < 3; ++j) d.scale[j] = (Real)(P->mesh == MESH_AFFINE ? P->geo.inv_half_h[j] : 1.0);
  return d;
}

// launch with optional event bracketing for per-kernel timing
esdg_status launch(esdg_problem* P, int kind, const void* fn, dim3 grid, dim3 block, void** args) {
  if (!fn) return fail(P, ESDG_EINVAL, "no kernel instantiated for this configuration");
  TimedLaunch tl{kind, nullptr, nullptr};
  if (P->timing) {
    HIPCHECK(P, hipEventCreate(&tl.start));
    HIPCHECK(P, hipEventCreate(&tl.stop));
    HIPCHECK(P, hipEventRecord(tl.start, P->stream));
  }
  HIPCHECK(P, hipLaunchKernel(fn, grid, block, args, 0, P->stream));
  if (P->timing) {
    HIPCHECK(P, hipEventRecord(tl.stop, P->stream));
    P->launches.push_back(tl);
  }
  return ESDG_OK;
}

#define TRY(x)                        \
  do {                                \
    esdg_status s_ = (x);             \
    if (s_ != ESDG_OK) return s_;     \
  } while (0)

// One fused stage launch: right-hand side of `uin` (surface and volume
// terms) and, for the RK modes, the stage update into out / R.
unsigned long long* lam_slot(esdg_problem* P, int k) { return P->LAM + k * kLamSlots; }

// Time stepping of one stage launch: fixed dt, or CFL from the lam slots.
struct StepCtl {
  double dt_fixed = 0.0, cfl = 0.0;
  int lam_cur = 0, lam_update = 0, t_mode = 0;
};

enum { BUF_U = 0, BUF_Y = 1, BUF_Y2 = 2, BUF_R = 3 };

// the stage-kernel instantiation and tile size for P's parameters
VolKernel pick_stage_kernel(const esdg_problem* P) {
  return P->dim == 2 ? stage_kernel_2d(P->prec, P->N, P->vf, P->mesh) : stage_kernel_3d(P->prec, P->N, P->vf, P->mesh);
}

// One fused stage launch over the tiles of `nprob` problems sharing P's
// parameters (descriptors `probs` in device memory): right-hand side of
// buf[in_idx] (surface and volume terms) and, for the RK modes, the stage
// update into buf[out_idx] / R; RHS mode may write to out_ext instead.
template <typename Real>
esdg_status run_stage_on(esdg_problem* P, const void* probs, int nprob, int64_t tiles, int in_idx, int out_idx,
                         void* out_ext, int mode, double coef_b, double coef_a, const StepCtl& ctl) {
  StageArgs<Real> a{};
  a.probs = (const ProbDesc<Real>*)probs;
  a.nprob = nprob;
  a.out_ext = (Real*)out_ext;
  a.in_idx = in_idx;
  a.out_idx = out_idx;
  a.mode = mode;
  a.surf = P->sf;
  a.coef_b = (Real)coef_b;
  a.coef_a = (Real)coef_a;
  a.dt_fixed = ctl.dt_fixed;
  a.cfl = ctl.cfl;
  a.lam_cur = ctl.lam_cur;
  a.lam_update = ctl.lam_update;
  a.t_mode = ctl.t_mode;
  a.ops = stage_ops<Real>(P);
  VolKernel k = pick_stage_kernel(P);
  if (!k.fn) return fail(P, ESDG_EINVAL, "no stage kernel for dim=%d p=%d flux=%d", P->dim, P->p, P->vf);
  void* args[] = {&a};
  return launch(P, ESDG_KERNEL_STAGE, k.fn, dim3((unsigned)tiles), dim3(k.threads), args);
}

template <typename Real>
esdg_status run_stage(esdg_problem* P, int in_idx, int out_idx, void* out_ext, int mode, double coef_b,
                      double coef_a, const StepCtl& ctl = StepCtl()) {
  const VolKernel k = pick_stage_kernel(P);
  if (!k.fn) return fail(P, ESDG_EINVAL, "no stage kernel for dim=%d p=%d flux=%d", P->dim, P->p, P->vf);
  return run_stage_on<Real>(P, P->DESC, 1, (P->E + k.epb - 1) / k.epb, in_idx, out_idx, out_ext, mode, coef_b,
                            coef_a, ctl);
}

// FP64 reduction of op over the state (and DU for the entropy rate); the
// result lands in SCAL[2..] (dt for RED_MAXLAMBDA, whose lam_max also goes
// to `slot` if given).
template <typename Real>
esdg_status run_reduce(esdg_problem* P, int op, double cfl, unsigned long long* slot = nullptr) {
  RedArgs<Real> a{};
  a.u = (const Real*)P->U;
  a.du = (const Real*)P->DU;
  a.metric = (const Real*)P->METRIC;
  a.partial = P->PARTIAL;
  a.E = P->E;
  a.N = P->N;
  a.dim = P->dim;
  a.nn = P->nn;
  a.J_affine = P->geo.J_affine;
  for (int j = 0; j < 3; ++j) a.inv_half_h[j] = P->geo.inv_half_h[j];
  for (int i = 0; i < P->N; ++i) a.w[i] = P->ops.w[i];
  a.gamma = P->gamma;
  int64_t per_block = P->red_per_block;
  void* args[] = {&a, &per_block};
  TRY(launch(P, ESDG_KERNEL_REDUCE, reduce_partial_for(P->prec, P->dim, P->mesh, op), dim3(P->red_blocks),
             dim3(kRedThreads), args));
  int K = op == RED_TOTALS ? P->nv : 1;
  double* out = P->SCAL + 2;
  int blocks = P->red_blocks, N = P->N;
  void* args2[] = {&P->PARTIAL, &blocks, &K, &out, &cfl, &N, &slot};
  return launch(P, ESDG_KERNEL_REDUCE, reduce_final_for(op), dim3(1), dim3(kRedThreads), args2);
}

// dispatch on internal precision
#define BY_PREC(P, fn, ...) ((P)->prec == PREC_FP32 ? fn<float>(__VA_ARGS__) : fn<double>(__VA_ARGS__))

esdg_status rhs_into(esdg_problem* P, void* out) {
  return BY_PREC(P, run_stage, P, BUF_U, BUF_U, out, MODE_RHS, 0.0, 0.0);
}

// elementwise precision conversion of n values on the handle's stream
esdg_status convert(esdg_problem* P, const void* src, void* dst, int to_fp64) {
  int64_t n = (int64_t)state_count(P);
  void* args[] = {(void*)&src, &dst, &n};
  return launch(P, -1, convert_kernel_for(to_fp64), dim3((unsigned)((n + 255) / 256)), dim3(256), args);
}

esdg_status check_handle(esdg_problem* P, bool need_state) {
  if (!P) return fail(nullptr, ESDG_EINVAL, "NULL problem handle");
  if (need_state && !P->have_state) return fail(P, ESDG_ESTATE, "no state set (call esdg_set_state first)");
  HIPCHECK(P, hipSetDevice(P->device));
  return ESDG_OK;
}

esdg_status read_scalars(esdg_problem* P, int first, int count, double* out) {
  HIPCHECK(P, hipMemcpyAsync(out, P->SCAL + first, sizeof(double) * count, hipMemcpyDeviceToHost, P->stream));
  HIPCHECK(P, hipStreamSynchronize(P->stream));
  return ESDG_OK;
}

void free_buffers(esdg_problem* P) {
  void* bufs[] = {P->U, P->Y, P->Y2, P->R, P->DU, P->STAGE64, P->METRIC, P->NFACE, P->PARTIAL, P->SCAL, P->LAM, P->FLAG,
                  P->DESC};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  for (auto& t : P->launches) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  P->launches.clear();
}

}  // namespace

extern "C" {

const char* esdg_version(void) { return "esdg-mi355x 0.1 (gfx950)"; }

const char* esdg_last_error(const esdg_problem* prob) {
  return prob ? prob->err.c_str() : g_thread_error.c_str();
}

esdg_status esdg_operators(int32_t p, double* x, double* w, double* D, double* Dt) {
  Operators ops;
  std::string err;
  if (p > ESDG_PMAX || !make_operators(p, &ops, &err))
    return fail(nullptr, ESDG_EINVAL, "%s", err.empty() ? "p out of range" : err.c_str());
  const int N = p + 1;
  for (int i = 0; i < N; ++i) {
    if (x) x[i] = ops.x[i];
    if (w) w[i] = ops.w[i];
    for (int j = 0; j < N; ++j) {
      if (D) D[i * N + j] = ops.D[i * N + j];
      if (Dt) Dt[i * N + j] = ops.Dt[i * N + j];
    }
  }
  return ESDG_OK;
}

esdg_status esdg_init_mesh(const esdg_mesh_desc* d, esdg_problem** out) {
  if (!d || !out) return fail(nullptr, ESDG_EINVAL, "NULL descriptor or output pointer");
  *out = nullptr;
  if (d->dim != 2 && d->dim != 3) return fail(nullptr, ESDG_EINVAL, "dim must be 2 or 3");
  if (d->p < 1 || d->p > ESDG_PMAX) return fail(nullptr, ESDG_EINVAL, "p must be in [1, %d]", ESDG_PMAX);
  if (!(d->gamma > 1.0)) return fail(nullptr, ESDG_EINVAL, "gamma must be > 1");
  if (d->volume_flux != ESDG_FLUX_RANOCHA && d->volume_flux != ESDG_FLUX_SHIMA &&
      d->volume_flux != ESDG_FLUX_CENTRAL)
    return fail(nullptr, ESDG_EINVAL, "volume flux must be RANOCHA, SHIMA or CENTRAL");
  if (d->surface_flux < 0 || d->surface_flux > 3) return fail(nullptr, ESDG_EINVAL, "unknown surface flux");
  if (d->precision != ESDG_FP64 && d->precision != ESDG_FP32)
    return fail(nullptr, ESDG_EINVAL, "unknown precision");
  int64_t ne = 1;
  for (int j = 0; j < d->dim; ++j) {
    if (d->n[j] < 1) return fail(nullptr, ESDG_EINVAL, "element counts must be >= 1");
    ne *= d->n[j];
  }
  if (ne > (int64_t)1 << 30) return fail(nullptr, ESDG_EINVAL, "at most 2^30 elements");

  esdg_problem* P = new esdg_problem();
  P->spec.dim = d->dim;
  P->spec.p = d->p;
  for (int j = 0; j < 3; ++j) {
    P->spec.n[j] = (j < d->dim) ? d->n[j] : 1;
    P->spec.lo[j] = d->lo[j];
    P->spec.hi[j] = d->hi[j];
  }
  P->spec.warp = d->warp;
  P->spec.coords = d->coords;
  P->dim = d->dim;
  P->p = d->p;
  P->N = d->p + 1;
  P->nv = d->dim + 2;
  P->vf = d->volume_flux;
  P->sf = d->surface_flux;
  P->prec = d->precision == ESDG_FP32 ? PREC_FP32 : PREC_FP64;
  P->rsize = P->prec == PREC_FP32 ? 4 : 8;
  P->gamma = d->gamma;
  P->stream = (hipStream_t)d->stream;
  std::string err;
  if (!make_operators(d->p, &P->ops, &err) || !make_geometry(P->spec, P->ops, &P->geo, &err)) {
    esdg_status st = fail(nullptr, ESDG_EINVAL, "%s", err.c_str());
    delete P;
    return st;
  }
  P->spec.coords = nullptr;  // never retained
  P->E = P->geo.E;
  P->nn = P->geo.nn;
  P->nf = P->geo.nf;
  P->mesh = P->geo.affine ? MESH_AFFINE : MESH_CURVED;

  hipError_t he = hipGetDevice(&P->device);
  if (he != hipSuccess) {
    esdg_status st = fail(nullptr, ESDG_EDEVICE, "hipGetDevice: %s", hipGetErrorString(he));
    delete P;
    return st;
  }
  // reduction geometry: fixed per problem size, so results are reproducible
  const int64_t total = P->E * P->nn;
  int64_t blocks = (total + kRedThreads - 1) / kRedThreads;
  if (blocks > 2048) blocks = 2048;
  P->red_blocks = (int)blocks;
  P->red_per_block = ((total + blocks - 1) / blocks + kRedThreads - 1) / kRedThreads * kRedThreads;

  const size_t ns = state_count(P) * P->rsize;
  struct {
    void** ptr;
    size_t bytes;
  } allocs[] = {{&P->U, ns},
                {&P->Y, ns},
                {&P->R, ns},
                {&P->DU, ns},
                {&P->Y2, ns},
                {(void**)&P->PARTIAL, sizeof(double) * 8 * (size_t)P->red_blocks},
                {(void**)&P->SCAL, sizeof(double) * 16},
                {(void**)&P->LAM, sizeof(unsigned long long) * 2 * kLamSlots},
                {(void**)&P->FLAG, sizeof(int)}};
  for (auto& a : allocs) {
    if (hipMalloc(a.ptr, a.bytes) != hipSuccess) {
      free_buffers(P);
      delete P;
      return fail(nullptr, ESDG_ENOMEM, "device allocation of %zu bytes failed", a.bytes);
    }
  }
  if (P->prec == PREC_FP32 && hipMalloc((void**)&P->STAGE64, state_count(P) * sizeof(double)) != hipSuccess) {
    free_buffers(P);
    delete P;
    return fail(nullptr, ESDG_ENOMEM, "device allocation of the FP64 staging buffer failed");
  }
  if (P->mesh == MESH_CURVED && P->prec == PREC_FP32) {
    // FP32 bulk: the metric terms are rounded once, on the host
    std::vector<float> mf(P->geo.metric.begin(), P->geo.metric.end());
    std::vector<float> nf(P->geo.nface.begin(), P->geo.nface.end());
    if (hipMalloc(&P->METRIC, mf.size() * 4) != hipSuccess || hipMalloc(&P->NFACE, nf.size() * 4) != hipSuccess) {
      free_buffers(P);
      delete P;
      return fail(nullptr, ESDG_ENOMEM, "device allocation of metric terms failed");
    }
    if (hipMemcpy(P->METRIC, mf.data(), mf.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(P->NFACE, nf.data(), nf.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      free_buffers(P);
      delete P;
      return fail(nullptr, ESDG_EDEVICE, "upload of metric terms failed");
    }
    std::vector<double>().swap(P->geo.metric);
    std::vector<double>().swap(P->geo.nface);
  } else if (P->mesh == MESH_CURVED) {
    const size_t mb = P->geo.metric.size() * P->rsize, fb = P->geo.nface.size() * P->rsize;
    if (hipMalloc(&P->METRIC, mb) != hipSuccess || hipMalloc(&P->NFACE, fb) != hipSuccess) {
      free_buffers(P);
      delete P;
      return fail(nullptr, ESDG_ENOMEM, "device allocation of metric terms failed");
    }
    hipError_t e1 = hipMemcpy(P->METRIC, P->geo.metric.data(), mb, hipMemcpyHostToDevice);
    hipError_t e2 = hipMemcpy(P->NFACE, P->geo.nface.data(), fb, hipMemcpyHostToDevice);
    if (e1 != hipSuccess || e2 != hipSuccess) {
      free_buffers(P);
      delete P;
      return fail(nullptr, ESDG_EDEVICE, "upload of metric terms failed");
    }
    // the device copy is authoritative; keep the host copy small
    std::vector<double>().swap(P->geo.metric);
    std::vector<double>().swap(P->geo.nface);
  }
  {
    const size_t db = P->prec == PREC_FP32 ? sizeof(ProbDesc<float>) : sizeof(ProbDesc<double>);
    hipError_t e1 = hipMalloc(&P->DESC, db);
    hipError_t e2 = hipErrorOutOfMemory;
    if (e1 == hipSuccess) {
      if (P->prec == PREC_FP32) {
        ProbDesc<float> d = prob_desc<float>(P, 0);
        e2 = hipMemcpy(P->DESC, &d, db, hipMemcpyHostToDevice);
      } else {
        ProbDesc<double> d = prob_desc<double>(P, 0);
        e2 = hipMemcpy(P->DESC, &d, db, hipMemcpyHostToDevice);
      }
    }
    if (e1 != hipSuccess || e2 != hipSuccess) {
      free_buffers(P);
      delete P;
      return fail(nullptr, ESDG_ENOMEM, "device problem descriptor failed");
    }
  }
  if (hipMemset(P->FLAG, 0, sizeof(int)) != hipSuccess || hipMemset(P->SCAL, 0, sizeof(double) * 16) != hipSuccess) {
    free_buffers(P);
    delete P;
    return fail(nullptr, ESDG_EDEVICE, "device initialisation failed");
  }
  *out = P;
  return ESDG_OK;
}

void esdg_destroy(esdg_problem* P) {
  if (!P) return;
  (void)hipSetDevice(P->device);
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  else (void)hipDeviceSynchronize();
  free_buffers(P);
  delete P;
}

esdg_status esdg_sizes(const esdg_problem* P, int64_t* n_elem, int32_t* nodes, int32_t* n_var) {
  if (!P) return fail(nullptr, ESDG_EINVAL, "NULL problem handle");
  if (n_elem) *n_elem = P->E;
  if (nodes) *nodes = P->nn;
  if (n_var) *n_var = P->nv;
  return ESDG_OK;
}

esdg_status esdg_set_stream(esdg_problem* P, void* stream) {
  if (!P) return fail(nullptr, ESDG_EINVAL, "NULL problem handle");
  P->stream = (hipStream_t)stream;
  return ESDG_OK;
}

esdg_status esdg_get_coords(const esdg_problem* P, double* x) {
  if (!P || !x) return fail(const_cast<esdg_problem*>(P), ESDG_EINVAL, "NULL argument");
  std::memcpy(x, P->geo.coords.data(), sizeof(double) * P->geo.coords.size());
  return ESDG_OK;
}

esdg_status esdg_set_state(esdg_problem* P, const double* u, int32_t where) {
  TRY(check_handle(P, false));
  if (!u) return fail(P, ESDG_EINVAL, "NULL state");
  const size_t bytes = state_count(P) * sizeof(double);
  if (P->prec == PREC_FP32) {
    const void* src = u;
    if (where != ESDG_DEVICE) {
      HIPCHECK(P, hipMemcpyAsync(P->STAGE64, u, bytes, hipMemcpyHostToDevice, P->stream));
      src = P->STAGE64;
    }
    TRY(convert(P, src, P->U, 0));
  } else {
    HIPCHECK(P, hipMemcpyAsync(P->U, u, bytes, where == ESDG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                               P->stream));
  }
  if (where != ESDG_DEVICE) HIPCHECK(P, hipStreamSynchronize(P->stream));
  P->have_state = true;
  P->lam_valid = false;
  return ESDG_OK;
}

esdg_status esdg_get_state(esdg_problem* P, double* u, int32_t where) {
  TRY(check_handle(P, true));
  if (!u) return fail(P, ESDG_EINVAL, "NULL output");
  const size_t bytes = state_count(P) * sizeof(double);
  if (P->prec == PREC_FP32) {
    TRY(convert(P, P->U, where == ESDG_DEVICE ? (void*)u : (void*)P->STAGE64, 1));
    if (where != ESDG_DEVICE) HIPCHECK(P, hipMemcpyAsync(u, P->STAGE64, bytes, hipMemcpyDeviceToHost, P->stream));
  } else {
    HIPCHECK(P, hipMemcpyAsync(u, P->U, bytes, where == ESDG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                               P->stream));
  }
  if (where != ESDG_DEVICE) HIPCHECK(P, hipStreamSynchronize(P->stream));
  return ESDG_OK;
}

esdg_status esdg_rhs(esdg_problem* P, double* du, int32_t where) {
  TRY(check_handle(P, true));
  if (!du) return fail(P, ESDG_EINVAL, "NULL output");
  const bool direct = where == ESDG_DEVICE;
  const size_t bytes = state_count(P) * sizeof(double);
  if (P->prec == PREC_FP32) {
    TRY(rhs_into(P, P->DU));
    TRY(convert(P, P->DU, direct ? (void*)du : (void*)P->STAGE64, 1));
    if (!direct) HIPCHECK(P, hipMemcpyAsync(du, P->STAGE64, bytes, hipMemcpyDeviceToHost, P->stream));
  } else {
    TRY(rhs_into(P, direct ? (void*)du : P->DU));
    if (!direct) HIPCHECK(P, hipMemcpyAsync(du, P->DU, bytes, hipMemcpyDeviceToHost, P->stream));
  }
  if (!direct) HIPCHECK(P, hipStreamSynchronize(P->stream));
  return ESDG_OK;
}

esdg_status esdg_step(esdg_problem* P, double dt, int32_t nsteps, double cfl, double* t_inout) {
  TRY(check_handle(P, true));
  if (nsteps < 0) return fail(P, ESDG_EINVAL, "nsteps must be >= 0");
  const bool use_cfl = !(dt > 0.0);
  if (use_cfl && !(cfl > 0.0)) return fail(P, ESDG_EINVAL, "dt <= 0 needs cfl > 0");
  if (nsteps == 0) return ESDG_OK;
  // classical RK4 in low-storage form: U (state), R (accumulator) and the
  // stage state, alternating between Y and Y2 (stage inputs are read across
  // element faces, so a stage never writes its own input)
  StepCtl ctl;
  if (!use_cfl) {
    ctl.dt_fixed = dt;
  } else {
    ctl.cfl = cfl;
    // the CFL value of the start state comes from the previous CFL step's
    // last stage; otherwise from one reduction
    if (!P->lam_valid) TRY(BY_PREC(P, run_reduce, P, RED_MAXLAMBDA, cfl, lam_slot(P, P->lam_cur)));
  }
  for (int s = 0; s < nsteps; ++s) {
    ctl.lam_cur = P->lam_cur;
    StepCtl first = ctl, last = ctl;
    first.t_mode = use_cfl ? (s == 0 ? 2 : 1) : 0;
    last.lam_update = use_cfl ? 1 : 0;
    TRY(BY_PREC(P, run_stage, P, BUF_U, BUF_Y, nullptr, MODE_RK_FIRST, 1.0 / 6.0, 0.5, first));
    TRY(BY_PREC(P, run_stage, P, BUF_Y, BUF_Y2, nullptr, MODE_RK_MID, 1.0 / 3.0, 0.5, ctl));
    TRY(BY_PREC(P, run_stage, P, BUF_Y2, BUF_Y, nullptr, MODE_RK_MID, 1.0 / 3.0, 1.0, ctl));
    TRY(BY_PREC(P, run_stage, P, BUF_Y, BUF_U, nullptr, MODE_RK_LAST, 1.0 / 6.0, 0.0, last));
    if (use_cfl) P->lam_cur = 1 - P->lam_cur;
  }
  P->lam_valid = use_cfl;
  if (t_inout) {
    if (use_cfl) {
      double tsum = 0.0;
      TRY(read_scalars(P, 1, 1, &tsum));
      *t_inout += tsum;
    } else {
      *t_inout += dt * nsteps;
    }
  }
  return ESDG_OK;
}

esdg_status esdg_entropy_rate(esdg_problem* P, double* dSdt) {
  TRY(check_handle(P, true));
  if (!dSdt) return fail(P, ESDG_EINVAL, "NULL output");
  TRY(rhs_into(P, P->DU));
  TRY(BY_PREC(P, run_reduce, P, RED_ENTROPY, 0.0));
  return read_scalars(P, 2, 1, dSdt);
}

esdg_status esdg_totals(esdg_problem* P, double* totals) {
  TRY(check_handle(P, true));
  if (!totals) return fail(P, ESDG_EINVAL, "NULL output");
  TRY(BY_PREC(P, run_reduce, P, RED_TOTALS, 0.0));
  return read_scalars(P, 2, P->nv, totals);
}

esdg_status esdg_max_dt(esdg_problem* P, double cfl, double* dt) {
  TRY(check_handle(P, true));
  if (!dt || !(cfl > 0.0)) return fail(P, ESDG_EINVAL, "need cfl > 0 and an output pointer");
  TRY(BY_PREC(P, run_reduce, P, RED_MAXLAMBDA, cfl));
  return read_scalars(P, 2, 1, dt);
}

esdg_status esdg_sync(esdg_problem* P) {
  TRY(check_handle(P, false));
  HIPCHECK(P, hipStreamSynchronize(P->stream));
  int flag = 0;
  HIPCHECK(P, hipMemcpy(&flag, P->FLAG, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) {
    HIPCHECK(P, hipMemset(P->FLAG, 0, sizeof(int)));
    return fail(P, ESDG_ENONPHYSICAL, "non-physical state (rho <= 0, p <= 0 or non-finite) met by a kernel");
  }
  return ESDG_OK;
}

esdg_status esdg_timing_enable(esdg_problem* P, int32_t enable) {
  if (!P) return fail(nullptr, ESDG_EINVAL, "NULL problem handle");
  P->timing = enable != 0;
  return ESDG_OK;
}

esdg_status esdg_timing_read(esdg_problem* P, int32_t kernel, double* total_ms, int64_t* launches) {
  TRY(check_handle(P, false));
  double sum = 0.0;
  int64_t cnt = 0;
  for (auto& t : P->launches) {
    if (t.kind != kernel) continue;
    HIPCHECK(P, hipEventSynchronize(t.stop));
    float ms = 0.0f;
    HIPCHECK(P, hipEventElapsedTime(&ms, t.start, t.stop));
    sum += ms;
    ++cnt;
  }
  if (total_ms) *total_ms = sum;
  if (launches) *launches = cnt;
  return ESDG_OK;
}

esdg_status esdg_timing_reset(esdg_problem* P) {
  TRY(check_handle(P, false));
  HIPCHECK(P, hipStreamSynchronize(P->stream));
  for (auto& t : P->launches) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  P->launches.clear();
  return ESDG_OK;
}

}  // extern "C"
