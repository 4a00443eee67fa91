// C ABI of the library (include/esdg.h): problem handles, device buffers,
// launch sequencing, the tile-variant autotuner and error reporting.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <new>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "problem.hpp"

using namespace esdg;

namespace {

thread_local std::string g_thread_error;

}  // namespace

namespace esdg {

esdg_status report(std::string* dst, esdg_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (dst) *dst = buf;
  g_thread_error = buf;
  return st;
}

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

esdg_status launch_kernel(const Launcher& L, int kind, const void* fn, dim3 grid, dim3 block, void** args) {
  if (!fn) return report(L.err, ESDG_EINVAL, "no kernel instantiated for this configuration");
  TimedLaunch tl{kind, nullptr, nullptr};
  if (L.timed) {
    ESDG_HIP(L.err, hipEventCreate(&tl.start));
    ESDG_HIP(L.err, hipEventCreate(&tl.stop));
    ESDG_HIP(L.err, hipEventRecord(tl.start, L.stream));
  }
  ESDG_HIP(L.err, hipLaunchKernel(fn, grid, block, args, 0, L.stream));
  if (L.timed) {
    ESDG_HIP(L.err, hipEventRecord(tl.stop, L.stream));
    try {
      L.timed->push_back(tl);
    } catch (const std::bad_alloc&) {
      (void)hipEventDestroy(tl.start);
      (void)hipEventDestroy(tl.stop);
      return report(L.err, ESDG_ENOMEM, "host memory exhausted (timing record)");
    }
  }
  return ESDG_OK;
}

// ---- tile-variant table (autotuner results), keyed by the kernel parameters
namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int, int>, int> g_tune;
int g_tune_version = 0;

std::tuple<int, int, int, int, int, int> tune_key(const esdg_problem* P) {
  return std::make_tuple(P->dim, P->N, P->vf, P->mesh, P->prec, P->nodes);
}
}  // namespace

// Variant used until the table holds one for the parameters (3D LGL; the
// measured winners per degree, precision and mesh kind, launches of 3-5 M
// nodes): the line layout (0) up to p = 3, where the kernel is bound by
// memory and the line's single pass over its pairs wins; the node layout (3)
// at p = 4; at p = 5 the pair layout (4) in FP64 and on affine FP32 meshes,
// the node layout on curved FP32 meshes; the pair layout at p = 6 (on curved
// FP64 meshes its one-z-plane-per-wave form) and p = 7.
static int default_tile_variant(const esdg_problem* P) {
  if (P->dim != 3 || P->nodes != NODES_LGL || P->N < 5) return 0;
  const bool fp64 = P->prec == PREC_FP64, curved = P->mesh == MESH_CURVED;
  if (P->N == 5) return 3;
  if (P->N == 6) return (!fp64 && curved) ? 3 : 4;
  return 4;
}

int tile_variant_of(const esdg_problem* P) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune.find(tune_key(P));
  return it == g_tune.end() ? default_tile_variant(P) : it->second;
}

int tile_table_version() {
  std::lock_guard<std::mutex> g(g_tune_mu);
  return g_tune_version;
}

void set_tile_variant(const esdg_problem* P, int v) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune.find(tune_key(P));
  const int cur = it == g_tune.end() ? default_tile_variant(P) : it->second;
  if (cur != v) ++g_tune_version;
  g_tune[tune_key(P)] = v;
}

// stage kernel of tile variant v for P (Gauss collocation has variant 0 only)
VolKernel kernel_of_variant(const esdg_problem* P, int v) {
  if (P->nodes == NODES_GAUSS) return v == 0 ? gauss_kernel_for(P->prec, P->dim, P->N, P->vf, false) : VolKernel{};
  return stage_kernel_for(P->prec, P->dim, P->N, P->vf, P->mesh, v);
}

VolKernel pick_stage_kernel(const esdg_problem* P) {
  return kernel_of_variant(P, P->nodes == NODES_GAUSS ? 0 : tile_variant_of(P));
}

bool one_generation(const void* fn, int threads, int64_t blocks) {
  static std::mutex mu;
  // (device, kernel) -> (compute units, workgroups resident at once)
  static std::map<std::pair<int, const void*>, std::pair<int64_t, int64_t>> sizes;
  int dev = 0;
  if (!fn || hipGetDevice(&dev) != hipSuccess) return false;
  try {
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_pair(dev, fn);
    auto it = sizes.find(key);
    if (it == sizes.end()) {
      int per_cu = 0, cus = 0;
      std::pair<int64_t, int64_t> v(0, 0);
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0) == hipSuccess &&
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
        v = std::make_pair((int64_t)cus, (int64_t)per_cu * cus);
      it = sizes.emplace(key, v).first;
    }
    return blocks > it->second.first && blocks <= it->second.second;
  } catch (...) {
    return false;
  }
}

VolKernel pick_projection_kernel(const esdg_problem* P) {
  if (P->nodes != NODES_GAUSS) return VolKernel{};
  return gauss_kernel_for(P->prec, P->dim, P->N, P->vf, true);
}

// partial: blocks x K doubles of block sums; out: the K results (both on the
// device).  The handle's buffers unless the caller brings others.
template <typename Real>
static esdg_status reduce_t(esdg_problem* P, const Launcher& L, int op, double cfl, unsigned long long* slot,
                            double* partial, double* out) {
  RedArgs<Real> a{};
  a.u = (const Real*)P->U;
  a.du = (const Real*)P->DU;
  a.metric = (const Real*)P->METRIC;
  a.partial = partial;
  a.E = P->E;
  a.N = P->N;
  a.dim = P->dim;
  a.nn = P->nn;
  a.J_affine = P->geo.J_affine;
  for (int j = 0; j < 3; ++j) a.inv_half_h[j] = P->geo.inv_half_h[j];
  for (int i = 0; i < P->N; ++i) a.w[i] = P->ops.w[i];
  a.gamma = P->gamma;
  for (int j = 0; j < 3; ++j) a.scale[j] = (Real)(P->mesh == MESH_AFFINE ? P->geo.inv_half_h[j] : 1.0);
  int64_t per_block = P->red_per_block;
  void* args[] = {&a, &per_block};
  ESDG_TRY(launch_kernel(L, ESDG_KERNEL_REDUCE, reduce_partial_for(P->prec, P->dim, P->mesh, op),
                         dim3(P->red_blocks), dim3(kRedThreads), args));
  int K = op == RED_TOTALS ? P->nv : 1;
  int blocks = P->red_blocks, N = P->N;
  void* args2[] = {&partial, &blocks, &K, &out, &cfl, &N, &slot};
  return launch_kernel(L, ESDG_KERNEL_REDUCE, reduce_final_for(op), dim3(1), dim3(kRedThreads), args2);
}

esdg_status run_reduce_into(esdg_problem* P, const Launcher& L, int op, double cfl, unsigned long long* slot,
                            double* partial, double* out) {
  return P->prec == PREC_FP32 ? reduce_t<float>(P, L, op, cfl, slot, partial, out)
                              : reduce_t<double>(P, L, op, cfl, slot, partial, out);
}

esdg_status run_reduce(esdg_problem* P, const Launcher& L, int op, double cfl, unsigned long long* slot) {
  return run_reduce_into(P, L, op, cfl, slot, P->PARTIAL, P->SCAL + 2);
}

esdg_status convert_state(esdg_problem* P, const Launcher& L, const void* src, void* dst, int to_fp64) {
  int64_t n = (int64_t)state_count(P);
  void* args[] = {(void*)&src, &dst, &n};
  return launch_kernel(L, -1, convert_kernel_for(to_fp64), dim3((unsigned)((n + 255) / 256)), dim3(256), args);
}

namespace {

__global__ void __launch_bounds__(64) copy_parity_kernel(double* time, unsigned long long* lam, int from) {
  const int t = threadIdx.x;
  lam[(1 - from) * kLamSlots + t] = lam[from * kLamSlots + t];
  if (t == 0) time[1 - from] = time[from];
}

__global__ void __launch_bounds__(64) set_scalar_kernel(double* dst, double v) {
  if (threadIdx.x == 0) dst[0] = v;
}

}  // namespace

esdg_status copy_parity(esdg_problem* P, const Launcher& L, int from) {
  double* t = P->SCAL;
  unsigned long long* lam = P->LAM;
  void* args[] = {&t, &lam, &from};
  return launch_kernel(L, -1, (const void*)&copy_parity_kernel, dim3(1), dim3(kLamSlots), args);
}

}  // namespace esdg

namespace {

// dispatch on internal precision
#define BY_PREC(P, fn, ...) ((P)->prec == PREC_FP32 ? fn<float>(__VA_ARGS__) : fn<double>(__VA_ARGS__))

template <typename Real>
esdg_status run_stage(esdg_problem* P, int in_idx, int out_idx, void* out_ext, int mode, double coef_b,
                      double coef_a, const StepCtl& ctl = StepCtl()) {
  const VolKernel k = pick_stage_kernel(P);
  return run_stage_on<Real>(P, launcher_of(P), k, P->DESC, nullptr, (P->E + k.epb - 1) / std::max(1, k.epb), in_idx,
                            out_idx, out_ext, mode, coef_b, coef_a, ctl);
}

esdg_status rhs_into(esdg_problem* P, void* out) {
  return BY_PREC(P, run_stage, P, BUF_U, BUF_DU, out, MODE_RHS, 0.0, 0.0);
}

esdg_status convert(esdg_problem* P, const void* src, void* dst, int to_fp64) {
  return convert_state(P, launcher_of(P), src, dst, to_fp64);
}

esdg_status check_handle(esdg_problem* P, bool need_state) {
  if (!P) return fail(nullptr, ESDG_EINVAL, "NULL problem handle");
  if (need_state && !P->have_state) return fail(P, ESDG_ESTATE, "no state set (call esdg_set_state first)");
  ESDG_HIP(&P->err, hipSetDevice(P->device));
  return ESDG_OK;
}

esdg_status read_scalars(esdg_problem* P, int first, int count, double* out) {
  ESDG_HIP(&P->err, hipMemcpyAsync(out, P->SCAL + first, sizeof(double) * count, hipMemcpyDeviceToHost, P->stream));
  ESDG_HIP(&P->err, hipStreamSynchronize(P->stream));
  return ESDG_OK;
}

// ESDG_ENONPHYSICAL (and the flag cleared) if a kernel has raised P's
// non-physical flag; no wait for the stream
esdg_status report_flag(esdg_problem* P) {
  if (!flag_raised(P)) return ESDG_OK;
  flag_clear(P);
  return fail(P, ESDG_ENONPHYSICAL, "non-physical state (rho <= 0, p <= 0 or non-finite) met by a kernel");
}

esdg_status set_time(esdg_problem* P, double t) {
  double* dst = P->SCAL + P->par;
  void* args[] = {&dst, &t};
  return launch_kernel(launcher_of(P), -1, (const void*)&set_scalar_kernel, dim3(1), dim3(64), args);
}

void free_buffers(esdg_problem* P) {
  void* bufs[] = {P->U,     P->Y,       P->Y2,   P->R,   P->DU,   P->STAGE64, P->METRIC,
                  P->NFACE, P->PARTIAL, P->SCAL, P->LAM, P->DESC, P->FACEB, P->FSTAR};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (P->FLAG_H) (void)hipHostFree(P->FLAG_H);
  for (auto& t : P->launches) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  P->launches.clear();
}

}  // namespace

// ---- allocation-free totals: the reduction's block partial sums live in a
// file-scope device array instead of the handle's buffer.  In host code
// `scratch` names a host-side stand-in, never the device memory: the
// device address comes from hipGetSymbolAddress, once per device, with that
// device current, and only that address is passed to kernels.
constexpr int kScratchDoubles = 2048 * 8;  // <= 2048 reduction blocks x (dim + 2) sums: 128 KiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on first use)
esdg_status scratch_address(esdg_problem* P, double** out) {
  if (P->device < 0 || P->device >= kMaxDevices) return fail(P, ESDG_EINVAL, "device index %d out of range", P->device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[P->device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(P, ESDG_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", P->device, hipGetErrorString(e));
    g_scratch_ptr[P->device] = (double*)ptr;
  }
  *out = g_scratch_ptr[P->device];
  return ESDG_OK;
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

// validation of a mesh descriptor shared by esdg_init_mesh and esdg_footprint
static esdg_status check_desc(const esdg_mesh_desc* d) {
  if (d->dim != 2 && d->dim != 3) return fail(nullptr, ESDG_EINVAL, "dim must be 2 or 3");
  if (d->p < 1 || d->p > ESDG_PMAX) return fail(nullptr, ESDG_EINVAL, "p must be in [1, %d]", ESDG_PMAX);
  if (!(d->gamma > 1.0)) return fail(nullptr, ESDG_EINVAL, "gamma must be > 1");
  if (d->volume_flux != ESDG_FLUX_RANOCHA && d->volume_flux != ESDG_FLUX_SHIMA &&
      d->volume_flux != ESDG_FLUX_CENTRAL)
    return fail(nullptr, ESDG_EINVAL, "volume flux must be RANOCHA, SHIMA or CENTRAL");
  if (d->surface_flux < 0 || d->surface_flux > 3) return fail(nullptr, ESDG_EINVAL, "unknown surface flux");
  if (d->precision != ESDG_FP64 && d->precision != ESDG_FP32)
    return fail(nullptr, ESDG_EINVAL, "unknown precision");
  if (d->nodes != ESDG_NODES_LGL && d->nodes != ESDG_NODES_GAUSS) return fail(nullptr, ESDG_EINVAL, "unknown node kind");
  if (d->nodes == ESDG_NODES_GAUSS && (d->warp != 0.0 || d->coords))
    return fail(nullptr, ESDG_EINVAL, "Gauss collocation is available on affine meshes only (warp 0, no coords)");
  int64_t ne = 1;
  for (int j = 0; j < d->dim; ++j) {
    if (d->n[j] < 1) return fail(nullptr, ESDG_EINVAL, "element counts must be >= 1");
    ne *= d->n[j];
  }
  if (ne > (int64_t)1 << 30) return fail(nullptr, ESDG_EINVAL, "at most 2^30 elements");
  return ESDG_OK;
}

// reduction geometry: fixed per problem size, so results are reproducible
static void reduction_blocks(int64_t total, int* blocks_out, int64_t* per_block) {
  int64_t blocks = (total + kRedThreads - 1) / kRedThreads;
  if (blocks > 2048) blocks = 2048;
  *blocks_out = (int)blocks;
  *per_block = ((total + blocks - 1) / blocks + kRedThreads - 1) / kRedThreads * kRedThreads;
}

esdg_status esdg_footprint(const esdg_mesh_desc* d, int64_t* bytes) {
  if (!d || !bytes) return fail(nullptr, ESDG_EINVAL, "NULL descriptor or output pointer");
  ESDG_TRY(check_desc(d));
  int64_t E = 1, nn = 1, nf = 1;
  for (int j = 0; j < d->dim; ++j) {
    E *= d->n[j];
    nn *= d->p + 1;
  }
  nf = nn / (d->p + 1);
  const int64_t rs = d->precision == ESDG_FP32 ? 4 : 8;
  const int64_t ns = E * (d->dim + 2) * nn;
  int64_t b = 5 * ns * rs;
  if (d->precision == ESDG_FP32) b += ns * 8;
  if (d->warp != 0.0 || d->coords) b += (E * (d->dim * d->dim + 1) * nn + (int64_t)d->dim * E * d->dim * nf) * rs;
  if (d->nodes == ESDG_NODES_GAUSS) b += E * 2 * d->dim * (d->dim + 4) * nf * rs;
  int blocks;
  int64_t per;
  reduction_blocks(E * nn, &blocks, &per);
  b += 8 * 8 * (int64_t)blocks + 16 * 8 + 2 * kLamSlots * 8 + (int64_t)sizeof(ProbDesc<double>);
  *bytes = b;
  return ESDG_OK;
}

static esdg_status init_mesh_impl(const esdg_mesh_desc* d, esdg_problem** out) {
  ESDG_TRY(check_desc(d));
  // optional device budget (bytes) for every problem: a problem whose
  // footprint exceeds it fails with ESDG_ENOMEM before any allocation
  if (const char* env = std::getenv("ESDG_DEVICE_BUDGET")) {
    int64_t need = 0;
    ESDG_TRY(esdg_footprint(d, &need));
    const long long budget = std::atoll(env);
    if (budget > 0 && need > budget)
      return fail(nullptr, ESDG_ENOMEM, "problem needs %lld device bytes, ESDG_DEVICE_BUDGET is %lld",
                  (long long)need, budget);
  }

  // owned until the handle is complete: every early return (and exception)
  // releases what was allocated so far
  struct Owner {
    esdg_problem* P = new esdg_problem();
    ~Owner() {
      if (P) {
        free_buffers(P);
        delete P;
      }
    }
  } own;
  esdg_problem* P = own.P;
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
  P->nodes = d->nodes == ESDG_NODES_GAUSS ? NODES_GAUSS : NODES_LGL;
  std::string err;
  const bool ops_ok =
      P->nodes == NODES_GAUSS ? make_gauss_operators(d->p, &P->ops, &err) : make_operators(d->p, &P->ops, &err);
  if (!ops_ok || !make_geometry(P->spec, P->ops, &P->geo, &err)) {
    return fail(nullptr, ESDG_EINVAL, "%s", err.c_str());
  }
  P->spec.coords = nullptr;  // never retained
  P->E = P->geo.E;
  P->nn = P->geo.nn;
  P->nf = P->geo.nf;
  P->mesh = P->geo.affine ? MESH_AFFINE : MESH_CURVED;

  hipError_t he = hipGetDevice(&P->device);
  if (he != hipSuccess) {
    return fail(nullptr, ESDG_EDEVICE, "hipGetDevice: %s", hipGetErrorString(he));
  }
  reduction_blocks(P->E * P->nn, &P->red_blocks, &P->red_per_block);

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
                {(void**)&P->LAM, sizeof(unsigned long long) * 2 * kLamSlots}};
  for (auto& a : allocs) {
    if (hipMalloc(a.ptr, a.bytes) != hipSuccess) {
      return fail(nullptr, ESDG_ENOMEM, "device allocation of %zu bytes failed", a.bytes);
    }
  }
  if (hipHostMalloc((void**)&P->FLAG_H, sizeof(int), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer((void**)&P->FLAG, P->FLAG_H, 0) != hipSuccess) {
    return fail(nullptr, ESDG_ENOMEM, "pinned host allocation of the non-physical flag failed");
  }
  flag_clear(P);
  if (P->nodes == NODES_GAUSS &&
      hipMalloc(&P->FACEB, (size_t)P->E * 2 * P->dim * (P->dim + 4) * P->nf * P->rsize) != hipSuccess) {
    return fail(nullptr, ESDG_ENOMEM, "device allocation of the face states failed");
  }
  if (P->prec == PREC_FP32 && hipMalloc((void**)&P->STAGE64, state_count(P) * sizeof(double)) != hipSuccess) {
    return fail(nullptr, ESDG_ENOMEM, "device allocation of the FP64 staging buffer failed");
  }
  if (P->mesh == MESH_CURVED && P->prec == PREC_FP32) {
    // FP32 bulk: the metric terms are rounded once, on the host
    std::vector<float> mf(P->geo.metric.begin(), P->geo.metric.end());
    std::vector<float> nf(P->geo.nface.begin(), P->geo.nface.end());
    if (hipMalloc(&P->METRIC, mf.size() * 4) != hipSuccess || hipMalloc(&P->NFACE, nf.size() * 4) != hipSuccess) {
      return fail(nullptr, ESDG_ENOMEM, "device allocation of metric terms failed");
    }
    if (hipMemcpyAsync(P->METRIC, mf.data(), mf.size() * 4, hipMemcpyHostToDevice, P->stream) != hipSuccess ||
        hipMemcpyAsync(P->NFACE, nf.data(), nf.size() * 4, hipMemcpyHostToDevice, P->stream) != hipSuccess ||
        hipStreamSynchronize(P->stream) != hipSuccess) {
      return fail(nullptr, ESDG_EDEVICE, "upload of metric terms failed");
    }
    std::vector<double>().swap(P->geo.metric);
    std::vector<double>().swap(P->geo.nface);
  } else if (P->mesh == MESH_CURVED) {
    const size_t mb = P->geo.metric.size() * P->rsize, fb = P->geo.nface.size() * P->rsize;
    if (hipMalloc(&P->METRIC, mb) != hipSuccess || hipMalloc(&P->NFACE, fb) != hipSuccess) {
      return fail(nullptr, ESDG_ENOMEM, "device allocation of metric terms failed");
    }
    hipError_t e1 = hipMemcpyAsync(P->METRIC, P->geo.metric.data(), mb, hipMemcpyHostToDevice, P->stream);
    hipError_t e2 = hipMemcpyAsync(P->NFACE, P->geo.nface.data(), fb, hipMemcpyHostToDevice, P->stream);
    if (e1 == hipSuccess && e2 == hipSuccess) e1 = hipStreamSynchronize(P->stream);
    if (e1 != hipSuccess || e2 != hipSuccess) {
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
        ProbDesc<float> d = prob_desc<float>(P, 0, INFINITY);
        e2 = hipMemcpyAsync(P->DESC, &d, db, hipMemcpyHostToDevice, P->stream);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(P->stream);
      } else {
        ProbDesc<double> d = prob_desc<double>(P, 0, INFINITY);
        e2 = hipMemcpyAsync(P->DESC, &d, db, hipMemcpyHostToDevice, P->stream);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(P->stream);
      }
    }
    if (e1 != hipSuccess || e2 != hipSuccess) {
      return fail(nullptr, ESDG_ENOMEM, "device problem descriptor failed");
    }
  }
  // cleared on the handle's stream (which need not be ordered with the null stream)
  if (hipMemsetAsync(P->SCAL, 0, sizeof(double) * 16, P->stream) != hipSuccess ||
      hipStreamSynchronize(P->stream) != hipSuccess) {
    return fail(nullptr, ESDG_EDEVICE, "device initialisation failed");
  }
  own.P = nullptr;
  *out = P;
  return ESDG_OK;
}

esdg_status esdg_init_mesh(const esdg_mesh_desc* d, esdg_problem** out) {
  if (!d || !out) return fail(nullptr, ESDG_EINVAL, "NULL descriptor or output pointer");
  *out = nullptr;
  try {
    return init_mesh_impl(d, out);
  } catch (const std::bad_alloc&) {
    return fail(nullptr, ESDG_ENOMEM, "host memory exhausted while building the problem");
  } catch (const std::exception& e) {
    return fail(nullptr, ESDG_EDEVICE, "%s", e.what());
  }
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

static esdg_status get_inv_jacobian_impl(esdg_problem* P, double* inv_j) {
  ESDG_TRY(check_handle(P, false));
  if (!inv_j) return fail(P, ESDG_EINVAL, "NULL argument");
  const size_t count = (size_t)P->E * P->nn;
  if (P->mesh != MESH_CURVED) {
    for (size_t i = 0; i < count; ++i) inv_j[i] = 1.0 / P->geo.J_affine;
    return ESDG_OK;
  }
  // the 1/J row of every element inside the device metric array
  // [E][dim*dim + 1][nn]: one strided copy of E rows of nn values
  const size_t row = (size_t)P->nn * P->rsize, pitch = (size_t)(P->dim * P->dim + 1) * row;
  const char* src = (const char*)P->METRIC + (size_t)P->dim * P->dim * row;
  if (P->rsize == sizeof(double)) {
    ESDG_HIP(&P->err, hipMemcpy2DAsync(inv_j, row, src, pitch, row, (size_t)P->E, hipMemcpyDeviceToHost, P->stream));
    ESDG_HIP(&P->err, hipStreamSynchronize(P->stream));
  } else {
    std::vector<float> f(count);
    ESDG_HIP(&P->err, hipMemcpy2DAsync(f.data(), row, src, pitch, row, (size_t)P->E, hipMemcpyDeviceToHost, P->stream));
    ESDG_HIP(&P->err, hipStreamSynchronize(P->stream));
    for (size_t i = 0; i < count; ++i) inv_j[i] = f[i];
  }
  return ESDG_OK;
}

esdg_status esdg_get_inv_jacobian(esdg_problem* P, double* inv_j) {
  // the FP32 path stages the values in a host vector: no exception crosses the ABI
  return guarded(P ? &P->err : nullptr, [&] { return get_inv_jacobian_impl(P, inv_j); });
}

esdg_status esdg_set_state(esdg_problem* P, const double* u, int32_t where) {
  ESDG_TRY(check_handle(P, false));
  if (!u) return fail(P, ESDG_EINVAL, "NULL state");
  const size_t bytes = state_count(P) * sizeof(double);
  if (P->prec == PREC_FP32) {
    const void* src = u;
    if (where != ESDG_DEVICE) {
      ESDG_HIP(&P->err, hipMemcpyAsync(P->STAGE64, u, bytes, hipMemcpyHostToDevice, P->stream));
      src = P->STAGE64;
    }
    ESDG_TRY(convert(P, src, P->U, 0));
  } else {
    ESDG_HIP(&P->err, hipMemcpyAsync(P->U, u, bytes, where == ESDG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                               P->stream));
  }
  if (where != ESDG_DEVICE) ESDG_HIP(&P->err, hipStreamSynchronize(P->stream));
  P->have_state = true;
  P->lam_valid = false;
  return ESDG_OK;
}

esdg_status esdg_get_state(esdg_problem* P, double* u, int32_t where) {
  ESDG_TRY(check_handle(P, true));
  if (!u) return fail(P, ESDG_EINVAL, "NULL output");
  const size_t bytes = state_count(P) * sizeof(double);
  if (P->prec == PREC_FP32) {
    ESDG_TRY(convert(P, P->U, where == ESDG_DEVICE ? (void*)u : (void*)P->STAGE64, 1));
    if (where != ESDG_DEVICE) ESDG_HIP(&P->err, hipMemcpyAsync(u, P->STAGE64, bytes, hipMemcpyDeviceToHost, P->stream));
  } else {
    ESDG_HIP(&P->err, hipMemcpyAsync(u, P->U, bytes, where == ESDG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                               P->stream));
  }
  if (where != ESDG_DEVICE) ESDG_HIP(&P->err, hipStreamSynchronize(P->stream));
  return ESDG_OK;
}

esdg_status esdg_rhs(esdg_problem* P, double* du, int32_t where) {
  ESDG_TRY(check_handle(P, true));
  if (!du) return fail(P, ESDG_EINVAL, "NULL output");
  const bool direct = where == ESDG_DEVICE;
  const size_t bytes = state_count(P) * sizeof(double);
  if (P->prec == PREC_FP32) {
    ESDG_TRY(rhs_into(P, P->DU));
    ESDG_TRY(convert(P, P->DU, direct ? (void*)du : (void*)P->STAGE64, 1));
    if (!direct) ESDG_HIP(&P->err, hipMemcpyAsync(du, P->STAGE64, bytes, hipMemcpyDeviceToHost, P->stream));
  } else {
    ESDG_TRY(rhs_into(P, direct ? (void*)du : P->DU));
    if (!direct) ESDG_HIP(&P->err, hipMemcpyAsync(du, P->DU, bytes, hipMemcpyDeviceToHost, P->stream));
  }
  if (!direct) ESDG_HIP(&P->err, hipStreamSynchronize(P->stream));
  return ESDG_OK;
}

esdg_status esdg_step(esdg_problem* P, double dt, int32_t nsteps, double cfl, double* t_inout) {
  ESDG_TRY(check_handle(P, true));
  if (nsteps < 0) return fail(P, ESDG_EINVAL, "nsteps must be >= 0");
  const bool use_cfl = !(dt > 0.0);
  if (use_cfl && !(cfl > 0.0)) return fail(P, ESDG_EINVAL, "dt <= 0 needs cfl > 0");
  // a state an earlier kernel found non-physical is not stepped
  ESDG_TRY(report_flag(P));
  if (t_inout) ESDG_TRY(set_time(P, *t_inout));
  if (nsteps > 0) {
    // classical RK4 in low-storage form (U state, R accumulator) or the 2N
    // scheme (R holds du); stage states alternate between Y and Y2 (stage
    // inputs are read across element faces, so a stage never writes its own
    // input)
    StepCtl ctl;
    if (!use_cfl) {
      ctl.dt_fixed = dt;
    } else {
      ctl.cfl = cfl;
      // the CFL value of the start state comes from the previous CFL step's
      // last stage; otherwise from one reduction
      if (!P->lam_valid) ESDG_TRY(run_reduce(P, launcher_of(P), RED_MAXLAMBDA, cfl, lam_slot(P, P->par)));
    }
    StagePlan plan[kCkStages];
    const int nst = step_plan(P->integrator, plan);
    for (int s = 0; s < nsteps; ++s) {
      ctl.par = P->par;
      StepCtl last = ctl;
      last.lam_update = use_cfl ? 1 : 0;
      for (int i = 0; i < nst; ++i)
        ESDG_TRY(BY_PREC(P, run_stage, P, plan[i].in, plan[i].out, nullptr, plan[i].mode, plan[i].b, plan[i].a,
                         i == nst - 1 ? last : ctl));
      P->par = 1 - P->par;
    }
    P->lam_valid = use_cfl;
  }
  if (t_inout) {
    ESDG_TRY(read_scalars(P, P->par, 1, t_inout));  // synchronises: this call's kernels have run
    ESDG_TRY(report_flag(P));
  }
  return ESDG_OK;
}

esdg_status esdg_set_integrator(esdg_problem* P, int32_t integrator) {
  if (!P) return fail(nullptr, ESDG_EINVAL, "NULL problem handle");
  if (integrator != ESDG_RK4 && integrator != ESDG_CK45) return fail(P, ESDG_EINVAL, "unknown integrator %d", integrator);
  P->integrator = integrator;
  return ESDG_OK;
}

esdg_status esdg_get_integrator(const esdg_problem* P, int32_t* integrator) {
  if (!P || !integrator) return fail(const_cast<esdg_problem*>(P), ESDG_EINVAL, "NULL argument");
  *integrator = P->integrator;
  return ESDG_OK;
}

esdg_status esdg_set_time(esdg_problem* P, double t) {
  ESDG_TRY(check_handle(P, false));
  return set_time(P, t);
}

esdg_status esdg_get_time(esdg_problem* P, double* t) {
  ESDG_TRY(check_handle(P, false));
  if (!t) return fail(P, ESDG_EINVAL, "NULL output");
  return read_scalars(P, P->par, 1, t);
}

esdg_status esdg_entropy_rate(esdg_problem* P, double* dSdt) {
  ESDG_TRY(check_handle(P, true));
  if (!dSdt) return fail(P, ESDG_EINVAL, "NULL output");
  ESDG_TRY(rhs_into(P, P->DU));
  ESDG_TRY(run_reduce(P, launcher_of(P), RED_ENTROPY, 0.0, nullptr));
  ESDG_TRY(read_scalars(P, 2, 1, dSdt));
  return report_flag(P);
}

esdg_status esdg_totals(esdg_problem* P, double* totals) {
  ESDG_TRY(check_handle(P, true));
  if (!totals) return fail(P, ESDG_EINVAL, "NULL output");
  ESDG_TRY(run_reduce(P, launcher_of(P), RED_TOTALS, 0.0, nullptr));
  ESDG_TRY(read_scalars(P, 2, P->nv, totals));
  return report_flag(P);
}

esdg_status esdg_totals_noalloc(esdg_problem* P, double* totals_dev) {
  ESDG_TRY(check_handle(P, true));
  if (!totals_dev) return fail(P, ESDG_EINVAL, "NULL output");
  const int64_t need = (int64_t)P->red_blocks * P->nv;
  if (need > kScratchDoubles)
    return fail(P, ESDG_EINVAL, "reduction needs %lld partial sums, above the static scratch of %d doubles",
                (long long)need, kScratchDoubles);
  double* partial = nullptr;
  ESDG_TRY(scratch_address(P, &partial));
  // untimed launcher: the timing records allocate host objects
  Launcher L;
  L.stream = P->stream;
  L.err = &P->err;
  // every block writes its K partials before the final pass reads them: no clearing needed
  ESDG_TRY(run_reduce_into(P, L, RED_TOTALS, 0.0, nullptr, partial, totals_dev));
  return report_flag(P);
}

esdg_status esdg_max_dt(esdg_problem* P, double cfl, double* dt) {
  ESDG_TRY(check_handle(P, true));
  if (!dt || !(cfl > 0.0)) return fail(P, ESDG_EINVAL, "need cfl > 0 and an output pointer");
  ESDG_TRY(run_reduce(P, launcher_of(P), RED_MAXLAMBDA, cfl, nullptr));
  ESDG_TRY(read_scalars(P, 2, 1, dt));
  return report_flag(P);
}

esdg_status esdg_sync(esdg_problem* P) {
  ESDG_TRY(check_handle(P, false));
  ESDG_HIP(&P->err, hipStreamSynchronize(P->stream));
  return report_flag(P);
}

esdg_status esdg_get_tile_variant(const esdg_problem* P, int32_t* variant, int32_t* elems_per_block) {
  if (!P) return fail(nullptr, ESDG_EINVAL, "NULL problem handle");
  const int v = tile_variant_of(P);
  if (variant) *variant = v;
  if (elems_per_block) *elems_per_block = pick_stage_kernel(P).epb;
  return ESDG_OK;
}

esdg_status esdg_set_tile_variant(esdg_problem* P, int32_t variant) {
  if (!P) return fail(nullptr, ESDG_EINVAL, "NULL problem handle");
  const VolKernel k = kernel_of_variant(P, variant);
  if (!k.fn) return fail(P, ESDG_EINVAL, "tile variant %d does not exist for dim=%d p=%d", variant, P->dim, P->p);
  if (P->FSTAR && !k.faces_once)
    return fail(P, ESDG_EINVAL, "tile variant %d has no once-per-face build at p=%d", variant, P->p);
  set_tile_variant(P, variant);
  return ESDG_OK;
}

esdg_status esdg_set_face_flux_mode(esdg_problem* P, int32_t mode) {
  ESDG_TRY(check_handle(P, false));
  if (mode != ESDG_FACES_FUSED && mode != ESDG_FACES_ONCE) return fail(P, ESDG_EINVAL, "unknown face flux mode %d", mode);
  if (mode == ESDG_FACES_ONCE && P->nodes != NODES_LGL)
    return fail(P, ESDG_EINVAL, "Legendre-Gauss problems evaluate their face fluxes per element only");
  if (mode == ESDG_FACES_ONCE && (P->dim != 3 || !pick_stage_kernel(P).faces_once))
    return fail(P, ESDG_EINVAL,
                "once-per-face mode needs a 3D problem whose tile variant is a node or pair tile, or a line tile "
                "up to p = 4 (dim=%d p=%d)", P->dim, P->p);
  if (mode == ESDG_FACES_ONCE && !P->FSTAR) {
    const size_t bytes = (size_t)P->E * P->dim * P->nv * P->nf * P->rsize;
    if (hipMalloc(&P->FSTAR, bytes) != hipSuccess) {
      P->FSTAR = nullptr;
      return fail(P, ESDG_ENOMEM, "device allocation of %zu bytes for the face fluxes failed", bytes);
    }
  }
  if (mode == ESDG_FACES_FUSED && P->FSTAR) {
    ESDG_HIP(&P->err, hipStreamSynchronize(P->stream));  // no launch in flight still reads it
    ESDG_HIP(&P->err, hipFree(P->FSTAR));
    P->FSTAR = nullptr;
  }
  return ESDG_OK;
}

esdg_status esdg_get_face_flux_mode(const esdg_problem* P, int32_t* mode) {
  if (!P || !mode) return fail(nullptr, ESDG_EINVAL, "NULL argument");
  *mode = P->FSTAR ? ESDG_FACES_ONCE : ESDG_FACES_FUSED;
  return ESDG_OK;
}

esdg_status esdg_autotune(esdg_problem* P, int32_t reps, int32_t* best, double* us_per_variant) {
  ESDG_TRY(check_handle(P, true));
  if (reps < 1) return fail(P, ESDG_EINVAL, "reps must be >= 1");
  // every variant computes the right-hand side of the current state into DU
  // (the state is not modified); variants that resolve to the same kernel
  // share one measurement
  double us[ESDG_TILE_VARIANTS];
  int epb[ESDG_TILE_VARIANTS];
  const void* fns[ESDG_TILE_VARIANTS];
  int pick = -1;
  Launcher L = launcher_of(P);
  L.timed = nullptr;
  hipEvent_t e0, e1;
  ESDG_HIP(&P->err, hipEventCreate(&e0));
  ESDG_HIP(&P->err, hipEventCreate(&e1));
  esdg_status st = ESDG_OK;
  for (int v = 0; v < ESDG_TILE_VARIANTS && st == ESDG_OK; ++v) {
    us[v] = -1.0;
    epb[v] = 0;
    fns[v] = nullptr;
    const VolKernel k = kernel_of_variant(P, v);
    if (!k.fn || (P->FSTAR && !k.faces_once)) continue;
    epb[v] = k.epb;
    fns[v] = k.fn;
    int same = -1;
    for (int w = 0; w < v; ++w)
      if (fns[w] == k.fn) same = w;
    if (same >= 0) {
      us[v] = us[same];
      continue;
    }
    const int64_t tiles = (P->E + k.epb - 1) / k.epb;
    auto one = [&]() {
      return P->prec == PREC_FP32
                 ? run_stage_on<float>(P, L, k, P->DESC, nullptr, tiles, BUF_U, BUF_DU, nullptr, MODE_RHS, 0, 0, StepCtl())
                 : run_stage_on<double>(P, L, k, P->DESC, nullptr, tiles, BUF_U, BUF_DU, nullptr, MODE_RHS, 0, 0,
                                        StepCtl());
    };
    for (int r = 0; r < 2 && st == ESDG_OK; ++r) st = one();
    if (st != ESDG_OK) break;
    if (hipEventRecord(e0, P->stream) != hipSuccess) st = fail(P, ESDG_EDEVICE, "hipEventRecord failed");
    for (int r = 0; r < reps && st == ESDG_OK; ++r) st = one();
    if (st != ESDG_OK) break;
    float ms = 0.0f;
    if (hipEventRecord(e1, P->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = fail(P, ESDG_EDEVICE, "event timing failed");
      break;
    }
    us[v] = 1000.0 * ms / reps;
    if (pick < 0 || us[v] < us[pick]) pick = v;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ESDG_TRY(st);
  if (pick < 0) return fail(P, ESDG_EINVAL, "no stage kernel for dim=%d p=%d", P->dim, P->p);
  set_tile_variant(P, pick);
  if (best) *best = pick;
  if (us_per_variant)
    for (int v = 0; v < ESDG_TILE_VARIANTS; ++v) us_per_variant[v] = us[v];
  return ESDG_OK;
}

esdg_status esdg_timing_enable(esdg_problem* P, int32_t enable) {
  if (!P) return fail(nullptr, ESDG_EINVAL, "NULL problem handle");
  P->timing = enable != 0;
  return ESDG_OK;
}

esdg_status esdg_timing_read(esdg_problem* P, int32_t kernel, double* total_ms, int64_t* launches) {
  ESDG_TRY(check_handle(P, false));
  double sum = 0.0;
  int64_t cnt = 0;
  for (auto& t : P->launches) {
    if (t.kind != kernel) continue;
    ESDG_HIP(&P->err, hipEventSynchronize(t.stop));
    float ms = 0.0f;
    ESDG_HIP(&P->err, hipEventElapsedTime(&ms, t.start, t.stop));
    sum += ms;
    ++cnt;
  }
  if (total_ms) *total_ms = sum;
  if (launches) *launches = cnt;
  return ESDG_OK;
}

esdg_status esdg_timing_reset(esdg_problem* P) {
  ESDG_TRY(check_handle(P, false));
  ESDG_HIP(&P->err, hipStreamSynchronize(P->stream));
  for (auto& t : P->launches) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  P->launches.clear();
  return ESDG_OK;
}

}  // extern "C"
