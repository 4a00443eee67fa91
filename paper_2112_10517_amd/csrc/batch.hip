// Batches (include/esdg.h): several problems advanced by one launch per
// group of equal kernel parameters and RK stage, eagerly or as replayed HIP
// graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <tuple>
#include <vector>

#include "problem.hpp"

using namespace esdg;

namespace {

// problems sharing one stage-kernel instantiation and one StageOps
struct BatchGroup {
  esdg_problem* rep = nullptr;
  std::vector<int> members;  // indices into esdg_batch::probs
  VolKernel k;
  int64_t tiles = 0;
  void* desc = nullptr;       // device ProbDesc<Real>[members]
  int* tile_prob = nullptr;   // device: member index (within the group) of every tile
  int integrator = ESDG_RK4;  // of every member, recorded when the batch is created
};

struct GraphEntry {
  bool cfl = false;
  double dt = 0.0, cfl_v = 0.0;
  int par = 0;
  hipGraphExec_t exec = nullptr;
};

// member i's time (slot par of its time slots), gathered by one kernel
__global__ void __launch_bounds__(256) gather_times_kernel(double* const* times, int par, int count, double* t_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  t_out[i] = times[i][par];
}

}  // namespace

struct esdg_batch {
  std::vector<esdg_problem*> probs;
  std::vector<double> t_end;
  std::vector<BatchGroup> groups;
  int device = 0;
  int flags = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<hipStream_t> aux;     // concurrent groups
  std::vector<hipEvent_t> join;     // one per aux stream
  hipEvent_t fork = nullptr, done = nullptr;
  std::vector<hipStream_t> mstreams;  // distinct member streams other than `stream`
  std::vector<hipEvent_t> mevents;
  int par = 0;        // step parity of every member at the start of the next step
  int version = -1;   // tile-variant table version the groups were built for
  std::vector<GraphEntry> graphs;
  double** time_ptrs = nullptr;  // device: SCAL of every member
  double* t_out = nullptr;       // device [count]
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> step_events;
  std::string err;
};

namespace {

esdg_status bfail(esdg_batch* b, esdg_status st, const char* msg) { return report(b ? &b->err : nullptr, st, "%s", msg); }

Launcher launcher_on(esdg_batch* b, hipStream_t s) {
  Launcher L;
  L.stream = s;
  L.timed = nullptr;
  L.err = &b->err;
  return L;
}

void free_groups(esdg_batch* b) {
  for (auto& g : b->groups) {
    if (g.desc) (void)hipFree(g.desc);
    if (g.tile_prob) (void)hipFree(g.tile_prob);
    g.desc = nullptr;
    g.tile_prob = nullptr;
  }
}

void drop_graphs(esdg_batch* b) {
  for (auto& e : b->graphs)
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
  b->graphs.clear();
}

template <typename Real>
esdg_status upload_group(esdg_batch* b, BatchGroup& g) {
  std::vector<ProbDesc<Real>> descs;
  std::vector<int> owner;
  int64_t tile0 = 0;
  for (size_t j = 0; j < g.members.size(); ++j) {
    esdg_problem* P = b->probs[g.members[j]];
    descs.push_back(prob_desc<Real>(P, (int)tile0, b->t_end[g.members[j]]));
    const int64_t t = (P->E + g.k.epb - 1) / g.k.epb;
    owner.insert(owner.end(), (size_t)t, (int)j);
    tile0 += t;
  }
  if (tile0 > ((int64_t)1 << 31) - 1) return bfail(b, ESDG_EINVAL, "a group of the batch has more than 2^31-1 tiles");
  g.tiles = tile0;
  ESDG_HIP(&b->err, hipMalloc(&g.desc, sizeof(ProbDesc<Real>) * descs.size()));
  ESDG_HIP(&b->err, hipMalloc((void**)&g.tile_prob, sizeof(int) * owner.size()));
  // on the batch stream (the members' streams need not be ordered with the null stream)
  ESDG_HIP(&b->err, hipMemcpyAsync(g.desc, descs.data(), sizeof(ProbDesc<Real>) * descs.size(), hipMemcpyHostToDevice,
                                   b->stream));
  ESDG_HIP(&b->err,
           hipMemcpyAsync(g.tile_prob, owner.data(), sizeof(int) * owner.size(), hipMemcpyHostToDevice, b->stream));
  ESDG_HIP(&b->err, hipStreamSynchronize(b->stream));
  return ESDG_OK;
}

// (re)build the per-group descriptor arrays for the current tile variants
esdg_status refresh_groups(esdg_batch* b) {
  const int ver = tile_table_version();
  if (ver == b->version && !b->groups.empty()) return ESDG_OK;
  ESDG_HIP(&b->err, hipStreamSynchronize(b->stream));  // descriptors in use by queued work
  drop_graphs(b);
  free_groups(b);
  for (auto& g : b->groups) {
    g.k = pick_stage_kernel(g.rep);
    if (!g.k.fn) return report(&b->err, ESDG_EINVAL, "no stage kernel for dim=%d p=%d", g.rep->dim, g.rep->p);
    ESDG_TRY(g.rep->prec == PREC_FP32 ? upload_group<float>(b, g) : upload_group<double>(b, g));
  }
  b->version = ver;
  return ESDG_OK;
}

// the launches of one RK step of every group (eager, or being captured)
template <typename Real>
esdg_status group_step(esdg_batch* b, BatchGroup& g, hipStream_t s, const StepCtl& ctl) {
  const Launcher L = launcher_on(b, s);
  StepCtl last = ctl;
  last.lam_update = ctl.cfl > 0.0 ? 1 : 0;
  StagePlan plan[kCkStages];
  const int nst = step_plan(g.integrator, plan);
  for (int i = 0; i < nst; ++i)
    ESDG_TRY(run_stage_on<Real>(g.rep, L, g.k, g.desc, g.tile_prob, g.tiles, plan[i].in, plan[i].out, nullptr,
                                plan[i].mode, plan[i].b, plan[i].a, i == nst - 1 ? last : ctl));
  return ESDG_OK;
}

esdg_status enqueue_step(esdg_batch* b, const StepCtl& ctl) {
  const bool conc = (b->flags & ESDG_BATCH_CONCURRENT) && b->groups.size() > 1;
  if (conc) ESDG_HIP(&b->err, hipEventRecord(b->fork, b->stream));
  std::vector<bool> used(b->aux.size(), false);
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    BatchGroup& g = b->groups[gi];
    hipStream_t s = b->stream;
    if (conc) {
      const size_t a = gi % b->aux.size();
      s = b->aux[a];
      if (!used[a]) ESDG_HIP(&b->err, hipStreamWaitEvent(s, b->fork, 0));
      used[a] = true;
    }
    ESDG_TRY(g.rep->prec == PREC_FP32 ? group_step<float>(b, g, s, ctl) : group_step<double>(b, g, s, ctl));
  }
  if (conc) {
    for (size_t a = 0; a < b->aux.size(); ++a) {
      if (!used[a]) continue;
      ESDG_HIP(&b->err, hipEventRecord(b->join[a], b->aux[a]));
      ESDG_HIP(&b->err, hipStreamWaitEvent(b->stream, b->join[a], 0));
    }
  }
  return ESDG_OK;
}

esdg_status graph_for(esdg_batch* b, const StepCtl& ctl, hipGraphExec_t* out) {
  const bool cfl = ctl.cfl > 0.0;
  for (auto& e : b->graphs) {
    if (e.cfl == cfl && e.par == ctl.par && (cfl ? e.cfl_v == ctl.cfl : e.dt == ctl.dt_fixed)) {
      *out = e.exec;
      return ESDG_OK;
    }
  }
  if (b->graphs.size() >= 8) {
    ESDG_HIP(&b->err, hipStreamSynchronize(b->stream));
    drop_graphs(b);
  }
  ESDG_HIP(&b->err, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  esdg_status st = enqueue_step(b, ctl);
  hipGraph_t graph = nullptr;
  hipError_t ee = hipStreamEndCapture(b->stream, &graph);
  if (st != ESDG_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (ee != hipSuccess) return report(&b->err, ESDG_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ee));
  GraphEntry e;
  e.cfl = cfl;
  e.dt = ctl.dt_fixed;
  e.cfl_v = ctl.cfl;
  e.par = ctl.par;
  hipError_t ie = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return report(&b->err, ESDG_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ie));
  b->graphs.push_back(e);
  *out = e.exec;
  return ESDG_OK;
}

// order work already queued on member streams before the batch's work
esdg_status sync_in(esdg_batch* b) {
  for (size_t i = 0; i < b->mstreams.size(); ++i) {
    ESDG_HIP(&b->err, hipEventRecord(b->mevents[i], b->mstreams[i]));
    ESDG_HIP(&b->err, hipStreamWaitEvent(b->stream, b->mevents[i], 0));
  }
  return ESDG_OK;
}

// and the batch's work before later work on member streams
esdg_status sync_out(esdg_batch* b) {
  if (b->mstreams.empty()) return ESDG_OK;
  ESDG_HIP(&b->err, hipEventRecord(b->done, b->stream));
  for (hipStream_t s : b->mstreams) ESDG_HIP(&b->err, hipStreamWaitEvent(s, b->done, 0));
  return ESDG_OK;
}

// members stepped outside the batch: move their time and CFL slots to the
// batch's parity
esdg_status align_parity(esdg_batch* b) {
  const Launcher L = launcher_on(b, b->stream);
  for (esdg_problem* P : b->probs) {
    if (P->par == b->par) continue;
    ESDG_TRY(copy_parity(P, L, P->par));
    P->par = b->par;
  }
  return ESDG_OK;
}

esdg_status check_batch(esdg_batch* b) {
  if (!b) return report(nullptr, ESDG_EINVAL, "NULL batch handle");
  ESDG_HIP(&b->err, hipSetDevice(b->device));
  for (esdg_problem* P : b->probs)
    if (!P->have_state) return bfail(b, ESDG_ESTATE, "a member of the batch has no state");
  for (const BatchGroup& g : b->groups)
    for (int m : g.members)
      if (b->probs[m]->integrator != g.integrator)
        return bfail(b, ESDG_EINVAL, "a member's integrator changed after the batch was created");
  return ESDG_OK;
}

esdg_status gather(esdg_batch* b, std::vector<double>* t) {
  int count = (int)b->probs.size();
  int par = b->par;
  void* args[] = {&b->time_ptrs, &par, &count, &b->t_out};
  ESDG_TRY(launch_kernel(launcher_on(b, b->stream), -1, (const void*)&gather_times_kernel,
                         dim3((unsigned)((count + 255) / 256)), dim3(256), args));
  t->resize(count);
  ESDG_HIP(&b->err, hipMemcpyAsync(t->data(), b->t_out, sizeof(double) * count, hipMemcpyDeviceToHost, b->stream));
  ESDG_HIP(&b->err, hipStreamSynchronize(b->stream));
  return ESDG_OK;
}

// first member whose non-physical flag is raised (no wait), or -1
int flagged_member(const esdg_batch* b) {
  for (size_t i = 0; i < b->probs.size(); ++i)
    if (flag_raised(b->probs[i])) return (int)i;
  return -1;
}

void destroy_batch(esdg_batch* b) {
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_graphs(b);
  free_groups(b);
  void* bufs[] = {b->time_ptrs, b->t_out};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  for (auto& e : b->step_events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
  for (hipEvent_t e : b->mevents) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->done) (void)hipEventDestroy(b->done);
  for (hipStream_t s : b->aux) (void)hipStreamDestroy(s);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

}  // namespace

namespace {

// Time every tile variant of group g on its own launch shape: reps
// right-hand-side launches over all of its members' tiles (into the members'
// RHS buffers; states unchanged) after one untimed launch; us per launch in
// us[v], -1 for a variant without a kernel.
template <typename Real>
esdg_status time_group_variants(esdg_batch* b, const BatchGroup& g, int32_t reps, hipEvent_t e0, hipEvent_t e1,
                                double* us) {
  const Launcher L = launcher_on(b, b->stream);
  const void* fns[ESDG_TILE_VARIANTS];
  for (int v = 0; v < ESDG_TILE_VARIANTS; ++v) {
    us[v] = -1.0;
    fns[v] = nullptr;
    BatchGroup t;
    t.rep = g.rep;
    t.members = g.members;
    t.integrator = g.integrator;
    t.k = kernel_of_variant(g.rep, v);
    if (!t.k.fn) continue;
    fns[v] = t.k.fn;
    int same = -1;
    for (int w = 0; w < v; ++w)
      if (fns[w] == t.k.fn) same = w;
    if (same >= 0) {
      us[v] = us[same];
      continue;
    }
    esdg_status st = upload_group<Real>(b, t);
    auto one = [&]() {
      return run_stage_on<Real>(t.rep, L, t.k, t.desc, t.tile_prob, t.tiles, BUF_U, BUF_DU, nullptr, MODE_RHS, 0, 0,
                                StepCtl());
    };
    if (st == ESDG_OK) st = one();
    if (st == ESDG_OK && hipEventRecord(e0, b->stream) != hipSuccess) st = bfail(b, ESDG_EDEVICE, "hipEventRecord failed");
    for (int r = 0; r < reps && st == ESDG_OK; ++r) st = one();
    float ms = 0.0f;
    if (st == ESDG_OK && (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      st = bfail(b, ESDG_EDEVICE, "event timing failed");
    (void)hipStreamSynchronize(b->stream);
    if (t.desc) (void)hipFree(t.desc);
    if (t.tile_prob) (void)hipFree(t.tile_prob);
    ESDG_TRY(st);
    us[v] = 1000.0 * ms / reps;
  }
  return ESDG_OK;
}

}  // namespace

extern "C" {

static esdg_status batch_create_impl(esdg_problem* const* probs, int32_t count, const double* t_end, void* stream,
                                      int32_t flags, esdg_batch** out) {
  if (!probs || !out || count < 1) return report(nullptr, ESDG_EINVAL, "need count >= 1 problems and an output pointer");
  *out = nullptr;
  if (flags & ~(ESDG_BATCH_GRAPHS | ESDG_BATCH_CONCURRENT)) return report(nullptr, ESDG_EINVAL, "unknown batch flags");
  for (int i = 0; i < count; ++i) {
    if (!probs[i]) return report(nullptr, ESDG_EINVAL, "NULL problem in the batch");
    for (int j = 0; j < i; ++j)
      if (probs[j] == probs[i]) return report(nullptr, ESDG_EINVAL, "a problem appears twice in the batch");
    if (probs[i]->device != probs[0]->device) return report(nullptr, ESDG_EINVAL, "batch members on different devices");
    if (probs[i]->FSTAR)
      return report(nullptr, ESDG_EINVAL, "batch member %d is in once-per-face mode (batches evaluate faces fused)", i);
    if (t_end && std::isnan(t_end[i])) return report(nullptr, ESDG_EINVAL, "NaN end time");
  }
  esdg_batch* b = new esdg_batch();
  // released on every early return or exception until the batch is complete
  struct Owner {
    esdg_batch* b;
    ~Owner() {
      if (b) destroy_batch(b);
    }
  } own{b};
  b->device = probs[0]->device;
  b->flags = flags;
  b->probs.assign(probs, probs + count);
  for (int i = 0; i < count; ++i) b->t_end.push_back(t_end ? t_end[i] : INFINITY);
  auto bail = [&](esdg_status st) {
    std::string msg = b->err;
    own.b = nullptr;
    destroy_batch(b);
    return report(nullptr, st, "%s", msg.c_str());
  };
  if (hipSetDevice(b->device) != hipSuccess) return bail(bfail(b, ESDG_EDEVICE, "hipSetDevice failed"));
  b->stream = (hipStream_t)stream;
  if (!b->stream) {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(bfail(b, ESDG_EDEVICE, "hipStreamCreateWithFlags failed"));
    b->own_stream = true;
  }
  // groups by kernel parameters, in order of first appearance
  for (int i = 0; i < count; ++i) {
    esdg_problem* P = probs[i];
    BatchGroup* hit = nullptr;
    for (auto& g : b->groups) {
      const esdg_problem* R = g.rep;
      if (R->dim == P->dim && R->p == P->p && R->vf == P->vf && R->sf == P->sf && R->mesh == P->mesh &&
          R->prec == P->prec && R->gamma == P->gamma && R->nodes == P->nodes && R->integrator == P->integrator) {
        hit = &g;
        break;
      }
    }
    if (!hit) {
      b->groups.emplace_back();
      hit = &b->groups.back();
      hit->rep = P;
      hit->integrator = P->integrator;
    }
    hit->members.push_back(i);
    if (P->stream != b->stream && std::find(b->mstreams.begin(), b->mstreams.end(), P->stream) == b->mstreams.end())
      b->mstreams.push_back(P->stream);
  }
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess)
    return bail(bfail(b, ESDG_EDEVICE, "hipEventCreate failed"));
  for (size_t i = 0; i < b->mstreams.size(); ++i) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
      return bail(bfail(b, ESDG_EDEVICE, "hipEventCreate failed"));
    b->mevents.push_back(e);
  }
  if (flags & ESDG_BATCH_CONCURRENT) {
    const size_t naux = std::min<size_t>(b->groups.size(), 8);
    for (size_t a = 0; a < naux && b->groups.size() > 1; ++a) {
      hipStream_t s;
      hipEvent_t e;
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
        return bail(bfail(b, ESDG_EDEVICE, "hipStreamCreateWithFlags failed"));
      b->aux.push_back(s);
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
        return bail(bfail(b, ESDG_EDEVICE, "hipEventCreate failed"));
      b->join.push_back(e);
    }
  }
  std::vector<double*> tp(count);
  for (int i = 0; i < count; ++i) tp[i] = probs[i]->SCAL;
  if (hipMalloc((void**)&b->time_ptrs, sizeof(double*) * count) != hipSuccess ||
      hipMalloc((void**)&b->t_out, sizeof(double) * count) != hipSuccess)
    return bail(bfail(b, ESDG_ENOMEM, "device allocation of the batch tables failed"));
  if (hipMemcpyAsync(b->time_ptrs, tp.data(), sizeof(double*) * count, hipMemcpyHostToDevice, b->stream) != hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return bail(bfail(b, ESDG_EDEVICE, "upload of the batch tables failed"));
  esdg_status st = refresh_groups(b);
  if (st != ESDG_OK) return bail(st);
  own.b = nullptr;
  *out = b;
  return ESDG_OK;
}

void esdg_batch_destroy(esdg_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  destroy_batch(b);
}

static esdg_status batch_step_impl(esdg_batch* b, double dt, int32_t nsteps, double cfl) {
  ESDG_TRY(check_batch(b));
  if (nsteps < 0) return bfail(b, ESDG_EINVAL, "nsteps must be >= 0");
  const bool use_cfl = !(dt > 0.0);
  if (use_cfl && !(cfl > 0.0)) return bfail(b, ESDG_EINVAL, "dt <= 0 needs cfl > 0");
  if (nsteps == 0) return ESDG_OK;
  // members an earlier kernel found non-physical are not stepped;
  // esdg_batch_sync names them and clears their flags
  const int flagged = flagged_member(b);
  if (flagged >= 0)
    return report(&b->err, ESDG_ENONPHYSICAL, "member %d met a non-physical state (see esdg_batch_sync)", flagged);
  ESDG_TRY(refresh_groups(b));
  ESDG_TRY(sync_in(b));
  const Launcher L = launcher_on(b, b->stream);
  // every member enters at the batch's parity, with the CFL value of its
  // current state in that slot (copied, or one reduction as in esdg_step)
  ESDG_TRY(align_parity(b));
  for (esdg_problem* P : b->probs) {
    if (use_cfl && !P->lam_valid) {
      ESDG_TRY(run_reduce(P, L, RED_MAXLAMBDA, cfl, lam_slot(P, b->par)));
      P->lam_valid = true;
    }
  }
  StepCtl ctl;
  if (use_cfl) ctl.cfl = cfl;
  else ctl.dt_fixed = dt;
  for (int s = 0; s < nsteps; ++s) {
    ctl.par = b->par;
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (b->timing) {
      ESDG_HIP(&b->err, hipEventCreate(&ev.first));
      ESDG_HIP(&b->err, hipEventCreate(&ev.second));
      b->step_events.push_back(ev);
    }
    hipGraphExec_t exec = nullptr;
    if (b->flags & ESDG_BATCH_GRAPHS) ESDG_TRY(graph_for(b, ctl, &exec));
    if (b->timing) ESDG_HIP(&b->err, hipEventRecord(ev.first, b->stream));
    if (exec) ESDG_HIP(&b->err, hipGraphLaunch(exec, b->stream));
    else ESDG_TRY(enqueue_step(b, ctl));
    if (b->timing) ESDG_HIP(&b->err, hipEventRecord(ev.second, b->stream));
    b->par = 1 - b->par;
    for (esdg_problem* P : b->probs) P->par = b->par;
  }
  for (esdg_problem* P : b->probs) P->lam_valid = use_cfl;
  return sync_out(b);
}

static esdg_status batch_rhs_impl(esdg_batch* b, double* const* du, int32_t where) {
  ESDG_TRY(check_batch(b));
  ESDG_TRY(refresh_groups(b));
  ESDG_TRY(sync_in(b));
  const Launcher L = launcher_on(b, b->stream);
  for (auto& g : b->groups) {
    esdg_status st = g.rep->prec == PREC_FP32
                         ? run_stage_on<float>(g.rep, L, g.k, g.desc, g.tile_prob, g.tiles, BUF_U, BUF_DU, nullptr,
                                               MODE_RHS, 0.0, 0.0, StepCtl())
                         : run_stage_on<double>(g.rep, L, g.k, g.desc, g.tile_prob, g.tiles, BUF_U, BUF_DU, nullptr,
                                                MODE_RHS, 0.0, 0.0, StepCtl());
    ESDG_TRY(st);
  }
  const bool host = where != ESDG_DEVICE;
  if (du) {
    for (size_t i = 0; i < b->probs.size(); ++i) {
      if (!du[i]) continue;
      esdg_problem* P = b->probs[i];
      const size_t bytes = state_count(P) * sizeof(double);
      if (P->prec == PREC_FP32) {
        ESDG_TRY(convert_state(P, L, P->DU, host ? (void*)P->STAGE64 : (void*)du[i], 1));
        if (host) ESDG_HIP(&b->err, hipMemcpyAsync(du[i], P->STAGE64, bytes, hipMemcpyDeviceToHost, b->stream));
      } else {
        ESDG_HIP(&b->err, hipMemcpyAsync(du[i], P->DU, bytes, host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                                         b->stream));
      }
    }
    if (host) ESDG_HIP(&b->err, hipStreamSynchronize(b->stream));
  }
  return sync_out(b);
}

static esdg_status batch_times_impl(esdg_batch* b, double* t) {
  if (!b || !t) return report(b ? &b->err : nullptr, ESDG_EINVAL, "NULL argument");
  ESDG_HIP(&b->err, hipSetDevice(b->device));
  ESDG_TRY(sync_in(b));
  ESDG_TRY(align_parity(b));
  std::vector<double> tv;
  ESDG_TRY(gather(b, &tv));
  std::copy(tv.begin(), tv.end(), t);
  return ESDG_OK;
}

static esdg_status batch_sync_impl(esdg_batch* b, int32_t* bad) {
  if (!b) return report(nullptr, ESDG_EINVAL, "NULL batch handle");
  ESDG_HIP(&b->err, hipSetDevice(b->device));
  if (bad) *bad = -1;
  ESDG_TRY(sync_in(b));
  ESDG_TRY(align_parity(b));
  ESDG_HIP(&b->err, hipStreamSynchronize(b->stream));
  const int i = flagged_member(b);
  if (i >= 0) {
    if (bad) *bad = (int32_t)i;
    flag_clear(b->probs[i]);
    return report(&b->err, ESDG_ENONPHYSICAL, "member %d met a non-physical state (rho <= 0, p <= 0 or non-finite)", i);
  }
  return ESDG_OK;
}

static esdg_status batch_autotune_impl(esdg_batch* b, int32_t reps) {
  ESDG_TRY(check_batch(b));
  if (reps < 1) return bfail(b, ESDG_EINVAL, "reps must be >= 1");
  ESDG_HIP(&b->err, hipStreamSynchronize(b->stream));
  // the members' own streams may still hold work on their states
  for (hipStream_t s : b->mstreams) ESDG_HIP(&b->err, hipStreamSynchronize(s));
  ESDG_TRY(refresh_groups(b));
  hipEvent_t e0, e1;
  ESDG_HIP(&b->err, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return bfail(b, ESDG_EDEVICE, "hipEventCreate failed");
  }
  esdg_status st = ESDG_OK;
  for (size_t gi = 0; gi < b->groups.size() && st == ESDG_OK; ++gi) {
    const BatchGroup& g = b->groups[gi];
    if (g.rep->nodes != NODES_LGL || g.rep->dim != 3) continue;  // one variant only
    double us[ESDG_TILE_VARIANTS];
    st = g.rep->prec == PREC_FP32 ? time_group_variants<float>(b, g, reps, e0, e1, us)
                                  : time_group_variants<double>(b, g, reps, e0, e1, us);
    int pick = -1;
    for (int v = 0; v < ESDG_TILE_VARIANTS && st == ESDG_OK; ++v)
      if (us[v] >= 0.0 && (pick < 0 || us[v] < us[pick])) pick = v;
    if (st == ESDG_OK && pick >= 0) set_tile_variant(g.rep, pick);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ESDG_TRY(st);
  return refresh_groups(b);
}

esdg_status esdg_batch_info(esdg_batch* b, int32_t* groups, int64_t* tiles) {
  if (!b) return report(nullptr, ESDG_EINVAL, "NULL batch handle");
  ESDG_TRY(refresh_groups(b));
  if (groups) *groups = (int32_t)b->groups.size();
  if (tiles) {
    int64_t t = 0;
    for (auto& g : b->groups) t += g.tiles;
    *tiles = t;
  }
  return ESDG_OK;
}

esdg_status esdg_batch_timing_enable(esdg_batch* b, int32_t enable) {
  if (!b) return report(nullptr, ESDG_EINVAL, "NULL batch handle");
  b->timing = enable != 0;
  return ESDG_OK;
}

static esdg_status batch_timing_read_impl(esdg_batch* b, double* total_ms, int64_t* steps) {
  if (!b) return report(nullptr, ESDG_EINVAL, "NULL batch handle");
  ESDG_HIP(&b->err, hipSetDevice(b->device));
  double sum = 0.0;
  for (auto& e : b->step_events) {
    ESDG_HIP(&b->err, hipEventSynchronize(e.second));
    float ms = 0.0f;
    ESDG_HIP(&b->err, hipEventElapsedTime(&ms, e.first, e.second));
    sum += ms;
  }
  if (total_ms) *total_ms = sum;
  if (steps) *steps = (int64_t)b->step_events.size();
  for (auto& e : b->step_events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  b->step_events.clear();
  return ESDG_OK;
}

const char* esdg_batch_last_error(const esdg_batch* b) { return b ? b->err.c_str() : ""; }

esdg_status esdg_batch_create(esdg_problem* const* probs, int32_t count, const double* t_end, void* stream,
                              int32_t flags, esdg_batch** out) {
  return guarded(nullptr, [&] { return batch_create_impl(probs, count, t_end, stream, flags, out); });
}

esdg_status esdg_batch_step(esdg_batch* b, double dt, int32_t nsteps, double cfl) {
  return guarded(b ? &b->err : nullptr, [&] { return batch_step_impl(b, dt, nsteps, cfl); });
}

esdg_status esdg_batch_rhs(esdg_batch* b, double* const* du, int32_t where) {
  return guarded(b ? &b->err : nullptr, [&] { return batch_rhs_impl(b, du, where); });
}

esdg_status esdg_batch_times(esdg_batch* b, double* t) {
  return guarded(b ? &b->err : nullptr, [&] { return batch_times_impl(b, t); });
}

esdg_status esdg_batch_sync(esdg_batch* b, int32_t* bad) {
  return guarded(b ? &b->err : nullptr, [&] { return batch_sync_impl(b, bad); });
}

esdg_status esdg_batch_autotune(esdg_batch* b, int32_t reps) {
  return guarded(b ? &b->err : nullptr, [&] { return batch_autotune_impl(b, reps); });
}

esdg_status esdg_batch_timing_read(esdg_batch* b, double* total_ms, int64_t* steps) {
  return guarded(b ? &b->err : nullptr, [&] { return batch_timing_read_impl(b, total_ms, steps); });
}

}  // extern "C"
