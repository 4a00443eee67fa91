// Serving (include/esdg.h): a continuous-batching loop over time-integration
// jobs.  Admission by device-memory footprint in arrival order; the admitted
// jobs are stepped together as one batch; jobs that reach their end time are
// retired and their memory is returned when their state is fetched.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <deque>
#include <exception>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "esdg.h"

namespace {

struct Job {
  esdg_mesh_desc mesh{};
  std::vector<double> u0;
  double t0 = 0.0, t_end = 0.0, t = 0.0;
  int64_t bytes = 0;
  int64_t steps = 0;
  int status = ESDG_JOB_QUEUED;
  esdg_problem* P = nullptr;
};

}  // namespace

struct esdg_server {
  esdg_server_config cfg{};
  int device = 0;
  hipStream_t admit_stream = nullptr;  // uploads of admitted jobs (their problems' stream)
  hipStream_t batch_stream = nullptr;  // steps of the batch
  std::unordered_map<int64_t, Job> jobs;
  std::deque<int64_t> queue;
  std::vector<int64_t> active;         // being stepped, in admission order
  std::vector<int64_t> finished;       // finished in the last tick
  esdg_batch* batch = nullptr;
  bool dirty = true;                   // batch membership changed
  int64_t used = 0, budget = 0;
  int64_t next_id = 1;
  std::string err;
};

namespace {

esdg_status sfail(esdg_server* S, esdg_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (S) S->err = buf;
  return st;
}

// Runs f, turning C++ exceptions into status codes (none crosses the C ABI).
template <typename F>
esdg_status sguard(esdg_server* S, F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return sfail(S, ESDG_ENOMEM, "host memory exhausted");
  } catch (const std::exception& e) {
    return sfail(S, ESDG_EDEVICE, "%s", e.what());
  }
}

void release(esdg_server* S, Job& j) {
  if (j.P) {
    esdg_destroy(j.P);
    j.P = nullptr;
    S->used -= j.bytes;
  }
}

// the admission rule: one more job of `bytes` fits beside `used` bytes and
// `active` jobs
bool admissible(int64_t bytes, int64_t used, int64_t budget, int64_t active, int64_t max_active) {
  if (max_active > 0 && active >= max_active) return false;
  return used + bytes <= budget;
}

// admit queued jobs in arrival order while they fit
esdg_status admit(esdg_server* S) {
  while (!S->queue.empty()) {
    Job& j = S->jobs[S->queue.front()];
    if (!admissible(j.bytes, S->used, S->budget, (int64_t)S->active.size(), S->cfg.max_active)) break;
    esdg_mesh_desc d = j.mesh;
    d.coords = nullptr;
    d.stream = S->admit_stream;
    esdg_status st = esdg_init_mesh(&d, &j.P);
    if (st == ESDG_OK) {
      S->used += j.bytes;
      st = esdg_set_state(j.P, j.u0.data(), ESDG_HOST);
      if (st == ESDG_OK) st = esdg_set_time(j.P, j.t0);
    }
    const int64_t id = S->queue.front();
    S->queue.pop_front();
    std::vector<double>().swap(j.u0);
    if (st != ESDG_OK) {
      sfail(S, st, "job %lld: %s", (long long)id, esdg_last_error(j.P));
      release(S, j);
      j.status = ESDG_JOB_FAILED;
      S->finished.push_back(id);
      continue;
    }
    j.status = ESDG_JOB_ACTIVE;
    j.t = j.t0;
    S->active.push_back(id);
    S->dirty = true;
  }
  return ESDG_OK;
}

esdg_status rebuild_batch(esdg_server* S) {
  if (S->batch) {
    esdg_batch_destroy(S->batch);
    S->batch = nullptr;
  }
  S->dirty = false;
  if (S->active.empty()) return ESDG_OK;
  std::vector<esdg_problem*> probs;
  std::vector<double> t_end;
  for (int64_t id : S->active) {
    probs.push_back(S->jobs[id].P);
    t_end.push_back(S->jobs[id].t_end);
  }
  esdg_status st = esdg_batch_create(probs.data(), (int32_t)probs.size(), t_end.data(), S->batch_stream, S->cfg.flags,
                                     &S->batch);
  if (st != ESDG_OK) return sfail(S, st, "batch: %s", esdg_last_error(nullptr));
  return ESDG_OK;
}

}  // namespace

extern "C" {

static esdg_status server_create_impl(const esdg_server_config* cfg, esdg_server** out) {
  if (!cfg || !out) return ESDG_EINVAL;
  *out = nullptr;
  if (cfg->steps_per_tick < 1 || !(cfg->cfl > 0.0) || cfg->max_active < 0 || cfg->hbm_budget < 0) return ESDG_EINVAL;
  esdg_server* S = new esdg_server();
  S->cfg = *cfg;
  if (hipGetDevice(&S->device) != hipSuccess ||
      hipStreamCreateWithFlags(&S->admit_stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&S->batch_stream, hipStreamNonBlocking) != hipSuccess) {
    esdg_server_destroy(S);
    return ESDG_EDEVICE;
  }
  S->budget = cfg->hbm_budget;
  if (S->budget == 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      esdg_server_destroy(S);
      return ESDG_EDEVICE;
    }
    S->budget = (int64_t)(0.9 * (double)free_b);
  }
  *out = S;
  return ESDG_OK;
}

void esdg_server_destroy(esdg_server* S) {
  if (!S) return;
  (void)hipSetDevice(S->device);
  if (S->batch) esdg_batch_destroy(S->batch);
  for (auto& kv : S->jobs) release(S, kv.second);
  if (S->admit_stream) (void)hipStreamDestroy(S->admit_stream);
  if (S->batch_stream) (void)hipStreamDestroy(S->batch_stream);
  delete S;
}

static esdg_status server_submit_impl(esdg_server* S, const esdg_job_desc* job, int64_t* job_id) {
  if (!S || !job || !job->u0) return sfail(S, ESDG_EINVAL, "NULL argument");
  if (!(job->t_end > job->t0)) return sfail(S, ESDG_EINVAL, "need t_end > t0");
  if (job->mesh.coords) return sfail(S, ESDG_EINVAL, "jobs take box meshes (coords must be NULL)");
  Job j;
  j.mesh = job->mesh;
  j.mesh.stream = nullptr;
  esdg_status st = esdg_footprint(&j.mesh, &j.bytes);
  if (st != ESDG_OK) return sfail(S, st, "%s", esdg_last_error(nullptr));
  if (j.bytes > S->budget) return sfail(S, ESDG_EINVAL, "job needs %lld bytes, more than the whole budget", (long long)j.bytes);
  int64_t E = 1, nn = 1;
  for (int k = 0; k < j.mesh.dim; ++k) {
    E *= j.mesh.n[k];
    nn *= j.mesh.p + 1;
  }
  j.u0.assign(job->u0, job->u0 + E * (j.mesh.dim + 2) * nn);
  j.t0 = job->t0;
  j.t_end = job->t_end;
  j.t = job->t0;
  const int64_t id = S->next_id++;
  S->jobs.emplace(id, std::move(j));
  S->queue.push_back(id);
  if (job_id) *job_id = id;
  return ESDG_OK;
}

static esdg_status server_tick_impl(esdg_server* S, int32_t* finished, int32_t* active, int32_t* queued) {
  if (!S) return ESDG_EINVAL;
  if (hipSetDevice(S->device) != hipSuccess) return sfail(S, ESDG_EDEVICE, "hipSetDevice failed");
  S->finished.clear();
  esdg_status st = ESDG_OK;
  if (S->dirty) st = rebuild_batch(S);
  if (st != ESDG_OK) return st;
  // enqueue the steps first, so that admissions overlap the device work
  const bool stepping = S->batch != nullptr;
  if (stepping) {
    st = esdg_batch_step(S->batch, 0.0, S->cfg.steps_per_tick, S->cfg.cfl);
    if (st != ESDG_OK) return sfail(S, st, "step: %s", esdg_batch_last_error(S->batch));
  }
  const size_t stepped = S->active.size();
  st = admit(S);
  if (st != ESDG_OK) return st;
  if (stepping) {
    int32_t bad = -1;
    std::vector<double> t(stepped);
    st = esdg_batch_sync(S->batch, &bad);
    while (st == ESDG_ENONPHYSICAL) {
      Job& j = S->jobs[S->active[bad]];
      j.status = ESDG_JOB_FAILED;
      st = esdg_batch_sync(S->batch, &bad);  // flags were cleared: reports the next one, if any
    }
    if (st != ESDG_OK) return sfail(S, st, "sync: %s", esdg_batch_last_error(S->batch));
    st = esdg_batch_times(S->batch, t.data());
    if (st != ESDG_OK) return sfail(S, st, "times: %s", esdg_batch_last_error(S->batch));
    std::vector<int64_t> keep;
    for (size_t i = 0; i < stepped; ++i) {
      const int64_t id = S->active[i];
      Job& j = S->jobs[id];
      j.t = t[i];
      j.steps += S->cfg.steps_per_tick;
      if (j.status == ESDG_JOB_FAILED) {
        S->finished.push_back(id);
        S->dirty = true;
      } else if (j.t >= j.t_end) {
        j.status = ESDG_JOB_DONE;
        S->finished.push_back(id);
        S->dirty = true;
      } else {
        keep.push_back(id);
      }
    }
    // jobs admitted during this tick follow the ones that were stepped
    keep.insert(keep.end(), S->active.begin() + stepped, S->active.end());
    S->active.swap(keep);
  }
  if (finished) *finished = (int32_t)S->finished.size();
  if (active) *active = (int32_t)S->active.size();
  if (queued) *queued = (int32_t)S->queue.size();
  return ESDG_OK;
}

esdg_status esdg_server_finished(esdg_server* S, int64_t* ids, int32_t max, int32_t* n) {
  if (!S) return ESDG_EINVAL;
  const int32_t k = std::min<int32_t>(max, (int32_t)S->finished.size());
  for (int32_t i = 0; i < k && ids; ++i) ids[i] = S->finished[i];
  if (n) *n = k;
  return ESDG_OK;
}

esdg_status esdg_server_job(esdg_server* S, int64_t id, int32_t* status, double* t, int64_t* steps) {
  if (!S) return ESDG_EINVAL;
  auto it = S->jobs.find(id);
  if (it == S->jobs.end()) return sfail(S, ESDG_EINVAL, "unknown job %lld", (long long)id);
  if (status) *status = it->second.status;
  if (t) *t = it->second.t;
  if (steps) *steps = it->second.steps;
  return ESDG_OK;
}

static esdg_status server_fetch_impl(esdg_server* S, int64_t id, double* u) {
  if (!S) return ESDG_EINVAL;
  auto it = S->jobs.find(id);
  if (it == S->jobs.end()) return sfail(S, ESDG_EINVAL, "unknown job %lld", (long long)id);
  Job& j = it->second;
  if (j.status != ESDG_JOB_DONE && j.status != ESDG_JOB_FAILED)
    return sfail(S, ESDG_ESTATE, "job %lld has not finished", (long long)id);
  esdg_status st = ESDG_OK;
  if (u && j.status == ESDG_JOB_DONE) st = esdg_get_state(j.P, u, ESDG_HOST);
  if (st != ESDG_OK) return sfail(S, st, "fetch: %s", esdg_last_error(j.P));
  release(S, j);
  S->jobs.erase(it);
  return ESDG_OK;
}

esdg_status esdg_server_memory(esdg_server* S, int64_t* used, int64_t* budget) {
  if (!S) return ESDG_EINVAL;
  if (used) *used = S->used;
  if (budget) *budget = S->budget;
  return ESDG_OK;
}

const char* esdg_server_last_error(const esdg_server* S) { return S ? S->err.c_str() : ""; }

esdg_status esdg_server_create(const esdg_server_config* cfg, esdg_server** out) {
  return sguard(nullptr, [&] { return server_create_impl(cfg, out); });
}

esdg_status esdg_server_submit(esdg_server* S, const esdg_job_desc* job, int64_t* job_id) {
  return sguard(S, [&] { return server_submit_impl(S, job, job_id); });
}

esdg_status esdg_server_tick(esdg_server* S, int32_t* finished, int32_t* active, int32_t* queued) {
  return sguard(S, [&] { return server_tick_impl(S, finished, active, queued); });
}

esdg_status esdg_server_fetch(esdg_server* S, int64_t id, double* u) {
  return sguard(S, [&] { return server_fetch_impl(S, id, u); });
}

esdg_status esdg_server_plan(const int64_t* queued_bytes, int32_t n_queued, int64_t used, int64_t budget,
                             int32_t active, int32_t max_active, int32_t* n_admit) {
  if (!n_admit || n_queued < 0 || (n_queued > 0 && !queued_bytes) || used < 0 || budget < 0 || active < 0 ||
      max_active < 0)
    return ESDG_EINVAL;
  int32_t k = 0;
  for (; k < n_queued; ++k) {
    if (queued_bytes[k] < 0) return ESDG_EINVAL;
    if (!admissible(queued_bytes[k], used, budget, (int64_t)active + k, max_active)) break;
    used += queued_bytes[k];
  }
  *n_admit = k;
  return ESDG_OK;
}

}  // extern "C"
