// Serving: continuous batching of ensemble-gradient jobs over one device
// pool (the ensemble_server_* entry points of ensode.h).  Included at the end
// of ensode.hip: it uses that file's validation, layout and dispatch helpers.
//
// Device side: serve_kernel is a persistent kernel.  Its grid is sized to the
// GPU; every block repeatedly takes the next 256-trajectory tile from a
// device-resident queue (one atomic counter over the packed jobs' tiles),
// runs the record (phase 0) or the reverse sweep (phase 1) of that tile --
// the same code as ensemble_record / ensemble_adjoint, so a trajectory's
// results do not depend on what it is packed with -- and exits when the
// queue is empty.
//
// Host side: jobs wait in FIFO order until their record fits in the pool
// (first-fit allocator with coalescing); admitted jobs of one family are
// packed into one launch on a free slot (stream).  Retiring a launch frees
// its jobs' memory; a job whose record ran out of pages is run again with a
// larger plan.
#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <unordered_map>
#include <vector>

#include "arena.h"

namespace {

struct ServeJob {
  FwdArgs fwd;
  AdjArgs adj;
  int64_t tile_begin;  // first tile of this job in the launch's queue
  int64_t n_tiles;
};

// Per-launch setup: the records' counters and save times, the two tile
// counters and the job flags (kernels rather than memsets).
__global__ void serve_setup_kernel(const ServeJob* jobs, int n_jobs, unsigned* next,
                                   int* flags) {
  const int j = blockIdx.x;
  const ServeJob& J = jobs[j];
  if (threadIdx.x < 8) J.fwd.rec.counters[threadIdx.x] = 0ull;
  if ((int)threadIdx.x < J.fwd.ivp.st.n)
    ((double*)J.fwd.rec.save_times)[threadIdx.x] = J.fwd.ivp.st.t[threadIdx.x];
  if (threadIdx.x == 0) flags[j] = 0;
  if (j == 0 && threadIdx.x < 2) next[threadIdx.x] = 0u;
}

// PHASE 0 records every tile, PHASE 1 sweeps every tile back: two launches
// on one stream, so each phase keeps the register budget of its own code.
template <class Sys, class Tab, class T, int PHASE>
__global__ void __launch_bounds__(256) serve_kernel(const ServeJob* jobs, int n_jobs,
                                                     int64_t n_tiles, unsigned* next,
                                                     int* flags) {
  __shared__ int64_t s_tile;
  __shared__ int s_job;
  for (;;) {
    __syncthreads();  // every thread is done with the previous tile's LDS
    if (threadIdx.x == 0) {
      const int64_t t = (int64_t)atomicAdd(next, 1u);
      int lo = 0, hi = n_jobs - 1;  // last job with tile_begin <= t
      while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (jobs[mid].tile_begin <= t) lo = mid;
        else hi = mid - 1;
      }
      s_tile = t;
      s_job = lo;
    }
    __syncthreads();
    const int64_t t = s_tile;
    if (t >= n_tiles) break;  // the queue is empty: every block gets here
    const int j = s_job;
    const ServeJob& J = jobs[j];
    const int64_t block = t - J.tile_begin;
    if constexpr (PHASE == 0) {
      erk_forward_body<Sys, Tab, T, MODE_RECORD, false>(J.fwd, block);
      const int64_t tr = block * blockDim.x + threadIdx.x;
      if (tr < J.fwd.ivp.n && J.fwd.rec.status[tr] == LANE_NOSPACE) atomicOr(&flags[j], 1);
    } else {
      erk_adjoint_body<Sys, Tab, T, false, false>(J.adj, block);
    }
  }
}

constexpr int SERVE_MAX_JOBS = 256;   // jobs packed into one launch
constexpr int SERVE_MAX_SLOTS = 8;
constexpr int SERVE_MAX_RETRIES = 3;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct SrvJob {
  ens_job desc;
  std::vector<double> save_times;
  int32_t state = ENS_JOB_WAITING;
  int64_t hint = 512;
  int retries = 0;
  size_t off = 0, bytes = 0;
  bool has_mem = false;
  ens_record rec{};
  double t_submit = 0, t_done = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  ServeJob* h_jobs = nullptr;  // pinned staging
  int* h_flags = nullptr;      // pinned
  ServeJob* d_jobs = nullptr;  // in the pool's control area
  int* d_flags = nullptr;
  unsigned* d_next = nullptr;
  std::vector<int64_t> ids;
  bool busy = false;
};

int family_of(const ens_problem& p) { return (p.system * 16 + p.method) * 4 + p.dtype; }

}  // namespace

struct ens_server {
  char* pool = nullptr;
  size_t pool_bytes = 0;
  char* arena_base = nullptr;
  ens_host::Arena arena;
  std::vector<Slot> slots;
  std::unordered_map<int64_t, SrvJob> jobs;
  std::deque<int64_t> waiting;
  int64_t next_id = 1;
  int64_t submitted = 0, completed = 0, failed = 0, retried = 0, lanes = 0;
  double t_first = -1, t_last = -1;
  std::vector<double> latencies;
  int cus = 0;
  std::map<int, int> blocks_per_cu;  // per family
};

namespace {

// The reverse sweep's per-save cotangents, [n_save][dim][n], at the end of
// the job's allocation.
size_t job_contrib_bytes(const SrvJob& J) {
  SysInfo si;
  sys_info(J.desc.prob.system, &si);
  const int nse = J.desc.ivp.n_save > 0 ? J.desc.ivp.n_save : 1;
  return align256((size_t)nse * si.d * J.desc.ivp.n * elem_size(J.desc.prob.dtype));
}

size_t job_record_bytes(const SrvJob& J, int64_t hint) {
  SysInfo si;
  sys_info(J.desc.prob.system, &si);
  const int nse = J.desc.ivp.n_save > 0 ? J.desc.ivp.n_save : 1;
  Layout L = layout(J.desc.ivp.n, nse, si.d, J.desc.prob.dtype, 0);
  const int64_t pages_per = (hint + PAGE_STEPS - 1) / PAGE_STEPS;
  const int64_t n_static = pages_per * J.desc.ivp.n;
  const int64_t n_over = n_static / 8 + 64;
  return L.fixed + 512 + (size_t)n_static * L.page_bytes + (size_t)n_over * (L.page_bytes + 8) +
         job_contrib_bytes(J);
}

void free_job_memory(ens_server* s, SrvJob& J) {
  if (J.has_mem) s->arena.release(J.off, J.bytes);
  J.has_mem = false;
}

void finish_job(ens_server* s, SrvJob& J, int32_t state) {
  free_job_memory(s, J);
  J.state = state;
  J.t_done = now_s();
  s->t_last = J.t_done;
  if (state == ENS_JOB_DONE) {
    ++s->completed;
    s->lanes += J.desc.ivp.n;
    s->latencies.push_back(J.t_done - J.t_submit);
  } else {
    ++s->failed;
  }
}

int retire(ens_server* s) {
  for (Slot& sl : s->slots) {
    if (!sl.busy) continue;
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return hip_fail(q, "serve launch");
    std::vector<int64_t> again;
    for (size_t k = 0; k < sl.ids.size(); ++k) {
      SrvJob& J = s->jobs[sl.ids[k]];
      const bool nospace = (sl.h_flags[k] & 1) != 0;
      if (nospace && J.retries < SERVE_MAX_RETRIES) {
        free_job_memory(s, J);
        J.hint *= 2;
        ++J.retries;
        ++s->retried;
        J.state = ENS_JOB_WAITING;
        again.push_back(sl.ids[k]);
      } else {
        finish_job(s, J, nospace ? ENS_JOB_FAILED : ENS_JOB_DONE);
      }
    }
    for (auto it = again.rbegin(); it != again.rend(); ++it) s->waiting.push_front(*it);
    sl.ids.clear();
    sl.busy = false;
  }
  return ENS_OK;
}

// One persistent launch of the packed jobs on slot `sl`.
int launch_slot(ens_server* s, Slot& sl, const std::vector<int64_t>& ids) {
  int64_t tiles = 0;
  for (size_t k = 0; k < ids.size(); ++k) {
    SrvJob& J = s->jobs[ids[k]];
    ens_job& d = J.desc;
    ens_tape_cfg tc{};
    const size_t cb = job_contrib_bytes(J);
    tc.pool = s->arena_base + J.off;
    tc.pool_bytes = J.bytes - cb;
    tc.ckpt_every = 0;
    tc.steps_per_traj = (int32_t)J.hint;
    SysInfo si;
    sys_info(d.prob.system, &si);
    const int nse = d.ivp.n_save > 0 ? d.ivp.n_save : 1;
    Layout L = layout(d.ivp.n, nse, si.d, d.prob.dtype, 0);
    PageSplit ps;
    if (!split_pages(L, d.ivp.n, tc.pool_bytes, (int32_t)J.hint, PAGE_STEPS, &ps))
      return fail(ENS_ENOSPACE, "serve: record plan does not fit its allocation");
    ens_ivp v = d.ivp;
    v.save_times = J.save_times.empty() ? nullptr : J.save_times.data();
    fill_record(&J.rec, &d.prob, &v, &tc, L, ps);
    ServeJob& H = sl.h_jobs[k];
    memset(&H, 0, sizeof H);
    H.fwd.ivp = ivp_args(&d.prob, &v);
    H.fwd.rec = view_of(&J.rec);
    H.fwd.y_save = d.y_save;
    H.fwd.lane_status = d.lane_status;
    H.adj.ivp = H.fwd.ivp;
    H.adj.rec = H.fwd.rec;
    H.adj.loss_kind = d.loss.kind;
    H.adj.loss_data = d.loss.data;
    H.adj.scale = d.loss.scale;
    H.adj.grad_p = d.grad_params;
    H.adj.grad_y0 = d.grad_y0;
    H.adj.loss_out = d.loss_out;
    H.adj.contrib = s->arena_base + J.off + tc.pool_bytes;
    H.tile_begin = tiles;
    H.n_tiles = grid_of(d.ivp.n);
    tiles += H.n_tiles;
    J.state = ENS_JOB_RUNNING;
  }
  const int n_jobs = (int)ids.size();
  hipError_t e = hipMemcpyAsync(sl.d_jobs, sl.h_jobs, n_jobs * sizeof(ServeJob),
                                hipMemcpyHostToDevice, sl.stream);
  if (e != hipSuccess) return hip_fail(e, "serve: job table");
  hipLaunchKernelGGL(serve_setup_kernel, dim3(n_jobs), dim3(64), 0, sl.stream, sl.d_jobs,
                     n_jobs, sl.d_next, sl.d_flags);
  const ens_problem& p0 = s->jobs[ids[0]].desc.prob;
  const int fam = family_of(p0);
  int rc = with_kernels(p0.system, p0.method, p0.dtype, [&](auto sy, auto me, auto ty) {
    using Sys = decltype(sy);
    using Tab = decltype(me);
    using T = decltype(ty);
    auto k0 = serve_kernel<Sys, Tab, T, 0>;
    auto k1 = serve_kernel<Sys, Tab, T, 1>;
    auto occ = [&](auto kern, int key) {
      auto it = s->blocks_per_cu.find(key);
      if (it != s->blocks_per_cu.end()) return it->second;
      int per_cu = 0;
      hipError_t oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, BLOCK, 0);
      if (oe != hipSuccess || per_cu < 1) per_cu = 1;
      s->blocks_per_cu[key] = per_cu;
      return per_cu;
    };
    const int64_t g0 = std::min<int64_t>(tiles, (int64_t)occ(k0, 2 * fam) * s->cus);
    const int64_t g1 = std::min<int64_t>(tiles, (int64_t)occ(k1, 2 * fam + 1) * s->cus);
    hipLaunchKernelGGL(k0, dim3((unsigned)g0), dim3(BLOCK), 0, sl.stream, sl.d_jobs, n_jobs,
                       tiles, sl.d_next, sl.d_flags);
    hipLaunchKernelGGL(k1, dim3((unsigned)g1), dim3(BLOCK), 0, sl.stream, sl.d_jobs, n_jobs,
                       tiles, sl.d_next + 1, sl.d_flags);
    return ENS_OK;
  });
  if (rc != ENS_OK) return rc;
  e = hipMemcpyAsync(sl.h_flags, sl.d_flags, n_jobs * sizeof(int), hipMemcpyDeviceToHost,
                     sl.stream);
  if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "serve launch");
  sl.ids = ids;
  sl.busy = true;
  return ENS_OK;
}

// Admit waiting jobs in FIFO order and pack them into launches, one family
// per launch, while slots are free.
int launch_waiting(ens_server* s) {
  for (Slot& sl : s->slots) {
    if (sl.busy) continue;
    if (s->waiting.empty()) break;
    const int fam = family_of(s->jobs[s->waiting.front()].desc.prob);
    std::vector<int64_t> pick;
    for (auto it = s->waiting.begin(); it != s->waiting.end();) {
      SrvJob& J = s->jobs[*it];
      if (family_of(J.desc.prob) != fam) {
        ++it;
        continue;
      }
      if ((int)pick.size() == SERVE_MAX_JOBS) break;
      const size_t need = job_record_bytes(J, J.hint);
      if (need > s->arena.size()) {  // can never run
        finish_job(s, J, ENS_JOB_FAILED);
        it = s->waiting.erase(it);
        continue;
      }
      size_t off;
      if (!s->arena.alloc(need, &off)) break;  // keep FIFO order within the family
      J.off = off;
      J.bytes = align256(need);
      J.has_mem = true;
      pick.push_back(*it);
      it = s->waiting.erase(it);
    }
    if (pick.empty()) break;
    const int rc = launch_slot(s, sl, pick);
    if (rc != ENS_OK) return rc;
  }
  return ENS_OK;
}

}  // namespace

extern "C" {

int ensemble_server_create(void* pool, size_t pool_bytes, int32_t n_slots, ens_server** out) {
  if (!pool || !out) return fail(ENS_EINVAL, "pool and out are required");
  if (((uintptr_t)pool & 255) != 0) return fail(ENS_EINVAL, "pool must be 256-byte aligned");
  if (n_slots < 1 || n_slots > SERVE_MAX_SLOTS)
    return fail(ENS_EINVAL, "n_slots must be in [1, %d]", SERVE_MAX_SLOTS);
  const size_t ctrl_per = align256(SERVE_MAX_JOBS * sizeof(ServeJob)) +
                          align256(SERVE_MAX_JOBS * sizeof(int)) + 256;
  const size_t ctrl = ctrl_per * n_slots;
  if (pool_bytes < ctrl + (1u << 20))
    return fail(ENS_EINVAL, "pool of %zu bytes is below the control area (%zu) + 1 MiB",
                pool_bytes, ctrl);
  ens_server* s = new ens_server();
  s->pool = (char*)pool;
  s->pool_bytes = pool_bytes;
  s->arena_base = (char*)pool + ctrl;
  s->arena.reset(pool_bytes - ctrl);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, dev);
  s->slots.resize(n_slots);
  char* c = (char*)pool;
  for (int k = 0; k < n_slots && e == hipSuccess; ++k) {
    Slot& sl = s->slots[k];
    sl.d_jobs = (ServeJob*)c;
    c += align256(SERVE_MAX_JOBS * sizeof(ServeJob));
    sl.d_flags = (int*)c;
    c += align256(SERVE_MAX_JOBS * sizeof(int));
    sl.d_next = (unsigned*)c;
    c += 256;
    e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_jobs, SERVE_MAX_JOBS * sizeof(ServeJob), 0);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_flags, SERVE_MAX_JOBS * sizeof(int), 0);
  }
  if (e != hipSuccess) {
    ensemble_server_destroy(s);
    return hip_fail(e, "server create");
  }
  *out = s;
  return ENS_OK;
}

int ensemble_server_submit(ens_server* s, const ens_job* job, int64_t* id) {
  if (!s || !job || !id) return fail(ENS_EINVAL, "bad arguments");
  SysInfo si;
  int rc;
  if ((rc = check_problem(&job->prob, &si)) != ENS_OK) return rc;
  if (job->prob.system == ENS_SYS_LV_UDE || job->prob.params_shared)
    return fail(ENS_EUNSUPPORTED, "served jobs have per-trajectory parameters (not the UDE)");
  if (job->prob.system >= ENS_SYS_USER_BASE)
    return fail(ENS_EUNSUPPORTED, "registered systems are not served");
  if ((rc = check_ivp(&job->ivp, true)) != ENS_OK) return rc;
  if (job->ivp.dense) return fail(ENS_EUNSUPPORTED, "served jobs save by the extra step (no dense output)");
  const ens_loss& L = job->loss;
  if (L.kind != ENS_LOSS_SUMSQ && L.kind != ENS_LOSS_MSE_TARGET && L.kind != ENS_LOSS_COTANGENT)
    return fail(ENS_EINVAL, "unknown loss kind %d", L.kind);
  if (L.kind != ENS_LOSS_SUMSQ && !L.data) return fail(ENS_EINVAL, "loss data is NULL");
  if (!job->y_save || !job->grad_params) return fail(ENS_EINVAL, "y_save and grad_params are required");
  if (job->steps_hint < 0) return fail(ENS_EINVAL, "steps_hint < 0");
  SrvJob J;
  J.desc = *job;
  if (job->ivp.n_save > 0) J.save_times.assign(job->ivp.save_times, job->ivp.save_times + job->ivp.n_save);
  J.desc.ivp.save_times = nullptr;
  J.hint = job->steps_hint > 0 ? job->steps_hint : 512;
  J.t_submit = now_s();
  if (s->t_first < 0) s->t_first = J.t_submit;
  *id = s->next_id++;
  s->jobs.emplace(*id, std::move(J));
  s->waiting.push_back(*id);
  ++s->submitted;
  return launch_waiting(s);
}

int ensemble_server_progress(ens_server* s, int32_t* n_active) {
  if (!s) return fail(ENS_EINVAL, "server is NULL");
  int rc = retire(s);
  if (rc == ENS_OK) rc = launch_waiting(s);
  if (n_active) {
    int32_t a = (int32_t)s->waiting.size();
    for (const Slot& sl : s->slots) a += sl.busy ? (int32_t)sl.ids.size() : 0;
    *n_active = a;
  }
  return rc;
}

int ensemble_server_poll(ens_server* s, int64_t id, int32_t* state) {
  if (!s || !state) return fail(ENS_EINVAL, "bad arguments");
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return fail(ENS_EINVAL, "unknown job %lld", (long long)id);
  *state = it->second.state;
  return ENS_OK;
}

int ensemble_server_wait(ens_server* s, int64_t id) {
  int32_t st = ENS_JOB_WAITING;
  int rc;
  while ((rc = ensemble_server_poll(s, id, &st)) == ENS_OK &&
         (st == ENS_JOB_WAITING || st == ENS_JOB_RUNNING)) {
    if ((rc = ensemble_server_progress(s, nullptr)) != ENS_OK) return rc;
    bool any = false;
    for (Slot& sl : s->slots) any |= sl.busy;
    if (!any && st == ENS_JOB_WAITING)
      return fail(ENS_ENOSPACE, "job %lld cannot be admitted", (long long)id);
  }
  return rc;
}

int ensemble_server_drain(ens_server* s) {
  if (!s) return fail(ENS_EINVAL, "server is NULL");
  for (;;) {
    int32_t a = 0;
    int rc = ensemble_server_progress(s, &a);
    if (rc != ENS_OK) return rc;
    if (a == 0) return ENS_OK;
    bool any = false;
    for (Slot& sl : s->slots) any |= sl.busy;
    if (!any) return fail(ENS_ENOSPACE, "%d jobs cannot be admitted", a);
  }
}

int ensemble_server_stats(const ens_server* s, ens_server_stats* out) {
  if (!s || !out) return fail(ENS_EINVAL, "bad arguments");
  memset(out, 0, sizeof *out);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->retried = s->retried;
  out->waiting = (int64_t)s->waiting.size();
  for (const Slot& sl : s->slots) out->running += sl.busy ? (int64_t)sl.ids.size() : 0;
  out->lanes_completed = s->lanes;
  std::vector<double> lat = s->latencies;
  std::sort(lat.begin(), lat.end());
  if (!lat.empty()) {
    auto q = [&](double f) {
      const size_t k = (size_t)std::min<double>(lat.size() - 1, std::ceil(f * lat.size()) - 1);
      return lat[k];
    };
    out->p50_latency_s = q(0.50);
    out->p99_latency_s = q(0.99);
    double sum = 0;
    for (double x : lat) sum += x;
    out->mean_latency_s = sum / lat.size();
  }
  out->busy_s = (s->t_first >= 0 && s->t_last >= s->t_first) ? s->t_last - s->t_first : 0.0;
  out->throughput = out->busy_s > 0 ? s->lanes / out->busy_s : 0.0;
  out->pool_in_use = s->arena.used();
  out->pool_peak = s->arena.peak();
  out->pool_arena = s->arena.size();
  return ENS_OK;
}

int ensemble_server_destroy(ens_server* s) {
  if (!s) return ENS_OK;
  for (Slot& sl : s->slots) {  // teardown: errors here have nowhere to go
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.h_jobs) (void)hipHostFree(sl.h_jobs);
    if (sl.h_flags) (void)hipHostFree(sl.h_flags);
  }
  delete s;
  return ENS_OK;
}

}  // extern "C"
