// Continuous-batching calibration server.
//
// Requests (one full calibration each, e.g. one per frequency band - the paper's setting of
// many more bands than nodes, abstract and Section 1) are admitted while others run:
//   * admission by HBM footprint: the server owns one device arena of the configured budget
//     and a request is admitted only when its exact workspace (coherencies, residual, normal
//     matrix, factor, scratch) fits in a free range (first fit), in arrival order;
//   * each admitted request occupies one slot: a library context with its own HIP stream
//     whose workspace is lent from the arena, so solves of different sizes run side by side
//     and their kernels overlap on the device;
//   * the predict and the initial residual (R = V - sum_k J_k C_k J_k^H) of every request
//     admitted in the same scheduling round are fused into persistent batched launches on a
//     shared stream, which the slots' streams wait on before their SAGE sweeps start.
// One scheduler thread owns every HIP call of the server; submit/wait only touch the
// request table.  All reductions in the path have a fixed order, so a solve's result does
// not depend on what else is running (bitwise).
#include "host_internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

using namespace ddc;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

constexpr int kJobRing = 16;
constexpr int kMaxJobsPerBatch = 256;

struct Req {
  ddc_obs obs{};
  ddc_sky sky{};
  std::vector<int32_t> offs;
  const void* vis = nullptr;
  double* jones = nullptr;
  ddc_cal_opts opts{};
  int64_t bytes = 0;
  size_t arena_off = 0;
  ObsDev od{};
  host::CalBufs cb;
  int slot = -1;
  int state = 0;                 // 0 pending, 1 running, 2 done
  ddc_status status = DDC_OK;
  std::string err;
  std::vector<ddc_lm_info> info;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

struct Slot {
  ddc_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ready = nullptr;
  hipEvent_t done = nullptr;
  int64_t req = -1;
};

struct JobBuf {
  PredictJob* dev = nullptr;
  ResidualJob* rdev = nullptr;
  hipEvent_t used = nullptr;
  std::vector<PredictJob> host;
  std::vector<ResidualJob> rhost;
  bool pending = false;
};

}  // namespace

struct ddc_server {
  int device = 0;
  int64_t budget = 0;
  char* arena = nullptr;
  std::map<size_t, size_t> free_list;        // offset -> size
  int64_t in_use = 0, peak = 0;
  hipStream_t batch_stream = nullptr;
  hipEvent_t batch_ev = nullptr;
  JobBuf ring[kJobRing];
  int ring_next = 0;
  int grid = 1024;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_submit, cv_done;
  std::deque<int64_t> pending;
  std::unordered_map<int64_t, Req> reqs;
  std::thread th;
  bool stop = false;
  int64_t next_id = 1;
  int64_t completed = 0;
  int max_running = 0;
  std::string err;
};

namespace {

ddc_status sfail(ddc_server* s, ddc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (s) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->err = buf;
  }
  return st;
}

// First-fit range allocator over the arena (256-byte granules).
bool arena_alloc(ddc_server* s, size_t bytes, size_t& off) {
  bytes = (bytes + 255) / 256 * 256;
  for (auto it = s->free_list.begin(); it != s->free_list.end(); ++it) {
    if (it->second >= bytes) {
      off = it->first;
      const size_t rest = it->second - bytes;
      s->free_list.erase(it);
      if (rest) s->free_list[off + bytes] = rest;
      s->in_use += (int64_t)bytes;
      s->peak = std::max(s->peak, s->in_use);
      return true;
    }
  }
  return false;
}

void arena_free(ddc_server* s, size_t off, size_t bytes) {
  bytes = (bytes + 255) / 256 * 256;
  s->in_use -= (int64_t)bytes;
  auto it = s->free_list.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != s->free_list.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    s->free_list.erase(nx);
  }
  if (it != s->free_list.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      s->free_list.erase(it);
    }
  }
}

void finish(ddc_server* s, Req& r, ddc_status st, const char* msg) {
  std::lock_guard<std::mutex> lk(s->mu);
  r.status = st;
  if (msg) r.err = msg;
  r.state = 2;
  r.t_done = now_s();
  s->completed += 1;
  s->cv_done.notify_all();
}

// Retire finished slots: copy reports, return the arena range, free the slot.
void retire(ddc_server* s, bool& any) {
  for (size_t i = 0; i < s->slots.size(); ++i) {
    Slot& sl = s->slots[i];
    if (sl.req < 0) continue;
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    any = true;
    Req* r;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      r = &s->reqs[sl.req];
    }
    ddc_status st = DDC_OK;
    const char* msg = nullptr;
    if (q != hipSuccess) {
      st = DDC_EDEVICE;
      msg = hipGetErrorString(q);
    } else {
      st = host::collect_infos(sl.ctx, r->cb, r->info.data(), nullptr);
      if (st != DDC_OK) msg = host::ctx_error(sl.ctx);
    }
    host::release_calibrate(r->cb);
    host::ctx_lend_workspace(sl.ctx, nullptr, 0);
    arena_free(s, r->arena_off, (size_t)r->bytes);
    sl.req = -1;
    finish(s, *r, st, msg);
  }
}

// One batched predict over the jobs, then one batched initial residual of the same requests
// (which reads the coherencies the predict wrote), both on the batch stream.
template <typename R>
hipError_t launch_batch(ddc_server* s, std::vector<PredictJob>& jobs, std::vector<ResidualJob>& rjobs) {
  if (jobs.empty()) return hipSuccess;
  JobBuf& jb = s->ring[s->ring_next];
  s->ring_next = (s->ring_next + 1) % kJobRing;
  if (jb.pending) {
    hipError_t e = hipEventSynchronize(jb.used);
    if (e != hipSuccess) return e;
  }
  int64_t total = 0;
  for (auto& j : jobs) {
    j.first_block = total;
    total += predict_blocks(j);
  }
  int64_t rtotal = 0;
  for (auto& j : rjobs) {
    j.first_block = rtotal;
    rtotal += residual_blocks(j);
  }
  jb.host = jobs;
  jb.rhost = rjobs;
  hipError_t e = hipMemcpyAsync(jb.dev, jb.host.data(), jobs.size() * sizeof(PredictJob),
                                hipMemcpyHostToDevice, s->batch_stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(jb.rdev, jb.rhost.data(), rjobs.size() * sizeof(ResidualJob),
                       hipMemcpyHostToDevice, s->batch_stream);
  if (e != hipSuccess) return e;
  e = launch_predict_batch<R>(jb.dev, (int)jobs.size(), total, s->grid, s->batch_stream);
  if (e != hipSuccess) return e;
  e = launch_residual_batch<R>(jb.rdev, (int)rjobs.size(), rtotal, s->grid, s->batch_stream);
  if (e != hipSuccess) return e;
  e = hipEventRecord(jb.used, s->batch_stream);
  jb.pending = true;
  return e;
}

// Admit pending requests in arrival order while a slot and an arena range are free.
void admit(ddc_server* s, bool& any) {
  std::vector<std::pair<int, int64_t>> admitted;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    while (!s->pending.empty()) {
      int free_slot = -1;
      for (size_t i = 0; i < s->slots.size(); ++i)
        if (s->slots[i].req < 0) {
          bool taken = false;
          for (auto& a : admitted) taken = taken || a.first == (int)i;
          if (!taken) {
            free_slot = (int)i;
            break;
          }
        }
      if (free_slot < 0) break;
      Req& r = s->reqs[s->pending.front()];
      size_t off = 0;
      if (!arena_alloc(s, (size_t)r.bytes, off)) break;
      r.arena_off = off;
      r.slot = free_slot;
      r.state = 1;
      r.t_admit = now_s();
      admitted.push_back({free_slot, s->pending.front()});
      s->pending.pop_front();
    }
    int running = 0;
    for (auto& sl : s->slots) running += sl.req >= 0;
    s->max_running = std::max(s->max_running, running + (int)admitted.size());
  }
  if (admitted.empty()) return;
  any = true;
  std::vector<PredictJob> jobs32, jobs64;
  std::vector<ResidualJob> res32, res64;
  std::vector<std::pair<int, int64_t>> started;
  for (auto& a : admitted) {
    Slot& sl = s->slots[a.first];
    Req* r;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      r = &s->reqs[a.second];
    }
    host::ctx_lend_workspace(sl.ctx, s->arena + r->arena_off, (size_t)r->bytes);
    ddc_status st = ddc_set_stream(sl.ctx, sl.stream);
    if (st == DDC_OK) st = host::ctx_obs(sl.ctx, &r->obs, r->od);
    if (st == DDC_OK) st = host::prepare_calibrate(sl.ctx, r->od, &r->sky, r->opts.n_sweeps,
                                                   r->opts.lm.n_iter,
                                                   r->opts.lm.precision, r->cb);
    if (st == DDC_OK && hipEventRecord(sl.ready, sl.stream) != hipSuccess) st = DDC_EDEVICE;
    if (st == DDC_OK && hipStreamWaitEvent(s->batch_stream, sl.ready, 0) != hipSuccess) st = DDC_EDEVICE;
    if (st != DDC_OK) {
      std::string msg = host::ctx_error(sl.ctx);
      host::release_calibrate(r->cb);
      host::ctx_lend_workspace(sl.ctx, nullptr, 0);
      arena_free(s, r->arena_off, (size_t)r->bytes);
      finish(s, *r, st, msg.c_str());
      continue;
    }
    PredictJob j = make_predict_job(r->od, r->sky.n_clusters, r->cb.doffs, r->sky.l, r->sky.m,
                                    r->sky.I, r->sky.Q, r->sky.U, r->sky.V, r->cb.coh);
    ResidualJob rj;
    rj.vis = r->vis;
    rj.coh = r->cb.coh;
    rj.jones = r->jones;
    rj.ant_p = r->od.ant_p;
    rj.ant_q = r->od.ant_q;
    rj.out = r->cb.Rb;
    rj.B = r->od.B;
    rj.plane = (int64_t)r->od.T * r->od.F * r->od.B;
    rj.N = r->od.N;
    rj.K = r->sky.n_clusters;
    rj.first_block = 0;
    const bool mixed = r->opts.lm.precision == DDC_MIXED;
    (mixed ? jobs32 : jobs64).push_back(j);
    (mixed ? res32 : res64).push_back(rj);
    started.push_back(a);
  }
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < jobs32.size() && e == hipSuccess; i += kMaxJobsPerBatch) {
    const size_t i1 = std::min(jobs32.size(), i + kMaxJobsPerBatch);
    std::vector<PredictJob> part(jobs32.begin() + i, jobs32.begin() + i1);
    std::vector<ResidualJob> rpart(res32.begin() + i, res32.begin() + i1);
    e = launch_batch<float>(s, part, rpart);
  }
  for (size_t i = 0; i < jobs64.size() && e == hipSuccess; i += kMaxJobsPerBatch) {
    const size_t i1 = std::min(jobs64.size(), i + kMaxJobsPerBatch);
    std::vector<PredictJob> part(jobs64.begin() + i, jobs64.begin() + i1);
    std::vector<ResidualJob> rpart(res64.begin() + i, res64.begin() + i1);
    e = launch_batch<double>(s, part, rpart);
  }
  if (e == hipSuccess) e = hipEventRecord(s->batch_ev, s->batch_stream);
  for (auto& a : started) {
    Slot& sl = s->slots[a.first];
    Req* r;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      r = &s->reqs[a.second];
    }
    ddc_status st = e == hipSuccess ? DDC_OK : DDC_EDEVICE;
    if (st == DDC_OK && hipStreamWaitEvent(sl.stream, s->batch_ev, 0) != hipSuccess) st = DDC_EDEVICE;
    if (st == DDC_OK) st = host::enqueue_sage(sl.ctx, r->od, r->vis, r->jones, r->opts, r->cb, true);
    if (st == DDC_OK && hipEventRecord(sl.done, sl.stream) != hipSuccess) st = DDC_EDEVICE;
    if (st != DDC_OK) {
      // the request's predict may already be queued on the batch stream, writing into its
      // arena range: both streams must be idle before the range can be handed out again
      (void)hipStreamSynchronize(s->batch_stream);
      (void)hipStreamSynchronize(sl.stream);
      std::string msg = e != hipSuccess ? hipGetErrorString(e) : host::ctx_error(sl.ctx);
      host::release_calibrate(r->cb);
      host::ctx_lend_workspace(sl.ctx, nullptr, 0);
      arena_free(s, r->arena_off, (size_t)r->bytes);
      finish(s, *r, st, msg.c_str());
      continue;
    }
    sl.req = a.second;
  }
}

void scheduler(ddc_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    bool any = false;
    retire(s, any);
    admit(s, any);
    std::unique_lock<std::mutex> lk(s->mu);
    bool busy = false;
    for (auto& sl : s->slots) busy = busy || sl.req >= 0;
    if (s->stop && s->pending.empty() && !busy) break;
    if (!any) {
      if (busy) s->cv_submit.wait_for(lk, std::chrono::microseconds(50));
      else if (s->pending.empty()) s->cv_submit.wait(lk, [&] { return s->stop || !s->pending.empty(); });
      else s->cv_submit.wait_for(lk, std::chrono::microseconds(200));
    }
  }
}

ddc_status check_request(ddc_server* s, const ddc_obs* obs, const ddc_sky* sky, const void* vis,
                         double* jones, const ddc_cal_opts* opts) {
  if (!obs || !sky || !vis || !jones || !opts) return sfail(s, DDC_EINVAL, "null request argument");
  if (obs->n_stations < 2 || obs->n_times < 1 || obs->n_chans < 1 || 8 * (int64_t)obs->n_stations > 32768)
    return sfail(s, DDC_EINVAL, "bad observation sizes");
  if (!obs->u || !obs->v || !obs->w || !obs->freq_hz) return sfail(s, DDC_EINVAL, "obs arrays must not be NULL");
  if (sky->n_clusters < 1 || !sky->cluster_offset || sky->cluster_offset[0] != 0)
    return sfail(s, DDC_EINVAL, "n_clusters >= 1 and cluster_offset[0] = 0 required");
  for (int k = 0; k < sky->n_clusters; ++k)
    if (sky->cluster_offset[k + 1] < sky->cluster_offset[k])
      return sfail(s, DDC_EINVAL, "cluster_offset must be non-decreasing");
  if (sky->cluster_offset[sky->n_clusters] > 0 &&
      (!sky->l || !sky->m || !sky->I || !sky->Q || !sky->U || !sky->V))
    return sfail(s, DDC_EINVAL, "sky arrays must not be NULL");
  if (opts->n_sweeps < 0 || opts->lm.n_iter < 0 || opts->lm.refine_max < 0 || opts->lm.refine_max > 8 ||
      (opts->lm.precision != DDC_FP64 && opts->lm.precision != DDC_MIXED) || !(opts->lm.tau > 0.0) ||
      !(opts->lm.mu_floor >= 0.0) || !(opts->lm.refine_tol >= 0.0))
    return sfail(s, DDC_EINVAL, "bad calibration options");
  return DDC_OK;
}

ObsDev size_only(const ddc_obs* obs) {
  ObsDev o{};
  o.N = obs->n_stations;
  o.T = obs->n_times;
  o.F = obs->n_chans;
  o.B = (int64_t)o.N * (o.N - 1) / 2;
  return o;
}

}  // namespace

extern "C" {

int64_t ddc_calibrate_footprint(const ddc_obs* obs, int32_t n_clusters, int32_t n_sweeps,
                                int32_t n_iter, int32_t precision) {
  if (!obs || obs->n_stations < 2 || obs->n_times < 1 || obs->n_chans < 1 || n_clusters < 1 ||
      n_sweeps < 0 || n_iter < 0 || (precision != DDC_FP64 && precision != DDC_MIXED))
    return -1;
  return host::calibrate_footprint(size_only(obs), n_clusters, n_sweeps, n_iter, precision);
}

ddc_status ddc_server_create(ddc_server** out, int32_t device, int32_t n_slots,
                             int64_t hbm_budget_bytes) {
  if (!out || n_slots < 1 || n_slots > 64 || hbm_budget_bytes < (64 << 10)) return DDC_EINVAL;
  *out = nullptr;
  ddc_server* s = new ddc_server();
  s->device = device;
  s->budget = hbm_budget_bytes;
  if (hipSetDevice(device) != hipSuccess ||
      hipMalloc(&s->arena, (size_t)hbm_budget_bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete s;
    return DDC_ENOMEM;
  }
  s->free_list[0] = (size_t)hbm_budget_bytes / 256 * 256;
  bool ok = hipStreamCreateWithFlags(&s->batch_stream, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&s->batch_ev, hipEventDisableTiming) == hipSuccess;
  for (auto& jb : s->ring) {
    ok = ok && hipMalloc(&jb.dev, kMaxJobsPerBatch * sizeof(PredictJob)) == hipSuccess &&
         hipMalloc(&jb.rdev, kMaxJobsPerBatch * sizeof(ResidualJob)) == hipSuccess &&
         hipEventCreateWithFlags(&jb.used, hipEventDisableTiming) == hipSuccess;
  }
  s->slots.resize(n_slots);
  for (auto& sl : s->slots) {
    ok = ok && ddc_create(&sl.ctx, device) == DDC_OK &&
         hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&sl.ready, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
  }
  hipDeviceProp_t prop;
  if (ok && hipGetDeviceProperties(&prop, device) == hipSuccess) s->grid = 4 * prop.multiProcessorCount;
  if (!ok) {
    (void)hipGetLastError();
    s->stop = true;
    ddc_server_destroy(s);
    return DDC_EDEVICE;
  }
  s->th = std::thread(scheduler, s);
  *out = s;
  return DDC_OK;
}

ddc_status ddc_server_destroy(ddc_server* s) {
  if (!s) return DDC_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_submit.notify_all();
  if (s->th.joinable()) s->th.join();
  (void)hipSetDevice(s->device);
  for (auto& sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.ctx) ddc_destroy(sl.ctx);
    if (sl.ready) (void)hipEventDestroy(sl.ready);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  if (s->batch_stream) (void)hipStreamSynchronize(s->batch_stream);
  for (auto& jb : s->ring) {
    if (jb.dev) (void)hipFree(jb.dev);
    if (jb.rdev) (void)hipFree(jb.rdev);
    if (jb.used) (void)hipEventDestroy(jb.used);
  }
  if (s->batch_ev) (void)hipEventDestroy(s->batch_ev);
  if (s->batch_stream) (void)hipStreamDestroy(s->batch_stream);
  if (s->arena) (void)hipFree(s->arena);
  delete s;
  return DDC_OK;
}

ddc_status ddc_server_submit(ddc_server* s, const ddc_obs* obs, const ddc_sky* sky,
                             const void* vis, double* jones, const ddc_cal_opts* opts,
                             int64_t* id) {
  if (!s || !id) return DDC_EINVAL;
  ddc_status st = check_request(s, obs, sky, vis, jones, opts);
  if (st != DDC_OK) return st;
  const int64_t bytes = ddc_calibrate_footprint(obs, sky->n_clusters, opts->n_sweeps,
                                                opts->lm.n_iter, opts->lm.precision);
  if (bytes < 0 || bytes > s->budget)
    return sfail(s, DDC_ENOMEM, "request needs %lld bytes, budget is %lld", (long long)bytes, (long long)s->budget);
  std::lock_guard<std::mutex> lk(s->mu);
  const int64_t rid = s->next_id++;
  Req& r = s->reqs[rid];
  r.obs = *obs;
  r.offs.assign(sky->cluster_offset, sky->cluster_offset + sky->n_clusters + 1);
  r.sky = *sky;
  r.sky.cluster_offset = r.offs.data();
  r.vis = vis;
  r.jones = jones;
  r.opts = *opts;
  r.bytes = bytes;
  r.info.resize((size_t)std::max(1, opts->n_sweeps * sky->n_clusters));
  r.t_submit = now_s();
  s->pending.push_back(rid);
  *id = rid;
  s->cv_submit.notify_all();
  return DDC_OK;
}

ddc_status ddc_server_wait(ddc_server* s, int64_t id, ddc_lm_info* info, double* latency_s,
                           double* queue_s) {
  if (!s) return DDC_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) {
    s->err = "unknown request id";
    return DDC_EINVAL;
  }
  s->cv_done.wait(lk, [&] { return it->second.state == 2; });
  Req& r = it->second;
  if (info) std::copy(r.info.begin(), r.info.end(), info);
  if (latency_s) *latency_s = r.t_done - r.t_submit;
  if (queue_s) *queue_s = r.t_admit > 0 ? r.t_admit - r.t_submit : 0.0;
  const ddc_status st = r.status;
  if (st != DDC_OK) s->err = r.err;
  s->reqs.erase(it);
  return st;
}

ddc_status ddc_server_stats(ddc_server* s, int64_t* completed, int32_t* max_running,
                            int64_t* peak_bytes) {
  if (!s) return DDC_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (completed) *completed = s->completed;
  if (max_running) *max_running = s->max_running;
  if (peak_bytes) *peak_bytes = s->peak;
  return DDC_OK;
}

const char* ddc_server_last_error(const ddc_server* s) { return s ? s->err.c_str() : "null server"; }

}  // extern "C"
