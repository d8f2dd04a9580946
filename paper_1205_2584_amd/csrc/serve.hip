// Request loop over cp_fit: FIFO admission against a device-memory budget,
// concurrent execution of admitted fits on per-slot streams, and a batch lane
// that runs the pending requests within the batched shapes in one
// cp_fit_batched launch while the next group collects.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "dgn.h"

namespace dgn {
dgn_ctx* ctx_over(int device, char* ws, size_t size);
size_t batched_ws_fit(const int64_t* dims, int R);
size_t batched_ws_call(int B);
}

namespace {

// First-fit allocator over [0, size) with 256-byte granularity.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }

 private:
  size_t size_, used_ = 0;
  std::map<size_t, size_t> free_;
};

struct Job {
  uint64_t id;
  dgn_request req;
  size_t need = 0, off = 0;
  double t_submit = 0, t_admit = 0;
};

// Largest batch the lane launches at once.
constexpr int kMaxLaneBatch = 1024;

bool lane_eligible(const dgn_request& r) {
  if (r.Y.order != 3 || (r.Y.dtype != DGN_F32 && r.Y.dtype != DGN_F64) || r.R < 1 || r.R > 8) return false;
  for (int n = 0; n < 3; ++n)
    if (r.Y.dims[n] < 1 || r.Y.dims[n] > 64) return false;
  return true;
}

}  // namespace

struct dgn_server {
  int device = 0;
  char* base = nullptr;
  size_t budget = 0;
  int slots = 1;
  dgn_opts opts;
  Arena* arena = nullptr;
  std::mutex mu;
  std::condition_variable cv_sched, cv_work, cv_idle;
  std::deque<Job> queue;
  std::deque<Job> lane_queue;     // requests for the batch lane, in arrival order
  std::vector<Job*> slot_job;     // per worker: assigned job or null
  std::vector<dgn_result> done;
  int running = 0;
  bool stop = false;
  uint64_t next_id = 1;
  std::vector<std::thread> workers;
  std::thread sched;
  std::thread lane;
  std::condition_variable cv_lane;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

void scheduler(dgn_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    s->cv_sched.wait(lk, [&] {
      if (s->stop) return true;
      if (s->queue.empty()) return false;
      for (Job* j : s->slot_job)
        if (!j) return true;
      return false;
    });
    if (s->stop) return;
    // admit from the head while a slot is free and the head fits
    while (!s->queue.empty()) {
      int free_slot = -1;
      for (int k = 0; k < s->slots; ++k)
        if (!s->slot_job[k]) { free_slot = k; break; }
      if (free_slot < 0) break;
      Job& head = s->queue.front();
      size_t off;
      if (!s->arena->alloc(head.need, &off)) break;  // wait for memory to free up
      Job* j = new Job(head);
      s->queue.pop_front();
      j->off = off;
      j->t_admit = s->now();
      s->slot_job[free_slot] = j;
      ++s->running;
    }
    s->cv_work.notify_all();
    // sleep until something changes (a completion or a submission)
    s->cv_sched.wait(lk);
    if (s->stop) return;
  }
}

void worker(dgn_server* s, int k) {
  hipSetDevice(s->device);
  hipStream_t st;
  hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    s->cv_work.wait(lk, [&] { return s->stop || s->slot_job[k] != nullptr; });
    if (s->stop && !s->slot_job[k]) break;
    Job* j = s->slot_job[k];
    lk.unlock();
    dgn_ctx* ctx = dgn::ctx_over(s->device, s->base + j->off, j->need);
    dgn_result r{};
    r.id = j->id;
    r.tag = j->req.tag;
    r.t_submit = j->t_submit;
    r.t_admit = j->t_admit;
    r.status = cp_fit(ctx, &j->req.Y, j->req.R, j->req.A, j->req.mu0, j->req.tol, j->req.max_iters,
                      &s->opts, &r.info, st);
    r.t_done = s->now();
    r.lane = 0;
    r.batch_size = 1;
    dgn_destroy(ctx);
    lk.lock();
    s->arena->release(j->off, j->need);
    s->done.push_back(r);
    s->slot_job[k] = nullptr;
    --s->running;
    delete j;
    s->cv_sched.notify_all();
    s->cv_lane.notify_all();
    s->cv_idle.notify_all();
  }
  lk.unlock();
  hipStreamDestroy(st);
}

// The batch lane: take the pending lane requests that share the head's
// (tol, max_iters), as many as fit the free arena, run them as one persistent
// cp_fit_batched launch, then take the next group.
void lane_worker(dgn_server* s) {
  hipSetDevice(s->device);
  hipStream_t st;
  hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  dgn_opts o = s->opts;
  o.batched_launch = DGN_BATCH_PERSISTENT;
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    s->cv_lane.wait(lk, [&] { return s->stop || !s->lane_queue.empty(); });
    if (s->stop && s->lane_queue.empty()) break;
    const double tol = s->lane_queue.front().req.tol;
    const int32_t max_iters = s->lane_queue.front().req.max_iters;
    std::vector<size_t> pick;
    size_t fit_bytes = 0, need = 0;
    const size_t avail = s->budget - s->arena->used();
    for (size_t k = 0; k < s->lane_queue.size() && (int)pick.size() < kMaxLaneBatch; ++k) {
      const Job& j = s->lane_queue[k];
      if (j.req.tol != tol || j.req.max_iters != max_iters) continue;
      const size_t fb = fit_bytes + dgn::batched_ws_fit(j.req.Y.dims, j.req.R);
      const size_t tot = fb + dgn::batched_ws_call((int)pick.size() + 1);
      if (tot > avail && !pick.empty()) break;
      pick.push_back(k);
      fit_bytes = fb;
      need = tot;
    }
    size_t off = 0;
    if (!s->arena->alloc(need, &off)) {
      // wait for memory to free up (a slot or an earlier batch finishing)
      s->cv_lane.wait(lk);
      continue;
    }
    std::vector<Job> batch;
    batch.reserve(pick.size());
    for (size_t k : pick) batch.push_back(s->lane_queue[k]);
    for (size_t q = pick.size(); q-- > 0;) s->lane_queue.erase(s->lane_queue.begin() + (long)pick[q]);
    const double t_admit = s->now();
    s->running += (int)batch.size();
    lk.unlock();
    const int B = (int)batch.size();
    std::vector<dgn_batch_fit> fits(B);
    for (int b = 0; b < B; ++b) {
      fits[b].Y = batch[b].req.Y;
      fits[b].R = batch[b].req.R;
      fits[b].mu0 = batch[b].req.mu0;
      for (int n = 0; n < 3; ++n) fits[b].A[n] = batch[b].req.A[n];
    }
    std::vector<dgn_fit_info> infos(B);
    dgn_ctx* ctx = dgn::ctx_over(s->device, s->base + off, need);
    const double t_launch = s->now();
    const dgn_status rc = cp_fit_batched(ctx, B, fits.data(), tol, max_iters, &o, infos.data(), st);
    const double t_ret = s->now();
    dgn_destroy(ctx);
    lk.lock();
    s->arena->release(off, need);
    for (int b = 0; b < B; ++b) {
      dgn_result r{};
      r.id = batch[b].id;
      r.tag = batch[b].req.tag;
      r.t_submit = batch[b].t_submit;
      r.t_admit = t_admit;
      r.info = infos[b];
      // per-fit completion from the device clock inside the launch
      const double td = t_launch + infos[b].t_done;
      r.t_done = (rc == DGN_OK || rc == DGN_ENONFINITE) && td < t_ret ? td : t_ret;
      if (rc == DGN_OK || rc == DGN_ENONFINITE)
        r.status = infos[b].reason == DGN_STOP_NONFINITE ? DGN_ENONFINITE : DGN_OK;
      else
        r.status = rc;
      r.lane = 1;
      r.batch_size = B;
      s->done.push_back(r);
    }
    s->running -= B;
    s->cv_sched.notify_all();
    s->cv_lane.notify_all();
    s->cv_idle.notify_all();
  }
  lk.unlock();
  hipStreamDestroy(st);
}

}  // namespace

extern "C" {

dgn_status dgn_server_create(dgn_server** out, int32_t device, size_t budget_bytes,
                             int32_t max_slots, const dgn_opts* opts) {
  if (!out || max_slots < 1 || max_slots > 64 || budget_bytes < 4096) return DGN_EINVAL;
  *out = nullptr;
  if (opts && opts->mu_rule != DGN_MU_PAPER && opts->mu_rule != DGN_MU_NIELSEN) return DGN_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return DGN_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return DGN_EHIP;
  dgn_server* s = new dgn_server();
  s->device = device;
  s->budget = budget_bytes;
  s->slots = max_slots;
  dgn_opts_default(&s->opts);
  if (opts) s->opts = *opts;
  s->opts.timing = 0;
  if (hipMalloc((void**)&s->base, budget_bytes) != hipSuccess) {
    delete s;
    return DGN_ENOMEM;
  }
  s->arena = new Arena(budget_bytes);
  s->slot_job.assign(max_slots, nullptr);
  for (int k = 0; k < max_slots; ++k) s->workers.emplace_back(worker, s, k);
  s->sched = std::thread(scheduler, s);
  s->lane = std::thread(lane_worker, s);
  *out = s;
  return DGN_OK;
}

dgn_status dgn_server_submit(dgn_server* s, const dgn_request* req, uint64_t* id) {
  if (!s || !req) return DGN_EINVAL;
  size_t need = 0;
  dgn_status st = dgn_workspace_size(&req->Y, req->R, &s->opts, &need);
  if (st != DGN_OK) return st;
  if (req->max_iters < 0 || !(req->tol >= 0.0)) return DGN_EINVAL;
  for (int n = 0; n < req->Y.order; ++n)
    if (!req->A[n]) return DGN_EINVAL;
  const bool to_lane = s->opts.serve_batch != 0 && lane_eligible(*req) && std::isfinite(req->mu0);
  if (to_lane)
    need = dgn::batched_ws_fit(req->Y.dims, req->R) + dgn::batched_ws_call(1);  // as a batch of one
  else
    need += 1 << 20;
  if (need > s->budget) return DGN_EBUSY;
  std::lock_guard<std::mutex> lk(s->mu);
  Job j;
  j.id = s->next_id++;
  j.req = *req;
  j.need = need;
  j.t_submit = s->now();
  if (to_lane) {
    s->lane_queue.push_back(j);
    s->cv_lane.notify_all();
  } else {
    s->queue.push_back(j);
    s->cv_sched.notify_all();
  }
  if (id) *id = j.id;
  return DGN_OK;
}

dgn_status dgn_server_poll(dgn_server* s, dgn_result* out, int32_t max, int32_t* n) {
  if (!s || (!out && max > 0) || max < 0) return DGN_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  const int k = (int)std::min<size_t>(s->done.size(), (size_t)max);
  for (int i = 0; i < k; ++i) out[i] = s->done[i];
  s->done.erase(s->done.begin(), s->done.begin() + k);
  if (n) *n = k;
  return DGN_OK;
}

dgn_status dgn_server_wait_idle(dgn_server* s) {
  if (!s) return DGN_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_idle.wait(lk, [&] { return s->queue.empty() && s->lane_queue.empty() && s->running == 0; });
  return DGN_OK;
}

dgn_status dgn_server_stats(dgn_server* s, size_t* in_use, int32_t* running, int32_t* queued) {
  if (!s) return DGN_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (in_use) *in_use = s->arena->used();
  if (running) *running = s->running;
  if (queued) *queued = (int32_t)(s->queue.size() + s->lane_queue.size());
  return DGN_OK;
}

double dgn_server_now(const dgn_server* s) { return s ? s->now() : 0.0; }

dgn_status dgn_server_destroy(dgn_server* s) {
  if (!s) return DGN_EINVAL;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_idle.wait(lk, [&] { return s->running == 0; });
    s->queue.clear();
    s->lane_queue.clear();
    s->stop = true;
  }
  s->cv_sched.notify_all();
  s->cv_work.notify_all();
  s->cv_lane.notify_all();
  s->sched.join();
  s->lane.join();
  for (auto& t : s->workers) t.join();
  hipSetDevice(s->device);
  hipFree(s->base);
  delete s->arena;
  delete s;
  return DGN_OK;
}

}  // extern "C"
