// Serving: many propagations overlapped on one GPU (continuous batching).
//
// A server owns one caller-provided device arena and a fixed number of slots
// (one HIP stream each).  vgtb_server_run takes a list of requests with
// arrival times and drives them to completion:
//   - arrival: a request joins the waiting queue when its arrival time has
//     passed on the server's clock;
//   - admission (FIFO): the head of the queue is admitted when a slot is free
//     and its workspace (vgtb_workspace_size) fits in the arena, first fit;
//   - initialisation (S_k^-1, ground state, field table) runs on a worker
//     thread, so the main loop keeps the running requests fed meanwhile;
//   - stepping: every running request has up to kDepth chunks of kChunk steps
//     queued on its own stream, so the requests' kernels overlap on the GPU;
//   - completion: the current history is read, the spectrum of Eqs. 15-16 is
//     computed (vgtb_spectrum), the results are copied to the request's host
//     buffers, and the slot and the arena range are released, which may admit
//     the next waiting request.
// Every context is independent and its kernels are deterministic, so a result
// does not depend on what else is running.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "vgtb.h"

namespace {

using Clock = std::chrono::steady_clock;
constexpr int64_t kChunk = 64;   // steps per vgtb_step call
constexpr size_t kDepth = 2;     // chunks queued per running request

// First-fit sub-allocator over the arena in 256-byte granules; freed ranges
// coalesce with their neighbours.
class ArenaAlloc {
 public:
  explicit ArenaAlloc(size_t capacity) { free_[0] = capacity & ~size_t(255); }
  bool take(size_t bytes, size_t &off) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      off = it->first;
      const size_t rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void give(size_t off, size_t bytes) {
    bytes = round(bytes);
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
  size_t peak() const { return peak_; }

 private:
  static size_t round(size_t b) { return (b + 255) & ~size_t(255); }
  std::map<size_t, size_t> free_;
  size_t used_ = 0, peak_ = 0;
};

struct Job {
  const vgtb_request *rq = nullptr;
  vgtb_options opt{};
  size_t ws = 0, off = 0;
  int slot = -1;
  vgtb_ctx *ctx = nullptr;
  int64_t issued = 0;
  std::deque<hipEvent_t> inflight;
  vgtb_status status = VGTB_OK;
  double t_admit = 0, t_ready = 0, t_done = 0;
};

}  // namespace

struct vgtb_server {
  char *arena = nullptr;
  size_t bytes = 0;
  int device = 0;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;   // idle events, reused
};

namespace {

hipEvent_t get_event(vgtb_server *s) {
  if (!s->events.empty()) {
    hipEvent_t e = s->events.back();
    s->events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

// Initialisation of one admitted request (worker thread).
void init_job(vgtb_server *s, Job *j) {
  (void)hipSetDevice(s->device);
  vgtb_status st = vgtb_create(j->rq->system, &j->opt, s->arena + j->off, j->ws,
                               s->streams[j->slot], &j->ctx);
  if (st == VGTB_OK) st = vgtb_ground_state(j->ctx, nullptr);
  if (st == VGTB_OK) st = vgtb_set_field_table(j->ctx, j->rq->n_field, j->rq->field);
  j->status = st;
}

// Results of a finished request into its host buffers.
vgtb_status finish_job(Job *j) {
  const vgtb_request *rq = j->rq;
  const int64_t n = rq->n_steps;
  std::vector<double> jall((size_t)std::max<int64_t>(n, 1) * 3);
  vgtb_status st = vgtb_read_observables(j->ctx, 0, n, jall.data(), nullptr, nullptr, nullptr);
  if (st != VGTB_OK) return st;
  if (rq->j_out) std::memcpy(rq->j_out, jall.data(), sizeof(double) * 3 * (size_t)n);
  if (rq->sigma_out && rq->n_omega > 0) {
    std::vector<double> jx((size_t)n), eps(2 * (size_t)rq->n_omega);
    for (int64_t t = 0; t < n; ++t) jx[t] = jall[3 * t];
    st = vgtb_spectrum(j->ctx, n, jx.data(), j->opt.dt, rq->n_omega, rq->omega, rq->e0, rq->tau0, 1,
                       rq->sigma_out, eps.data());
  }
  return st;
}

}  // namespace

extern "C" {

vgtb_status vgtb_server_create(void *dev_arena, size_t arena_bytes, int32_t max_active,
                               vgtb_server **out) {
  if (!dev_arena || !out || arena_bytes == 0 || max_active < 1 || max_active > 64)
    return VGTB_E_INVAL;
  if (reinterpret_cast<uintptr_t>(dev_arena) % 256 != 0) return VGTB_E_INVAL;
  auto *s = new vgtb_server;
  s->arena = static_cast<char *>(dev_arena);
  s->bytes = arena_bytes;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return VGTB_E_DEVICE;
  }
  for (int i = 0; i < max_active; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      return VGTB_E_DEVICE;
    }
    s->streams.push_back(st);
  }
  *out = s;
  return VGTB_OK;
}

vgtb_status vgtb_server_run(vgtb_server *s, int32_t n, const vgtb_request *reqs,
                            vgtb_request_stats *stats, vgtb_server_stats *summary) {
  if (!s || n < 0 || (n > 0 && !reqs)) return VGTB_E_INVAL;
  (void)hipSetDevice(s->device);
  std::vector<Job> jobs((size_t)n);
  for (int i = 0; i < n; ++i) {
    Job &j = jobs[i];
    j.rq = &reqs[i];
    j.opt = reqs[i].options;
    if (!reqs[i].system || reqs[i].n_steps < 1 || reqs[i].n_field < 1 || !reqs[i].field ||
        (reqs[i].n_omega > 0 && !reqs[i].omega)) {
      j.status = VGTB_E_INVAL;
      continue;
    }
    // The whole history is kept so that J(t) can be returned and transformed.
    j.opt.history_capacity = (int32_t)std::min<int64_t>(reqs[i].n_steps, INT32_MAX);
    j.status = vgtb_workspace_size(reqs[i].system, &j.opt, &j.ws);
    if (j.status == VGTB_OK && j.ws > s->bytes) j.status = VGTB_E_NOMEM;
  }
  std::vector<int> order((size_t)n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return reqs[a].arrival_s < reqs[b].arrival_s; });

  ArenaAlloc alloc(s->bytes);
  std::vector<bool> slot_busy(s->streams.size(), false);
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Job *> init_q, ready_q;
  bool stop = false;
  std::thread worker([&] {
    for (;;) {
      Job *j = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return stop || !init_q.empty(); });
        if (init_q.empty()) return;
        j = init_q.front();
        init_q.pop_front();
      }
      init_job(s, j);
      std::lock_guard<std::mutex> lk(mu);
      ready_q.push_back(j);
    }
  });

  const auto t0 = Clock::now();
  auto now_s = [&] { return std::chrono::duration<double>(Clock::now() - t0).count(); };
  size_t next = 0;
  int done = 0, peak_active = 0, running_now = 0;
  std::deque<Job *> waiting;
  std::vector<Job *> running;
  double k_steps = 0.0;
  auto release = [&](Job *j) {
    if (j->ctx) vgtb_destroy(j->ctx);
    j->ctx = nullptr;
    for (auto e : j->inflight) s->events.push_back(e);
    j->inflight.clear();
    if (j->slot >= 0) {
      alloc.give(j->off, j->ws);
      slot_busy[j->slot] = false;
      --running_now;
    }
    j->t_done = now_s();
    ++done;
  };
  while (done < n) {
    bool progress = false;
    const double t = now_s();
    while (next < order.size() && reqs[order[next]].arrival_s <= t) {
      waiting.push_back(&jobs[order[next++]]);
      progress = true;
    }
    // Admission, first come first served.
    while (!waiting.empty()) {
      Job *j = waiting.front();
      if (j->status != VGTB_OK) {   // invalid or larger than the arena
        waiting.pop_front();
        j->t_admit = now_s();
        release(j);
        progress = true;
        continue;
      }
      int slot = -1;
      for (size_t i = 0; i < slot_busy.size(); ++i)
        if (!slot_busy[i]) {
          slot = (int)i;
          break;
        }
      size_t off = 0;
      if (slot < 0 || !alloc.take(j->ws, off)) break;
      waiting.pop_front();
      slot_busy[slot] = true;
      j->slot = slot;
      j->off = off;
      j->t_admit = now_s();
      peak_active = std::max(peak_active, ++running_now);
      {
        std::lock_guard<std::mutex> lk(mu);
        init_q.push_back(j);
      }
      cv.notify_one();
      progress = true;
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      while (!ready_q.empty()) {
        Job *j = ready_q.front();
        ready_q.pop_front();
        j->t_ready = now_s();
        if (j->status == VGTB_OK) running.push_back(j);
        else release(j);
        progress = true;
      }
    }
    // Keep every running request fed, retire finished chunks, finish requests.
    for (size_t r = 0; r < running.size();) {
      Job *j = running[r];
      while (j->status == VGTB_OK && j->inflight.size() < kDepth && j->issued < j->rq->n_steps) {
        const int64_t ns = std::min<int64_t>(kChunk, j->rq->n_steps - j->issued);
        j->status = vgtb_step(j->ctx, ns);
        hipEvent_t e = get_event(s);
        if (j->status == VGTB_OK && (!e || hipEventRecord(e, s->streams[j->slot]) != hipSuccess))
          j->status = VGTB_E_DEVICE;
        if (e) j->inflight.push_back(e);
        j->issued += ns;
        progress = true;
      }
      while (!j->inflight.empty()) {
        const hipError_t q = hipEventQuery(j->inflight.front());
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) j->status = VGTB_E_DEVICE;
        s->events.push_back(j->inflight.front());
        j->inflight.pop_front();
        progress = true;
      }
      const bool all_issued = j->issued >= j->rq->n_steps;
      if (j->status != VGTB_OK || (all_issued && j->inflight.empty())) {
        if (j->status == VGTB_OK) j->status = vgtb_synchronize(j->ctx);
        if (j->status == VGTB_OK) j->status = finish_job(j);
        if (j->status == VGTB_OK) k_steps += (double)j->rq->system->n_k * (double)j->rq->n_steps;
        release(j);
        running.erase(running.begin() + r);
        progress = true;
        continue;
      }
      ++r;
    }
    if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(100));
  }
  {
    std::lock_guard<std::mutex> lk(mu);
    stop = true;
  }
  cv.notify_all();
  worker.join();
  double last = 0.0;
  for (int i = 0; i < n; ++i) {
    const Job &j = jobs[i];
    if (stats) {
      stats[i].status = j.status;
      stats[i].slot = j.slot;
      stats[i].workspace_bytes = j.ws;
      stats[i].arrival_s = reqs[i].arrival_s;
      stats[i].admitted_s = j.t_admit;
      stats[i].ready_s = j.t_ready;
      stats[i].finished_s = j.t_done;
    }
    last = std::max(last, j.t_done);
  }
  if (summary) {
    summary->makespan_s = n ? last : 0.0;
    summary->k_steps = k_steps;
    summary->k_steps_per_s = (n && last > 0.0) ? k_steps / last : 0.0;
    summary->peak_bytes = alloc.peak();
    summary->peak_active = peak_active;
  }
  return VGTB_OK;
}

void vgtb_server_destroy(vgtb_server *s) {
  if (!s) return;
  for (auto st : s->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (auto e : s->events) (void)hipEventDestroy(e);
  delete s;
}

}  // extern "C"
