// Scheduling core of the serving loop (continuous batching of propagation
// requests on one GPU), kept apart from every GPU call so that the same code
// can be built on the host against a stub engine and checked with the thread
// and address sanitizers.
//
//   - arrival: a request joins the FIFO when its arrival time has passed;
//   - admission: the head of the FIFO is admitted when a slot is free and its
//     workspace fits in the arena (first fit over 256-byte granules);
//   - initialisation runs on one worker thread, so the main loop keeps the
//     running requests fed meanwhile; the worker touches only the job it was
//     handed, and hands it back through a mutex-protected queue;
//   - stepping: every running request keeps up to kDepth chunks of kChunk
//     steps queued on its slot, each followed by a completion marker;
//   - completion: results are written, the job is destroyed, and its slot and
//     arena range are released, which may admit the next waiting request.
// Every failure is recorded per request (status and message); the others go on.
#pragma once

#include <algorithm>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <exception>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "vgtb.h"

namespace vgtb_srv {

// What the scheduler needs from the device side.  Thread use: init() runs on
// the worker thread, everything else on the thread that called run().
struct Engine {
  virtual ~Engine() = default;
  virtual vgtb_status workspace(const vgtb_request &rq, const vgtb_options &opt, size_t *bytes,
                                std::string &msg) = 0;
  // Initialise an admitted request in [off, off + bytes) of the arena, bound
  // to slot; *job is set on success (and may be set on failure, then destroy()
  // releases it).
  virtual vgtb_status init(const vgtb_request &rq, const vgtb_options &opt, size_t off, size_t bytes,
                           int slot, void **job, std::string &msg) = 0;
  virtual vgtb_status step(void *job, int64_t n, std::string &msg) = 0;
  // A marker after the work queued so far on the slot; poll(): 1 reached,
  // 0 not yet, -1 failed.  recycle() takes back a marker.
  virtual vgtb_status mark(int slot, void **marker, std::string &msg) = 0;
  virtual int poll(void *marker) = 0;
  virtual void recycle(void *marker) = 0;
  // Wait for the job's work and write the request's results.
  virtual vgtb_status finish(void *job, const vgtb_request &rq, const vgtb_options &opt,
                             std::string &msg) = 0;
  // Wait for the job's queued work, then release it.
  virtual void destroy(void *job) = 0;
};

constexpr int64_t kChunk = 64;   // steps per step() call
constexpr size_t kDepth = 2;     // chunks queued per running request

// First-fit sub-allocator in 256-byte granules; freed ranges coalesce.
class ArenaAlloc {
 public:
  explicit ArenaAlloc(size_t capacity) {
    const size_t c = capacity & ~size_t(255);
    if (c) free_[0] = c;
  }
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
  size_t used() const { return used_; }
  static size_t round(size_t b) { return (b + 255) & ~size_t(255); }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0, peak_ = 0;
};

struct Job {
  int index = 0;
  const vgtb_request *rq = nullptr;
  vgtb_options opt{};
  size_t ws = 0, off = 0;
  int slot = -1;
  void *job = nullptr;
  int64_t issued = 0;
  std::deque<void *> inflight;
  vgtb_status status = VGTB_OK;
  std::string msg;
  bool admitted = false;
  double t_admit = 0, t_ready = 0, t_done = 0;
};

inline void set_message(vgtb_request_stats &st, const std::string &m) {
  const size_t n = std::min(m.size(), sizeof(st.message) - 1);
  std::memcpy(st.message, m.data(), n);
  st.message[n] = '\0';
}

// Serve n requests with an arena of arena_bytes and n_slots slots; fills
// stats (n entries) and summary when they are not null.
inline vgtb_status run(Engine &eng, size_t arena_bytes, int n_slots, int n, const vgtb_request *reqs,
                       vgtb_request_stats *stats, vgtb_server_stats *summary) {
  using Clock = std::chrono::steady_clock;
  std::vector<Job> jobs((size_t)n);
  for (int i = 0; i < n; ++i) {
    Job &j = jobs[i];
    j.index = i;
    j.rq = &reqs[i];
    j.opt = reqs[i].options;
    if (!reqs[i].system || reqs[i].n_steps < 1 || reqs[i].n_field < 1 || !reqs[i].field ||
        (reqs[i].n_omega > 0 && !reqs[i].omega) || reqs[i].n_omega < 0) {
      j.status = VGTB_E_INVAL;
      j.msg = "request needs a system, n_steps >= 1, a field table of n_field >= 1 rows and an omega grid when n_omega > 0";
      continue;
    }
    // The whole history is kept so that J(t) can be returned and transformed.
    j.opt.history_capacity = (int32_t)std::min<int64_t>(reqs[i].n_steps, INT32_MAX);
    j.status = eng.workspace(reqs[i], j.opt, &j.ws, j.msg);
    if (j.status == VGTB_OK && ArenaAlloc::round(j.ws) > (arena_bytes & ~size_t(255))) {
      j.status = VGTB_E_NOMEM;
      j.msg = "workspace of " + std::to_string(j.ws) + " bytes exceeds the arena of " +
              std::to_string(arena_bytes);
    }
  }
  std::vector<int> order((size_t)n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return reqs[a].arrival_s < reqs[b].arrival_s; });

  ArenaAlloc alloc(arena_bytes);
  std::vector<bool> slot_busy((size_t)n_slots, false);
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Job *> init_q, ready_q;   // both guarded by mu
  bool stop = false;                   // guarded by mu
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
      // The worker owns *j until it is pushed onto ready_q.
      try {
        j->status = eng.init(*j->rq, j->opt, j->off, j->ws, j->slot, &j->job, j->msg);
      } catch (const std::exception &e) {
        j->status = VGTB_E_DEVICE;
        j->msg = std::string("initialisation threw: ") + e.what();
      } catch (...) {
        j->status = VGTB_E_DEVICE;
        j->msg = "initialisation threw";
      }
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
    if (j->job) eng.destroy(j->job);   // waits for the job's queued work
    j->job = nullptr;
    for (void *m : j->inflight) eng.recycle(m);
    j->inflight.clear();
    if (j->admitted) {
      alloc.give(j->off, j->ws);
      slot_busy[(size_t)j->slot] = false;
      --running_now;
    }
    j->t_done = now_s();
    ++done;
  };
  while (done < n) {
    bool progress = false;
    const double t = now_s();
    while (next < order.size() && reqs[order[next]].arrival_s <= t) {
      waiting.push_back(&jobs[(size_t)order[next++]]);
      progress = true;
    }
    // Admission, first come first served.
    while (!waiting.empty()) {
      Job *j = waiting.front();
      if (j->status != VGTB_OK) {   // invalid, or larger than the whole arena
        waiting.pop_front();
        j->t_admit = j->t_ready = now_s();
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
      slot_busy[(size_t)slot] = true;
      j->slot = slot;
      j->off = off;
      j->admitted = true;
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
      std::deque<Job *> ready;
      {
        std::lock_guard<std::mutex> lk(mu);
        ready.swap(ready_q);
      }
      for (Job *j : ready) {
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
        j->status = eng.step(j->job, ns, j->msg);
        if (j->status != VGTB_OK) break;
        void *m = nullptr;
        j->status = eng.mark(j->slot, &m, j->msg);
        if (m) j->inflight.push_back(m);
        j->issued += ns;
        progress = true;
      }
      while (!j->inflight.empty()) {
        const int q = eng.poll(j->inflight.front());
        if (q == 0) break;
        if (q < 0 && j->status == VGTB_OK) {
          j->status = VGTB_E_DEVICE;
          j->msg = "a queued chunk of steps failed on the device";
        }
        eng.recycle(j->inflight.front());
        j->inflight.pop_front();
        progress = true;
      }
      const bool all_issued = j->issued >= j->rq->n_steps;
      if (j->status != VGTB_OK || (all_issued && j->inflight.empty())) {
        if (j->status == VGTB_OK) j->status = eng.finish(j->job, *j->rq, j->opt, j->msg);
        if (j->status == VGTB_OK) k_steps += (double)j->rq->system->n_k * (double)j->rq->n_steps;
        release(j);
        running.erase(running.begin() + (long)r);
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
    const Job &j = jobs[(size_t)i];
    if (stats) {
      vgtb_request_stats &st = stats[i];
      st.status = j.status;
      st.slot = j.admitted ? j.slot : -1;
      st.workspace_bytes = j.ws;
      st.arrival_s = reqs[i].arrival_s;
      st.admitted_s = j.t_admit;
      st.ready_s = j.t_ready;
      st.finished_s = j.t_done;
      set_message(st, j.status == VGTB_OK ? std::string() : j.msg);
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

}  // namespace vgtb_srv
