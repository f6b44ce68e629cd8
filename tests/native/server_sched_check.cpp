// Host check of the serving scheduler (server_core.h) against a stub engine:
// no GPU, built with the thread sanitizer or the address + undefined-behaviour
// sanitizers by tests/test_server_host.py.
//
// The stub engine stands in for the device: every call sleeps or keeps a
// per-slot timeline instead of launching work, records which thread made it,
// and writes deterministic results.  The check runs a stream of requests with
// staggered arrivals through a small arena and a few slots, including an
// invalid request, one larger than the arena, one whose initialisation fails
// and one whose stepping fails, and verifies:
//   - every request ends with the expected status and a message when failed;
//   - the results of the good requests are exactly the stub's;
//   - at no admission did the resident requests exceed the arena;
//   - init() runs only on the worker thread, every other call on the caller's;
//   - every marker and job the engine handed out was given back.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "server_core.h"

namespace {

using Clock = std::chrono::steady_clock;

#define CHECK(cond)                                                              \
  do {                                                                           \
    if (!(cond)) {                                                               \
      std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #cond);    \
      std::exit(1);                                                              \
    }                                                                            \
  } while (0)

struct StubJob {
  const vgtb_request *rq;
  int slot;
  int64_t stepped = 0;
};
struct Marker {
  Clock::time_point ready;
};

class StubEngine : public vgtb_srv::Engine {
 public:
  explicit StubEngine(int slots) : busy_(slots, Clock::now()) {}
  std::thread::id main_id = std::this_thread::get_id();
  std::atomic<int> jobs_live{0}, markers_live{0}, inits{0};
  std::mutex mu;
  std::set<std::thread::id> init_threads;

  vgtb_status workspace(const vgtb_request &rq, const vgtb_options &, size_t *bytes,
                        std::string &msg) override {
    CHECK(std::this_thread::get_id() == main_id);
    if (rq.system->n_atoms <= 0) {
      msg = "stub: no atoms";
      return VGTB_E_INVAL;
    }
    *bytes = (size_t)rq.system->n_atoms * 4096 + 100;   // not a multiple of 256 on purpose
    return VGTB_OK;
  }
  vgtb_status init(const vgtb_request &rq, const vgtb_options &opt, size_t off, size_t bytes, int slot,
                   void **job, std::string &msg) override {
    CHECK(std::this_thread::get_id() != main_id);
    CHECK(opt.history_capacity == rq.n_steps);
    CHECK(off % 256 == 0 && bytes >= (size_t)rq.system->n_atoms * 4096);
    {
      std::lock_guard<std::mutex> lk(mu);
      init_threads.insert(std::this_thread::get_id());
    }
    ++inits;
    std::this_thread::sleep_for(std::chrono::microseconds(300 * (rq.system->n_atoms % 5)));
    *job = new StubJob{&rq, slot};
    ++jobs_live;
    if (rq.system->n_electrons < 0) {
      msg = "stub: initialisation failed";
      return VGTB_E_NOT_PD;
    }
    return VGTB_OK;
  }
  vgtb_status step(void *job, int64_t n, std::string &msg) override {
    CHECK(std::this_thread::get_id() == main_id);
    auto *j = static_cast<StubJob *>(job);
    CHECK(n >= 1 && n <= vgtb_srv::kChunk && j->stepped + n <= j->rq->n_steps);
    if (j->rq->system->n_k == 99 && j->stepped >= 64) {
      msg = "stub: step failed";
      return VGTB_E_DEVICE;
    }
    j->stepped += n;
    auto &b = busy_[(size_t)j->slot];
    b = std::max(b, Clock::now()) + std::chrono::microseconds(20 * n);
    return VGTB_OK;
  }
  vgtb_status mark(int slot, void **marker, std::string &) override {
    CHECK(std::this_thread::get_id() == main_id);
    *marker = new Marker{busy_[(size_t)slot]};
    ++markers_live;
    return VGTB_OK;
  }
  int poll(void *marker) override {
    CHECK(std::this_thread::get_id() == main_id);
    return Clock::now() >= static_cast<Marker *>(marker)->ready ? 1 : 0;
  }
  void recycle(void *marker) override {
    CHECK(std::this_thread::get_id() == main_id);
    delete static_cast<Marker *>(marker);
    --markers_live;
  }
  vgtb_status finish(void *job, const vgtb_request &rq, const vgtb_options &, std::string &) override {
    CHECK(std::this_thread::get_id() == main_id);
    auto *j = static_cast<StubJob *>(job);
    CHECK(j->stepped == rq.n_steps);
    for (int64_t t = 0; t < rq.n_steps; ++t)
      for (int a = 0; a < 3; ++a) rq.j_out[3 * t + a] = expected(rq, t, a);
    return VGTB_OK;
  }
  void destroy(void *job) override {
    CHECK(std::this_thread::get_id() == main_id);
    delete static_cast<StubJob *>(job);
    --jobs_live;
  }
  static double expected(const vgtb_request &rq, int64_t t, int a) {
    return rq.system->n_atoms * 1000.0 + (double)t + 0.25 * a;
  }

 private:
  std::vector<Clock::time_point> busy_;
};

}  // namespace

int main() {
  const int n_req = 40, slots = 3;
  const size_t arena = 24 * 4096 + 1000;   // room for a few of the requests at once
  std::vector<vgtb_system> systems((size_t)n_req);
  std::vector<vgtb_request> reqs((size_t)n_req);
  std::vector<std::vector<double>> jout((size_t)n_req);
  std::vector<double> field(3, 0.0);
  for (int i = 0; i < n_req; ++i) {
    vgtb_system &s = systems[(size_t)i];
    s = vgtb_system{};
    s.n_atoms = 1 + (i * 7) % 11;   // 1 .. 11 -> 4 KB .. 44 KB
    s.n_k = 1 + i % 4;
    s.n_electrons = 1.0;
    vgtb_request &r = reqs[(size_t)i];
    r = vgtb_request{};
    r.system = &s;
    r.n_steps = 50 + (i * 37) % 300;
    r.n_field = 1;
    r.field = field.data();
    r.arrival_s = 0.002 * (i % 9);
    jout[(size_t)i].assign((size_t)r.n_steps * 3, -1.0);
    r.j_out = jout[(size_t)i].data();
  }
  // Planted failures.
  systems[5].n_atoms = 0;                 // invalid (workspace)
  systems[6].n_atoms = 400;               // larger than the arena
  systems[7].n_electrons = -1.0;          // initialisation fails
  systems[8].n_k = 99;                    // stepping fails after one chunk
  reqs[9].n_steps = 0;                    // invalid request
  reqs[10].system = nullptr;              // invalid request

  StubEngine eng(slots);
  std::vector<vgtb_request_stats> stats((size_t)n_req);
  vgtb_server_stats summ{};
  CHECK(vgtb_srv::run(eng, arena, slots, n_req, reqs.data(), stats.data(), &summ) == VGTB_OK);

  double k_steps = 0.0;
  for (int i = 0; i < n_req; ++i) {
    const vgtb_request_stats &st = stats[(size_t)i];
    const vgtb_status want = i == 5 || i == 9 || i == 10 ? VGTB_E_INVAL
                             : i == 6                    ? VGTB_E_NOMEM
                             : i == 7                    ? VGTB_E_NOT_PD
                             : i == 8                    ? VGTB_E_DEVICE
                                                         : VGTB_OK;
    if (st.status != want) std::fprintf(stderr, "request %d: status %d, want %d (%s)\n", i, st.status, want, st.message);
    CHECK(st.status == want);
    CHECK((st.message[0] != '\0') == (want != VGTB_OK));
    CHECK(st.arrival_s <= st.admitted_s + 1e-9 && st.admitted_s <= st.ready_s && st.ready_s <= st.finished_s);
    if (want == VGTB_OK) {
      k_steps += (double)systems[(size_t)i].n_k * (double)reqs[(size_t)i].n_steps;
      for (int64_t t = 0; t < reqs[(size_t)i].n_steps; ++t)
        for (int a = 0; a < 3; ++a)
          CHECK(jout[(size_t)i][(size_t)(3 * t + a)] == StubEngine::expected(reqs[(size_t)i], t, a));
    }
    if (i == 5 || i == 6 || i == 9 || i == 10) CHECK(st.slot == -1);
  }
  // Footprint: whenever a request was admitted, the requests then resident fit.
  for (int i = 0; i < n_req; ++i) {
    if (stats[(size_t)i].slot < 0) continue;
    size_t resident = 0;
    int in_slots = 0;
    for (int k = 0; k < n_req; ++k) {
      const vgtb_request_stats &o = stats[(size_t)k];
      if (o.slot >= 0 && o.admitted_s <= stats[(size_t)i].admitted_s && stats[(size_t)i].admitted_s < o.finished_s) {
        resident += vgtb_srv::ArenaAlloc::round(o.workspace_bytes);
        ++in_slots;
      }
    }
    CHECK(resident <= arena);
    CHECK(in_slots <= slots);
  }
  CHECK(summ.k_steps == k_steps);
  CHECK(summ.peak_active >= 2 && summ.peak_active <= slots);
  CHECK(summ.peak_bytes <= arena);
  CHECK(eng.jobs_live == 0 && eng.markers_live == 0);
  CHECK(eng.inits == n_req - 4);
  CHECK(eng.init_threads.size() == 1);
  std::printf("server scheduler host check: %d requests, makespan %.3f s, peak %d active, %zu bytes: OK\n",
              n_req, summ.makespan_s, summ.peak_active, (size_t)summ.peak_bytes);
  return 0;
}
