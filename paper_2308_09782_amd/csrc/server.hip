// Serving: many propagations overlapped on one GPU (continuous batching).
//
// The scheduling (arrival, admission by arena footprint, the initialisation
// worker, chunked stepping, completion) is server_core.h; this file is its
// device side: one non-blocking stream per slot, the library's contexts
// carved from the server's arena, HIP events as chunk markers, and the
// results of a finished request (J(t) and the spectrum of Eqs. 15-16).
//
// Contexts of a server launch every step directly (VGTB_OPT_NO_GRAPHS): no
// stream capture runs while the worker thread initialises another request,
// and the requests' streams carry no cross-stream dependency.  SCC requests
// also stay off the small-system path: its workgroups meet at a grid-wide
// barrier, which needs every workgroup of the launch resident at once, and
// kernels of other requests on other streams may hold the compute units it
// waits for.  Every context is independent and its kernels are
// deterministic, so a result does not depend on what else is running.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "server_core.h"
#include "vgtb.h"

struct vgtb_server {
  char *arena = nullptr;
  size_t bytes = 0;
  int device = 0;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;   // idle markers, reused (main thread only)
};

namespace {

// The options every context of a server is created with (the same for its
// workspace size and its creation).
vgtb_options server_options(const vgtb_request &rq, const vgtb_options &opt) {
  vgtb_options o = opt;
  o.flags |= VGTB_OPT_NO_GRAPHS;
  if (rq.system && rq.system->gamma) o.flags |= VGTB_OPT_NO_SMALL_PATH;
  return o;
}

std::string ctx_error(vgtb_ctx *c, const char *what) {
  const char *m = vgtb_last_error(c);
  return std::string(what) + ": " + (m ? m : "");
}

class HipEngine : public vgtb_srv::Engine {
 public:
  explicit HipEngine(vgtb_server *s) : s_(s) {}

  vgtb_status workspace(const vgtb_request &rq, const vgtb_options &opt, size_t *bytes,
                        std::string &msg) override {
    const vgtb_options o = server_options(rq, opt);
    const vgtb_status st = vgtb_workspace_size(rq.system, &o, bytes);
    if (st != VGTB_OK) msg = ctx_error(nullptr, "vgtb_workspace_size");
    return st;
  }

  vgtb_status init(const vgtb_request &rq, const vgtb_options &opt, size_t off, size_t bytes, int slot,
                   void **job, std::string &msg) override {
    if (hipSetDevice(s_->device) != hipSuccess) {
      msg = "hipSetDevice failed on the initialisation thread";
      return VGTB_E_DEVICE;
    }
    const vgtb_options o = server_options(rq, opt);
    vgtb_ctx *c = nullptr;
    vgtb_status st = vgtb_create(rq.system, &o, s_->arena + off, bytes, s_->streams[(size_t)slot], &c);
    if (st != VGTB_OK) {
      msg = ctx_error(nullptr, "vgtb_create");
      return st;
    }
    *job = c;
    st = vgtb_ground_state(c, nullptr);
    if (st != VGTB_OK) {
      msg = ctx_error(c, "vgtb_ground_state");
      return st;
    }
    st = vgtb_set_field_table(c, rq.n_field, rq.field);
    if (st != VGTB_OK) msg = ctx_error(c, "vgtb_set_field_table");
    return st;
  }

  vgtb_status step(void *job, int64_t n, std::string &msg) override {
    vgtb_ctx *c = static_cast<vgtb_ctx *>(job);
    const vgtb_status st = vgtb_step(c, n);
    if (st != VGTB_OK) msg = ctx_error(c, "vgtb_step");
    return st;
  }

  vgtb_status mark(int slot, void **marker, std::string &msg) override {
    hipEvent_t e = nullptr;
    if (!s_->events.empty()) {
      e = s_->events.back();
      s_->events.pop_back();
    } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      msg = "hipEventCreateWithFlags failed";
      return VGTB_E_DEVICE;
    }
    *marker = e;
    const hipError_t r = hipEventRecord(e, s_->streams[(size_t)slot]);
    if (r != hipSuccess) {
      msg = std::string("hipEventRecord: ") + hipGetErrorString(r);
      return VGTB_E_DEVICE;
    }
    return VGTB_OK;
  }

  int poll(void *marker) override {
    const hipError_t q = hipEventQuery(static_cast<hipEvent_t>(marker));
    if (q == hipSuccess) return 1;
    return q == hipErrorNotReady ? 0 : -1;
  }

  void recycle(void *marker) override { s_->events.push_back(static_cast<hipEvent_t>(marker)); }

  vgtb_status finish(void *job, const vgtb_request &rq, const vgtb_options &opt,
                     std::string &msg) override {
    vgtb_ctx *c = static_cast<vgtb_ctx *>(job);
    vgtb_status st = vgtb_synchronize(c);
    if (st != VGTB_OK) {
      msg = ctx_error(c, "vgtb_synchronize");
      return st;
    }
    const int64_t n = rq.n_steps;
    std::vector<double> jall((size_t)n * 3);
    st = vgtb_read_observables(c, 0, n, jall.data(), nullptr, nullptr, nullptr);
    if (st != VGTB_OK) {
      msg = ctx_error(c, "vgtb_read_observables");
      return st;
    }
    if (rq.j_out) std::memcpy(rq.j_out, jall.data(), sizeof(double) * 3 * (size_t)n);
    if (rq.sigma_out && rq.n_omega > 0) {
      if (n < 2) {
        msg = "a spectrum needs at least two steps";
        return VGTB_E_INVAL;
      }
      std::vector<double> jx((size_t)n);
      for (int64_t t = 0; t < n; ++t) jx[(size_t)t] = jall[3 * (size_t)t];
      st = vgtb_spectrum(c, n, jx.data(), opt.dt, rq.n_omega, rq.omega, rq.e0, rq.tau0, 1, rq.sigma_out,
                         nullptr);
      if (st != VGTB_OK) msg = ctx_error(c, "vgtb_spectrum");
    }
    return st;
  }

  void destroy(void *job) override { vgtb_destroy(static_cast<vgtb_ctx *>(job)); }

 private:
  vgtb_server *s_;
};

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
  if (hipSetDevice(s->device) != hipSuccess) return VGTB_E_DEVICE;
  HipEngine eng(s);
  try {
    return vgtb_srv::run(eng, s->bytes, (int)s->streams.size(), n, reqs, stats, summary);
  } catch (...) {
    return VGTB_E_DEVICE;   // host allocation failure inside the scheduler
  }
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
