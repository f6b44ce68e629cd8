// Spectrum of a current trace (paper Eqs. 15-16) on the device, streamed
// through a bounded device scratch:
//   sigma(w) = (1/E0) sum_t c_t (J_t - <J>) exp(-t / tau0) exp(i w t)
//   epsilon(w) = 1 + 4 pi i sigma(w) / w
// with trapezoid weights c_t on t_n = n dt.  The trace and the frequency grid
// are cut into chunks that fit the scratch, so any length of run and any
// grid size is handled by a scratch of a few thousand doubles: the mean is
// summed chunk by chunk on the device, then every frequency chunk accumulates
// its sums over the time chunks.  One chunk layout serves every caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>

#include "vgtb_internal.h"

namespace vgtb {
namespace {

constexpr int kSpecThreads = 256;

__device__ inline double block_sum(double v, double *red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kSpecThreads / 64; ++w) s += red[w];
  __syncthreads();
  return s;   // valid on thread 0
}

// sum[0] (+)= sum of the chunk; with last, sum[0] becomes the mean over nt.
__global__ __launch_bounds__(kSpecThreads) void k_spec_sum(const double *__restrict__ j, int len,
                                                           int first, int last, int64_t nt,
                                                           double *sum) {
  __shared__ double red[kSpecThreads / 64];
  double s = 0.0;
  for (int t = threadIdx.x; t < len; t += kSpecThreads) s += j[t];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    const double acc = (first ? 0.0 : sum[0]) + s;
    sum[0] = last ? acc / (double)nt : acc;
  }
}

// One block per frequency of the chunk: acc[w] (+)= the chunk's share of the
// filtered transform.  The chunk holds samples t0 .. t0 + len - 1 of nt.
// With last, sigma and epsilon of the frequency are written.
__global__ __launch_bounds__(kSpecThreads) void k_spec_chunk(
    const double *__restrict__ j, int64_t t0, int len, int64_t nt, double dt,
    const double *__restrict__ mean, const double *__restrict__ omega, double e0, double tau0,
    int first, int last, double2 *__restrict__ acc, double2 *__restrict__ sigma,
    double2 *__restrict__ eps) {
  __shared__ double red[kSpecThreads / 64];
  const int w = blockIdx.x;
  const double om = omega[w];
  const double m = mean ? mean[0] : 0.0;
  double re = 0.0, im = 0.0;
  for (int i = threadIdx.x; i < len; i += kSpecThreads) {
    const int64_t t = t0 + i;
    const double tt = (double)t * dt;
    const double wt = (t == 0 || t == nt - 1) ? 0.5 * dt : dt;   // trapezoid weights
    const double g = (j[i] - m) * exp(-tt / tau0) * wt;
    double sn, cs;
    sincos(om * tt, &sn, &cs);
    re += cs * g;
    im += sn * g;
  }
  re = block_sum(re, red);
  im = block_sum(im, red);
  if (threadIdx.x == 0) {
    double2 a = first ? make_double2(0.0, 0.0) : acc[w];
    a.x += re;
    a.y += im;
    acc[w] = a;
    if (last) {
      const double sr = a.x / e0, si = a.y / e0;
      sigma[w] = make_double2(sr, si);
      eps[w] = make_double2(1.0 - 4.0 * M_PI * si / om, 4.0 * M_PI * sr / om);
    }
  }
}

}  // namespace

size_t spectrum_min_scratch() { return 2 + 7 * 2 + 64; }

hipError_t spectrum_chunked(double *scratch, size_t cap, hipStream_t s, int64_t n_t,
                            const double *j_host, double dt, int64_t n_w, const double *omega_host,
                            double e0, double tau0, bool subtract_mean, void *sigma_host,
                            void *eps_host) {
  if (cap < spectrum_min_scratch()) return hipErrorInvalidValue;
  // Layout (doubles): [0] sum / mean, [1] pad, omega chunk (wc), acc (2 wc),
  // sigma (2 wc), eps (2 wc), J chunk (tc).  wc even keeps the double2 parts
  // 16-byte aligned.
  // At most half the scratch for the frequency parts, the rest for the trace.
  size_t wc = std::min<size_t>((size_t)n_w, 1024);
  wc = std::min(wc, (cap - 2 - 64) / 14);
  wc = std::max<size_t>(2, wc & ~(size_t)1);
  const size_t tc = std::min<size_t>(cap - 2 - 7 * wc, (size_t)1 << 30);
  double *sum = scratch;
  double *om = scratch + 2;
  double2 *acc = reinterpret_cast<double2 *>(om + wc);
  double2 *sig = acc + wc;
  double2 *ep = sig + wc;
  double *jc = reinterpret_cast<double *>(ep + wc);
  const bool resident = (size_t)n_t <= tc;   // the whole trace fits: upload once
  hipError_t e = hipSuccess;
  auto upload = [&](int64_t t0, int len) {
    return hipMemcpyAsync(jc, j_host + t0, sizeof(double) * (size_t)len, hipMemcpyHostToDevice, s);
  };
  auto chunk_len = [&](int64_t t0) { return (int)std::min<int64_t>((int64_t)tc, n_t - t0); };
  if (subtract_mean) {
    for (int64_t t0 = 0; t0 < n_t; t0 += (int64_t)tc) {
      const int len = chunk_len(t0);
      if ((e = upload(t0, len)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_spec_sum, dim3(1), dim3(kSpecThreads), 0, s, jc, len, t0 == 0 ? 1 : 0,
                         t0 + len >= n_t ? 1 : 0, n_t, sum);
    }
  }
  if (resident && !subtract_mean && (e = upload(0, (int)n_t)) != hipSuccess) return e;
  for (int64_t w0 = 0; w0 < n_w; w0 += (int64_t)wc) {
    const int nwc = (int)std::min<int64_t>((int64_t)wc, n_w - w0);
    if ((e = hipMemcpyAsync(om, omega_host + w0, sizeof(double) * nwc, hipMemcpyHostToDevice, s)) != hipSuccess)
      return e;
    for (int64_t t0 = 0; t0 < n_t; t0 += (int64_t)tc) {
      const int len = chunk_len(t0);
      if (!resident && (e = upload(t0, len)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_spec_chunk, dim3(nwc), dim3(kSpecThreads), 0, s, jc, t0, len, n_t, dt,
                         subtract_mean ? sum : nullptr, om, e0, tau0, t0 == 0 ? 1 : 0,
                         t0 + len >= n_t ? 1 : 0, acc, sig, ep);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (sigma_host &&
        (e = hipMemcpyAsync(static_cast<double2 *>(sigma_host) + w0, sig, sizeof(double2) * nwc,
                            hipMemcpyDeviceToHost, s)) != hipSuccess)
      return e;
    if (eps_host &&
        (e = hipMemcpyAsync(static_cast<double2 *>(eps_host) + w0, ep, sizeof(double2) * nwc,
                            hipMemcpyDeviceToHost, s)) != hipSuccess)
      return e;
    // The next frequency chunk overwrites omega, acc, sigma and eps.
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  }
  return hipStreamSynchronize(s);
}

// ---------------------------------------------------------------------------
// The same spectrum without any allocation, for callers that cannot allocate
// device memory (code under stream capture, tight serving loops): its scratch
// is a fixed array in the library's device image, one copy per GPU, held until
// the process ends.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kStaticSpectrumDoubles = size_t(1) << 17;   // 1 MiB per GPU
static __device__ __align__(256) double scratch[kStaticSpectrumDoubles];

constexpr int kMaxDevices = 64;
// Device address of scratch per GPU, looked up once per device (the host-side
// name of the array is not a device address).
std::atomic<double *> g_scratch_ptr[kMaxDevices];

double *scratch_on(int device) {
  double *p = g_scratch_ptr[device].load(std::memory_order_acquire);
  if (p) return p;
  void *addr = nullptr;
  if (hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch)) != hipSuccess || !addr) return nullptr;
  p = static_cast<double *>(addr);
  g_scratch_ptr[device].store(p, std::memory_order_release);
  return p;
}

}  // namespace
}  // namespace vgtb

extern "C" vgtb_status vgtb_spectrum_noalloc(int64_t n_t, const double *j_host, double dt, int64_t n_w,
                                             const double *omega_host, double e0, double tau0,
                                             int subtract_mean, void *sigma_host, void *eps_host,
                                             void *hip_stream) {
  if (n_t < 2 || n_w < 1 || !j_host || !omega_host || !(std::fabs(e0) > 0.0) || !(tau0 > 0.0) ||
      !std::isfinite(dt)) {
    vgtb::set_last_error("vgtb_spectrum_noalloc: needs n_t >= 2, n_w >= 1, the trace and the grid, "
                         "e0 != 0, tau0 > 0 and a finite dt");
    return VGTB_E_INVAL;
  }
  if (n_t > (int64_t)1 << 30 || n_w > (int64_t)1 << 24) {
    vgtb::set_last_error("vgtb_spectrum_noalloc: n_t above 2^30 or n_w above 2^24");
    return VGTB_E_INVAL;
  }
  for (int64_t i = 0; i < n_w; ++i)
    if (!(std::fabs(omega_host[i]) > 0.0)) {
      vgtb::set_last_error("vgtb_spectrum_noalloc: frequencies must be nonzero");
      return VGTB_E_INVAL;
    }
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess || device < 0 || device >= vgtb::kMaxDevices) {
    vgtb::set_last_error("vgtb_spectrum_noalloc: no usable current device");
    return VGTB_E_DEVICE;
  }
  double *sp = vgtb::scratch_on(device);
  if (!sp) {
    vgtb::set_last_error("vgtb_spectrum_noalloc: hipGetSymbolAddress of the static scratch failed");
    return VGTB_E_DEVICE;
  }
  const hipError_t e = vgtb::spectrum_chunked(sp, vgtb::kStaticSpectrumDoubles,
                                              static_cast<hipStream_t>(hip_stream), n_t, j_host, dt, n_w,
                                              omega_host, e0, tau0, subtract_mean != 0, sigma_host,
                                              eps_host);
  if (e != hipSuccess) {
    vgtb::set_last_error(hipGetErrorString(e));
    return VGTB_E_DEVICE;
  }
  return VGTB_OK;
}
