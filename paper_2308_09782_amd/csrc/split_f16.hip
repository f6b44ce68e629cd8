// Operands of the fp16 form of the dense product (S^-1 - I) W (Eq. 6 in the
// deviation form): each complex operand is scaled per k-point by a power of
// two s (so that its largest component lies in [2^13, 2^14), well inside
// fp16's range) and split as x s = hi + lo with hi = fp16(x s) and
// lo = fp16(x s - hi), four 16-bit planes (re_hi, re_lo, im_hi, im_lo).  The
// product kernel divides by s_A s_W, which is exact.
//
// The scale of W is taken from the current W (a per-k maximum in two short
// kernels, block partials then their maximum), so no value can leave fp16's
// range whatever the size of W at a given step.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "vgtb_internal.h"

namespace vgtb {
namespace {

constexpr int kParts = 128;   // partial maxima per k-point

__device__ inline float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_down(v, off, 64));
  return v;
}

// Largest |re|, |im| of an n x n complex matrix per k (minus the identity when
// asked), as kParts partials per k.  NaNs are skipped (fmaxf); they reach the
// product unchanged and are caught with the trace.
template <typename C2>
__global__ __launch_bounds__(256) void k_absmax_part(const C2 *__restrict__ src, int n,
                                                     int minus_identity, float *__restrict__ part) {
  __shared__ float red[4];
  const int k = blockIdx.y, tid = threadIdx.x;
  const size_t nn = (size_t)n * n;
  const C2 *sk = src + (size_t)k * nn;
  float m = 0.0f;
  for (size_t e = (size_t)blockIdx.x * 256 + tid; e < nn; e += (size_t)kParts * 256) {
    const C2 v = sk[e];
    double re = (double)v.x;
    if (minus_identity && e / n == e % n) re -= 1.0;
    m = fmaxf(m, fmaxf(fabsf((float)re), fabsf((float)v.y)));
  }
  m = wave_max(m);
  if ((tid & 63) == 0) red[tid >> 6] = m;
  __syncthreads();
  if (tid == 0) part[(size_t)k * kParts + blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// scale[k] = 2^e with max * 2^e in [2^13, 2^14); 1 for an all-zero or
// non-finite matrix; e clamped to [-100, 100] (a float power of two).
__global__ void k_absmax_scale(const float *__restrict__ part, int nk, float *__restrict__ scale) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  float m = 0.0f;
  for (int b = 0; b < kParts; ++b) m = fmaxf(m, part[(size_t)k * kParts + b]);
  float sc = 1.0f;
  if (m > 0.0f && isfinite(m)) sc = ldexpf(1.0f, max(-100, min(100, 13 - ilogbf(m))));
  scale[k] = sc;
}

__device__ inline uint16_t f16_bits(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
__device__ inline float f16_value(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

// W (complex64, n x n per k) into the k-packed planes of the product's B
// operand: W[r][c] at ((r / 8) np + c) 8 + r % 8 of each plane, zero beyond n.
// A thread takes one column and eight consecutive rows: one 16-byte store per plane.
__global__ __launch_bounds__(256) void k_split_w_f16(const float2 *__restrict__ w,
                                                     const float *__restrict__ scale,
                                                     uint16_t *__restrict__ planes, int n, int np,
                                                     int nk) {
  const int k = blockIdx.z, r8 = blockIdx.y;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= np) return;
  const float sc = scale[k];
  const float2 *wk = w + (size_t)k * n * n;
  uint32_t p[4][4];
#pragma unroll
  for (int i = 0; i < 8; i += 2) {
    uint16_t h[4][2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int r = r8 * 8 + i + t;
      const float2 v = (r < n && c < n) ? wk[(size_t)r * n + c] : make_float2(0.0f, 0.0f);
      const float xr = v.x * sc, xi = v.y * sc;
      h[0][t] = f16_bits(xr);
      h[1][t] = f16_bits(xr - f16_value(h[0][t]));
      h[2][t] = f16_bits(xi);
      h[3][t] = f16_bits(xi - f16_value(h[2][t]));
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q][i / 2] = (uint32_t)h[q][0] | ((uint32_t)h[q][1] << 16);
  }
  const size_t plane = (size_t)nk * np * np;
  const size_t off = (size_t)k * np * np + ((size_t)r8 * np + c) * 8;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    *reinterpret_cast<uint4 *>(planes + q * plane + off) = make_uint4(p[q][0], p[q][1], p[q][2], p[q][3]);
}

// A = S^-1 - I (complex128, n x n per k) into row-major planes np x np, zero beyond n.
__global__ __launch_bounds__(256) void k_split_a_f16(const double2 *__restrict__ sinv,
                                                     const float *__restrict__ scale,
                                                     uint16_t *__restrict__ planes, int n, int np,
                                                     int nk) {
  const int k = blockIdx.z, i = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= np) return;
  double2 v = make_double2(0.0, 0.0);
  if (i < n && j < n) v = sinv[(size_t)k * n * n + (size_t)i * n + j];
  if (i == j && i < n) v.x -= 1.0;
  const double sc = (double)scale[k];
  const double xr = v.x * sc, xi = v.y * sc;
  const uint16_t rh = f16_bits((float)xr), ih = f16_bits((float)xi);
  const uint16_t rl = f16_bits((float)(xr - (double)f16_value(rh)));
  const uint16_t il = f16_bits((float)(xi - (double)f16_value(ih)));
  const size_t plane = (size_t)nk * np * np;
  const size_t idx = (size_t)k * np * np + (size_t)i * np + j;
  planes[idx] = rh;
  planes[plane + idx] = rl;
  planes[2 * plane + idx] = ih;
  planes[3 * plane + idx] = il;
}

int blocks(long long n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

int f16_scale_parts() { return kParts; }

void launch_f16_scale(const double2 *src, int n, int nk, bool minus_identity, float *part, float *scale,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_absmax_part<double2>, dim3(kParts, nk), dim3(256), 0, s, src, n,
                     minus_identity ? 1 : 0, part);
  hipLaunchKernelGGL(k_absmax_scale, dim3(blocks(nk, 64)), dim3(64), 0, s, part, nk, scale);
}

void launch_f16_scale(const float2 *src, int n, int nk, float *part, float *scale, hipStream_t s) {
  hipLaunchKernelGGL(k_absmax_part<float2>, dim3(kParts, nk), dim3(256), 0, s, src, n, 0, part);
  hipLaunchKernelGGL(k_absmax_scale, dim3(blocks(nk, 64)), dim3(64), 0, s, part, nk, scale);
}

void launch_split_w_f16(const float2 *w, const float *scale, uint16_t *planes, int n, int np, int nk,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_split_w_f16, dim3(blocks(np, 256), np / 8, nk), dim3(256), 0, s, w, scale, planes,
                     n, np, nk);
}

void launch_split_a_f16(const double2 *sinv, const float *scale, uint16_t *planes, int n, int np,
                        int nk, hipStream_t s) {
  hipLaunchKernelGGL(k_split_a_f16, dim3(blocks(np, 256), np, nk), dim3(256), 0, s, sinv, scale, planes,
                     n, np, nk);
}

}  // namespace vgtb
