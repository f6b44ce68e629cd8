// Operands of the fp16 form of the dense product (S^-1 - I) W (Eq. 6 in the
// deviation form): each complex operand is scaled per k-point by a power of
// two s (so that its largest component lies in [2^13, 2^14), well inside
// fp16's range) and split as x s = hi + lo with hi = fp16(x s) and
// lo = fp16(x s - hi), four 16-bit planes (re_hi, re_lo, im_hi, im_lo).  The
// product kernel divides by s_A s_W, which is exact.
//
// The scale of W is a function of the current W alone, so no value can leave
// fp16's range whatever the size of W at a given step: the sparse product
// writes W's planes with the scale of the previous step and raises the per-k
// maximum (spread over kMaxSlots slots); the check below sets the scale that
// maximum calls for, and a k-point whose scale changed (rare: W changes little
// from step to step) is split again from the complex64 W.  The planes are thus the same as a split
// with the current maximum's scale.  The scale of S^-1 - I comes from block
// partial maxima once, when the context is created.
#include <hip/hip_runtime.h>

#include <algorithm>
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

__device__ inline float pow2_scale(float m) { return f16_pow2_scale(m); }

__global__ void k_absmax_scale(const float *__restrict__ part, int nk, float *__restrict__ scale) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  float m = 0.0f;
  for (int b = 0; b < kParts; ++b) m = fmaxf(m, part[(size_t)k * kParts + b]);
  scale[k] = pow2_scale(m);
}

__global__ void k_scale_check(unsigned *__restrict__ wmax, float *__restrict__ scale,
                              int *__restrict__ flag, int nk) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  unsigned *wk = wmax + (size_t)k * kMaxSlots * kMaxStride;
  unsigned m = 0u;
  for (int i = 0; i < kMaxSlots; ++i) {
    m = max(m, wk[i * kMaxStride]);
    wk[i * kMaxStride] = 0u;
  }
  const float sc = pow2_scale(__uint_as_float(m));
  flag[k] = sc != scale[k];
  scale[k] = sc;
}

__global__ void k_scale_init(unsigned *__restrict__ wmax, float *__restrict__ scale, int nk) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  for (int i = 0; i < kMaxSlots; ++i) wmax[((size_t)k * kMaxSlots + i) * kMaxStride] = 0u;
  scale[k] = 1.0f;
}

__device__ inline uint16_t f16_bits(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
__device__ inline float f16_value(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

// W (complex64, n x n per k) into the k-packed planes of the product's B
// operand: W[r][c] at ((r / 8) np + c) 8 + r % 8 of each plane, zero beyond n.
// A thread takes one column and eight consecutive rows at a time (one 16-byte
// store per plane), the row groups strided by gridDim.y.
__global__ __launch_bounds__(256) void k_split_w_f16(const float2 *__restrict__ w,
                                                     const float *__restrict__ scale,
                                                     uint16_t *__restrict__ planes, int n, int np,
                                                     int nk, const int *__restrict__ flag) {
  const int k = blockIdx.z;
  if (flag != nullptr && flag[k] == 0) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= np) return;
  const float sc = scale[k];
  const float2 *wk = w + (size_t)k * n * n;
  const size_t plane = (size_t)nk * np * np;
  for (int r8 = blockIdx.y; r8 < np / 8; r8 += gridDim.y) {
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
    const size_t off = (size_t)k * np * np + ((size_t)r8 * np + c) * 8;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      *reinterpret_cast<uint4 *>(planes + q * plane + off) = make_uint4(p[q][0], p[q][1], p[q][2], p[q][3]);
  }
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

void launch_f16_scale_check(unsigned *wmax, float *scale, int *flag, int nk, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_check, dim3(blocks(nk, 64)), dim3(64), 0, s, wmax, scale, flag, nk);
}

void launch_f16_scale_init(unsigned *wmax, float *scale, int nk, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_init, dim3(blocks(nk, 64)), dim3(64), 0, s, wmax, scale, nk);
}

void launch_split_w_f16(const float2 *w, const float *scale, uint16_t *planes, int n, int np, int nk,
                        const int *flag, hipStream_t s) {
  hipLaunchKernelGGL(k_split_w_f16, dim3(blocks(np, 256), std::min(np / 8, 32), nk), dim3(256), 0, s, w,
                     scale, planes, n, np, nk, flag);
}

void launch_split_a_f16(const double2 *sinv, const float *scale, uint16_t *planes, int n, int np,
                        int nk, hipStream_t s) {
  hipLaunchKernelGGL(k_split_a_f16, dim3(blocks(np, 256), np, nk), dim3(256), 0, s, sinv, scale, planes,
                     n, np, nk);
}

}  // namespace vgtb
