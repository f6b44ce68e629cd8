// Batched complex GEMM Y = A * B with every operand split into two bf16
// parts (x = x_hi + x_lo, x_hi = bf16(x), x_lo = bf16(x - x_hi)) and the
// product formed as A_hi B_hi + A_hi B_lo + A_lo B_hi with FP32 accumulation
// on the gfx950 bf16 matrix cores (v_mfma_f32_16x16x32_bf16): the reduced-
// precision form of the dense product S_k^-1 W of Eq. 6.  The dropped
// A_lo B_lo term and the split leave about 2^-17 relative error per product.
//
// Operand storage (bf16 planes, p = re_hi, re_lo, im_hi, im_lo; np = padded N,
// a multiple of 64, zero-filled beyond N):
//   A: plane p, batch k: row-major np x np            (A[i][kk] at i*np + kk)
//   B: plane p, batch k: k-packed (np/8) x np x 8     (B[kk][j] at ((kk/8)*np + j)*8 + kk%8)
// so that the eight consecutive kk one lane feeds to an MFMA are 16 bytes.
// Output: row-major N x N complex64.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "vgtb_internal.h"

namespace vgtb {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline bf16x8 as_bf16x8(uint4 u) { return __builtin_bit_cast(bf16x8, u); }
__device__ inline uint4 negate8(uint4 u) {
  return make_uint4(u.x ^ 0x80008000u, u.y ^ 0x80008000u, u.z ^ 0x80008000u, u.w ^ 0x80008000u);
}
__device__ inline v4f mma(uint4 a, uint4 b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a), as_bf16x8(b), c, 0, 0, 0);
}

constexpr int BM = 64, BN = 64, BK = 32;   // workgroup tile; 4 wavefronts of 32x32
constexpr int NT = 256;
constexpr int APAD = 40;                    // bf16 per LDS row of A (32 + 8 pad)

__global__ __launch_bounds__(NT) void k_cgemm_bf16x3(const uint16_t *__restrict__ A,
                                                     const uint16_t *__restrict__ B,
                                                     float2 *__restrict__ Y, int n, int np,
                                                     int batch_count, int tiles_m, int tiles_n) {
  // LDS: A [plane][row][k] (padded rows), B [plane][k/8][col][8].
  __shared__ uint4 As[4][BM][APAD / 8];
  __shared__ uint4 Bs[4][BK / 8][BN];

  const int tiles = tiles_m * tiles_n;
  const int nwg = tiles * batch_count;
  int lin = blockIdx.x + blockIdx.y * tiles;
  if ((nwg & 7) == 0) lin = (lin & 7) * (nwg >> 3) + (lin >> 3);
  const int batch = lin / tiles;
  const int tile = lin % tiles;
  const int bm = (tile / tiles_n) * BM;
  const int bn = (tile % tiles_n) * BN;

  const size_t plane = (size_t)batch_count * np * np;     // elements per plane
  const size_t boff = (size_t)batch * np * np;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave >> 1) * 32, wn0 = (wave & 1) * 32;
  const int lr = lane & 15, lg = lane >> 4;

  v4f cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
      ci[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    }

  // Per stage each thread moves 4 uint4 of A and 4 of B (4 planes x 64 x 32 bf16 each).
  uint4 ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int L = tid + i * NT;          // 0 .. 1023
      const int p = L >> 8, r = (L >> 2) & 63, c = L & 3;
      ra[i] = *reinterpret_cast<const uint4 *>(A + p * plane + boff + (size_t)(bm + r) * np + k0 + c * 8);
      const int kb = (L >> 6) & 3, col = L & 63;
      rb[i] = *reinterpret_cast<const uint4 *>(B + p * plane + boff + ((size_t)(k0 / 8 + kb) * np + bn + col) * 8);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int L = tid + i * NT;
      As[L >> 8][(L >> 2) & 63][L & 3] = ra[i];
      Bs[L >> 8][(L >> 6) & 3][L & 63] = rb[i];
    }
  };

  const int nkt = np / BK;
  load(0);
  for (int kt = 0; kt < nkt; ++kt) {
    __syncthreads();                 // previous stage fully consumed
    store();
    __syncthreads();
    if (kt + 1 < nkt) load((kt + 1) * BK);
    uint4 fa[2][4], fb[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int p = 0; p < 4; ++p) fa[a][p] = As[p][wm0 + a * 16 + lr][lg];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int p = 0; p < 4; ++p) fb[b][p] = Bs[p][lg][wn0 + b * 16 + lr];
    // planes: 0 re_hi, 1 re_lo, 2 im_hi, 3 im_lo
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const uint4 nih = negate8(fa[a][2]), nil = negate8(fa[a][3]);
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        v4f r = cr[a][b], m = ci[a][b];
        // Re += ar br - ai bi
        r = mma(fa[a][0], fb[b][0], r);
        r = mma(fa[a][0], fb[b][1], r);
        r = mma(fa[a][1], fb[b][0], r);
        r = mma(nih, fb[b][2], r);
        r = mma(nih, fb[b][3], r);
        r = mma(nil, fb[b][2], r);
        // Im += ar bi + ai br
        m = mma(fa[a][0], fb[b][2], m);
        m = mma(fa[a][0], fb[b][3], m);
        m = mma(fa[a][1], fb[b][2], m);
        m = mma(fa[a][2], fb[b][0], m);
        m = mma(fa[a][2], fb[b][1], m);
        m = mma(fa[a][3], fb[b][0], m);
        cr[a][b] = r;
        ci[a][b] = m;
      }
    }
  }

  float2 *Yb = Y + (size_t)batch * n * n;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = bm + wm0 + a * 16 + 4 * lg + j;
        const int col = bn + wn0 + b * 16 + lr;
        if (row < n && col < n) Yb[(size_t)row * n + col] = make_float2(cr[a][b][j], ci[a][b][j]);
      }
}

}  // namespace

void launch_cgemm_bf16x3(const uint16_t *a, const uint16_t *b, float2 *y, int n, int np, int batch,
                         hipStream_t s) {
  const int tm = np / BM, tn = np / BN;
  hipLaunchKernelGGL(k_cgemm_bf16x3, dim3(tm * tn, batch), dim3(NT), 0, s, a, b, y, n, np, batch,
                     tm, tn);
}

}  // namespace vgtb
