// Batched complex GEMM Y = A * B with every operand split into two 16-bit
// parts (x = x_hi + x_lo, x_hi = r(x), x_lo = r(x - x_hi)) and the product
// formed as A_hi B_hi + A_hi B_lo + A_lo B_hi with FP32 accumulation on the
// gfx950 matrix cores: the reduced-precision form of the dense product S_k^-1 W
// of Eq. 6.  Element type E = 0: bf16 (v_mfma_f32_16x16x32_bf16; the split and
// the dropped A_lo B_lo term leave about 2^-17 relative error per product);
// E = 1: fp16 (v_mfma_f32_16x16x32_f16) on operands scaled by powers of two
// sa[k], sb[k] into fp16's range, about 2^-21; the epilogue divides by
// sa[k] sb[k] (exact).
//
// Operand storage (16-bit planes, p = re_hi, re_lo, im_hi, im_lo; np = padded N,
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
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // 8 packed 16-bit values

// Sign flip of eight packed 16-bit values (bf16 and fp16 keep the sign in bit 15).
__device__ inline u32x4 negate8(u32x4 u) { return u ^ 0x80008000u; }
template <int E>
__device__ inline v4f mma(u32x4 a, u32x4 b, v4f c) {
  if constexpr (E == 0)
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                  __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
}
// 1 / (sa[k] sb[k]) for the fp16 form (powers of two), 1 for bf16.
__device__ inline float unscale(const float *sa, const float *sb, int k) {
  return sa ? 1.0f / (sa[k] * sb[k]) : 1.0f;
}

constexpr int BM = 64, BN = 64, BK = 32;   // workgroup tile; 4 wavefronts of 32x32
constexpr int NT = 256;
constexpr int APAD = 40;                    // 16-bit values per LDS row of A (32 + 8 pad)

template <int E>
__global__ __launch_bounds__(NT) void k_cgemm_split16(const uint16_t *__restrict__ A,
                                                     const uint16_t *__restrict__ B,
                                                     float2 *__restrict__ Y, int n, int np,
                                                     int batch_count, int tiles_m, int tiles_n,
                                                     const float *__restrict__ sa,
                                                     const float *__restrict__ sb) {
  // LDS: A [plane][row][k] (padded rows), B [plane][k/8][col][8].
  __shared__ u32x4 As[4][BM][APAD / 8];
  __shared__ u32x4 Bs[4][BK / 8][BN];

  const int tiles = tiles_m * tiles_n;
  const int lin = xcd_slot(blockIdx.x + blockIdx.y * tiles, tiles * batch_count);
  const int batch = lin / tiles;
  int tm, tn;
  grouped_tile(lin % tiles, tiles_m, tiles_n, 4, tm, tn);
  const int bm = tm * BM;
  const int bn = tn * BN;

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

  // Per stage each thread moves 4 u32x4 of A and 4 of B (4 planes x 64 x 32 bf16 each).
  u32x4 ra[4], rb[4];
#define VG_LOAD64(k0)                                                                          \
  do {                                                                                         \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                            \
      const int L = tid + i * NT;                                                              \
      ra[i] = *reinterpret_cast<const u32x4 *>(A + (L >> 8) * plane + boff +                   \
                                               (size_t)(bm + ((L >> 2) & 63)) * np + (k0) + (L & 3) * 8); \
      rb[i] = *reinterpret_cast<const u32x4 *>(B + (L >> 8) * plane + boff +                   \
                                               ((size_t)((k0) / 8 + ((L >> 6) & 3)) * np + bn + (L & 63)) * 8); \
    }                                                                                          \
  } while (0)

  const int nkt = np / BK;
  VG_LOAD64(0);
  for (int kt = 0; kt < nkt; ++kt) {
    __syncthreads();                 // previous stage fully consumed
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int L = tid + i * NT;
      As[L >> 8][(L >> 2) & 63][L & 3] = ra[i];
      Bs[L >> 8][(L >> 6) & 3][L & 63] = rb[i];
    }
    __syncthreads();
    if (kt + 1 < nkt) VG_LOAD64((kt + 1) * BK);
    u32x4 fa[2][4], fb[2][4];
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
      const u32x4 nih = negate8(fa[a][2]), nil = negate8(fa[a][3]);
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        v4f r = cr[a][b], m = ci[a][b];
        // Re += ar br - ai bi
        r = mma<E>(fa[a][0], fb[b][0], r);
        r = mma<E>(fa[a][0], fb[b][1], r);
        r = mma<E>(fa[a][1], fb[b][0], r);
        r = mma<E>(nih, fb[b][2], r);
        r = mma<E>(nih, fb[b][3], r);
        r = mma<E>(nil, fb[b][2], r);
        // Im += ar bi + ai br
        m = mma<E>(fa[a][0], fb[b][2], m);
        m = mma<E>(fa[a][0], fb[b][3], m);
        m = mma<E>(fa[a][1], fb[b][2], m);
        m = mma<E>(fa[a][2], fb[b][0], m);
        m = mma<E>(fa[a][2], fb[b][1], m);
        m = mma<E>(fa[a][3], fb[b][0], m);
        cr[a][b] = r;
        ci[a][b] = m;
      }
    }
  }

  float2 *Yb = Y + (size_t)batch * n * n;
  const float us = unscale(sa, sb, batch);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = bm + wm0 + a * 16 + 4 * lg + j;
        const int col = bn + wn0 + b * 16 + lr;
        if (row < n && col < n)
          Yb[(size_t)row * n + col] = make_float2(us * cr[a][b][j], us * ci[a][b][j]);
      }
#undef VG_LOAD64
}

// Large tiles for np a multiple of 128: 128 x 128 per workgroup of WGM x WGN
// wavefronts (several per SIMD, so one wave's stalls are covered by another),
// each computing (128/WGM) x (128/WGN) from 16 x 16 MFMA tiles.
// Software pipeline, one workgroup per CU:
//  - LDS double-buffered (2 x 72 KB); stage kt+1 is written from registers
//    after the first group of MFMAs of stage kt, and the global loads of
//    stage kt+2 are issued right after, so they have a whole stage to land;
//  - the twelve partial products are grouped by the B plane they read, and
//    the next plane's B fragments are read while the current plane's MFMAs run.
constexpr int BM2 = 128, BN2 = 128;

template <int E, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void k_cgemm_split16_128(const uint16_t *__restrict__ A,
                                                                     const uint16_t *__restrict__ B,
                                                                     float2 *__restrict__ Y, int n,
                                                                     int np, int batch_count,
                                                                     int tiles_m, int tiles_n,
                                                                     const float *__restrict__ sa,
                                                                     const float *__restrict__ sb) {
  constexpr int NT2 = 64 * WGM * WGN;
  constexpr int TM = BM2 / WGM / 16, TN = BN2 / WGN / 16;
  constexpr int LD = 2048 / NT2;             // u32x4 per thread per operand and stage
  __shared__ u32x4 As[2][4][BM2][APAD / 8];
  __shared__ u32x4 Bs[2][4][BK / 8][BN2];

  const int tiles = tiles_m * tiles_n;
  const int lin = xcd_slot(blockIdx.x + blockIdx.y * tiles, tiles * batch_count);
  const int batch = lin / tiles;
  int tm, tn;
  grouped_tile(lin % tiles, tiles_m, tiles_n, 4, tm, tn);
  const int bm = tm * BM2;
  const int bn = tn * BN2;

  const size_t plane = (size_t)batch_count * np * np;
  const size_t boff = (size_t)batch * np * np;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WGN) * (BM2 / WGM), wn0 = (wave % WGN) * (BN2 / WGN);
  const int lr = lane & 15, lg = lane >> 4;

  v4f cr[TM][TN], ci[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      cr[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
      ci[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    }

  // Per stage: 2048 u32x4 of A (4 planes x 128 rows x 4) and 2048 of B (4 x 4 x 128).
  // A element L of a plane is row AROW(L), 16-byte column ACOL(L): sixteen
  // consecutive lanes take sixteen rows of one column, so their LDS stores hit
  // distinct banks (row stride APAD = 80 bytes), like the fragment reads; a
  // wavefront still loads whole 64-byte row segments from global memory.
#define AROW(L) (((L) & 15) | ((((L) >> 6) & 7) << 4))
#define ACOL(L) (((L) >> 4) & 3)
  // Global loads run ahead of the LDS writes by PF stages: the loads of stage
  // kt+1+PF are issued during stage kt and written to LDS during stage kt+PF.
  // PF = 2 needs a second register set, which sixteen wavefronts (128
  // registers each) cannot hold; they use PF = 1.
  constexpr int PF = (WGM * WGN >= 16) ? 1 : 2;
  u32x4 ra0[LD], rb0[LD], ra1[LD], rb1[LD];
#define VG_LOAD128(ra, rb, k0)                                                                 \
  do {                                                                                         \
    _Pragma("unroll") for (int i = 0; i < LD; ++i) {                                           \
      const int L = tid + i * NT2;                                                             \
      ra[i] = *reinterpret_cast<const u32x4 *>(A + (L >> 9) * plane + boff +                   \
                                               (size_t)(bm + AROW(L)) * np + (k0) + ACOL(L) * 8); \
      rb[i] = *reinterpret_cast<const u32x4 *>(B + (L >> 9) * plane + boff +                   \
                                               ((size_t)((k0) / 8 + ((L >> 7) & 3)) * np + bn + (L & 127)) * 8); \
    }                                                                                          \
  } while (0)
#define VG_STORE128(ra, rb, buf)                                                               \
  do {                                                                                         \
    _Pragma("unroll") for (int i = 0; i < LD; ++i) {                                           \
      const int L = tid + i * NT2;                                                             \
      As[buf][L >> 9][AROW(L)][ACOL(L)] = ra[i];                                               \
      Bs[buf][L >> 9][(L >> 7) & 3][L & 127] = rb[i];                                          \
    }                                                                                          \
  } while (0)
#define VG_READB(dst, buf, pb)                                                                 \
  _Pragma("unroll") for (int b = 0; b < TN; ++b) dst[b] = Bs[buf][pb][lg][wn0 + b * 16 + lr]

  const int nkt = np / BK;   // even: np is a multiple of 128
  // One stage: the twelve partial products of LDS buffer cur; between the
  // first group and the rest, LDS buffer cur^1 receives stage kt+1 from (ra, rb)
  // and (ra, rb) starts loading stage kt+1+PF.
  auto stage = [&](int kt, int cur, u32x4 (&ra)[LD], u32x4 (&rb)[LD]) {
    u32x4 fa[TM][4], nf2[TM], nf3[TM], fb0[TN], fb1[TN];
#pragma unroll
    for (int a = 0; a < TM; ++a) {
#pragma unroll
      for (int p = 0; p < 4; ++p) fa[a][p] = As[cur][p][wm0 + a * 16 + lr][lg];
      nf2[a] = negate8(fa[a][2]);
      nf3[a] = negate8(fa[a][3]);
    }
    VG_READB(fb0, cur, 0);
    VG_READB(fb1, cur, 1);
    // B plane 0 (re_hi): Re += Ar_hi Br_hi + Ar_lo Br_hi;  Im += Ai_hi Br_hi + Ai_lo Br_hi
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        cr[a][b] = mma<E>(fa[a][0], fb0[b], cr[a][b]);
        ci[a][b] = mma<E>(fa[a][2], fb0[b], ci[a][b]);
        cr[a][b] = mma<E>(fa[a][1], fb0[b], cr[a][b]);
        ci[a][b] = mma<E>(fa[a][3], fb0[b], ci[a][b]);
      }
    if (kt + 1 < nkt) {
      VG_STORE128(ra, rb, cur ^ 1);
      if (kt + 1 + PF < nkt) VG_LOAD128(ra, rb, (kt + 1 + PF) * BK);
    }
    VG_READB(fb0, cur, 2);
    // B plane 1 (re_lo): Re += Ar_hi Br_lo;  Im += Ai_hi Br_lo
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        cr[a][b] = mma<E>(fa[a][0], fb1[b], cr[a][b]);
        ci[a][b] = mma<E>(fa[a][2], fb1[b], ci[a][b]);
      }
    VG_READB(fb1, cur, 3);
    // B plane 2 (im_hi): Re -= Ai_hi Bi_hi + Ai_lo Bi_hi;  Im += Ar_hi Bi_hi + Ar_lo Bi_hi
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        cr[a][b] = mma<E>(nf2[a], fb0[b], cr[a][b]);
        ci[a][b] = mma<E>(fa[a][0], fb0[b], ci[a][b]);
        cr[a][b] = mma<E>(nf3[a], fb0[b], cr[a][b]);
        ci[a][b] = mma<E>(fa[a][1], fb0[b], ci[a][b]);
      }
    // B plane 3 (im_lo): Re -= Ai_hi Bi_lo;  Im += Ar_hi Bi_lo
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        cr[a][b] = mma<E>(nf2[a], fb1[b], cr[a][b]);
        ci[a][b] = mma<E>(fa[a][0], fb1[b], ci[a][b]);
      }
    __syncthreads();
  };

  VG_LOAD128(ra0, rb0, 0);
  VG_STORE128(ra0, rb0, 0);
  __syncthreads();
  if (nkt > 1) VG_LOAD128(ra0, rb0, BK);                 // stage 1, stored during stage 0
  if (PF == 2 && nkt > 2) VG_LOAD128(ra1, rb1, 2 * BK);  // stage 2, stored during stage 1
  for (int kt = 0; kt < nkt; kt += 2) {
    stage(kt, 0, ra0, rb0);
    if (PF == 2) stage(kt + 1, 1, ra1, rb1);
    else stage(kt + 1, 1, ra0, rb0);
  }
#undef VG_LOAD128
#undef VG_STORE128
#undef VG_READB
#undef AROW
#undef ACOL

  float2 *Yb = Y + (size_t)batch * n * n;
  const float us = unscale(sa, sb, batch);
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = bm + wm0 + a * 16 + 4 * lg + j;
        const int col = bn + wn0 + b * 16 + lr;
        if (row < n && col < n)
          Yb[(size_t)row * n + col] = make_float2(us * cr[a][b][j], us * ci[a][b][j]);
      }
}

// tile: 1 = 64 x 64 (four wavefronts); 128 x 128 (np a multiple of 128 only)
// with 2 = sixteen wavefronts of 32 x 32, 3 = eight of 64 x 32, 4 = eight of
// 32 x 64, 5 = four of 64 x 64 (fewer LDS fragment reads per matrix
// instruction, fewer wavefronts to cover stalls); 0 = 2 where allowed from
// np = 512 up, else 1.
template <int E>
static void launch_e(const uint16_t *a, const uint16_t *b, float2 *y, int n, int np, int batch,
                     hipStream_t s, int tile, const float *sa, const float *sb) {
  if (tile == 0) tile = (np % BM2 == 0 && np >= 512) ? 2 : 1;
  if (tile >= 2 && tile <= 5 && np % BM2 == 0) {
    const int tm = np / BM2, tn = np / BN2;
    const dim3 grid(tm * tn, batch);
    if (tile == 2)
      hipLaunchKernelGGL((k_cgemm_split16_128<E, 4, 4>), grid, dim3(64 * 16), 0, s, a, b, y, n, np, batch, tm, tn, sa, sb);
    else if (tile == 3)
      hipLaunchKernelGGL((k_cgemm_split16_128<E, 2, 4>), grid, dim3(64 * 8), 0, s, a, b, y, n, np, batch, tm, tn, sa, sb);
    else if (tile == 4)
      hipLaunchKernelGGL((k_cgemm_split16_128<E, 4, 2>), grid, dim3(64 * 8), 0, s, a, b, y, n, np, batch, tm, tn, sa, sb);
    else
      hipLaunchKernelGGL((k_cgemm_split16_128<E, 2, 2>), grid, dim3(64 * 4), 0, s, a, b, y, n, np, batch, tm, tn, sa, sb);
  } else {
    const int tm = np / BM, tn = np / BN;
    hipLaunchKernelGGL((k_cgemm_split16<E>), dim3(tm * tn, batch), dim3(NT), 0, s, a, b, y, n, np, batch,
                       tm, tn, sa, sb);
  }
}

}  // namespace

void launch_cgemm_bf16x3(const uint16_t *a, const uint16_t *b, float2 *y, int n, int np, int batch,
                         hipStream_t s, int tile) {
  launch_e<0>(a, b, y, n, np, batch, s, tile, nullptr, nullptr);
}

void launch_cgemm_f16x3(const uint16_t *a, const uint16_t *b, float2 *y, int n, int np, int batch,
                        const float *sa, const float *sb, hipStream_t s, int tile) {
  launch_e<1>(a, b, y, n, np, batch, s, tile, sa, sb);
}

}  // namespace vgtb
