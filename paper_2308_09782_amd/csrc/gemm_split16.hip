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
// The imaginary part is accumulated as +Im in even 32-deep stages and as -Im in
// odd ones (operands and accumulator negated, which is exact): the matrix
// instruction's accumulation is biased toward -infinity (on random operands
// about -0.09 ulp of the largest term per instruction), and in Y - Y^dag the
// imaginary parts of (i, j) and (j, i) add, so an unalternated bias would drift
// the density at every step; alternating the sign cancels it.  The real parts
// subtract in Y - Y^dag, so their biases cancel by themselves.
//
// Operand storage (16-bit planes, p = re_hi, re_lo, im_hi, im_lo; np = padded N,
// a multiple of 64, zero-filled beyond N):
//   A (bf16 form): kADither copies of the four planes, whose lo planes carry
//      dithered roundings of the constant S^-1 - I; the product of step n
//      reads copy n mod kADither (lev_ctr = the device step counter; the
//      plainly rounded middle copy without it).  The fp16 form has one copy;
//   A: plane p, batch k: row-major np x np            (A[i][kk] at i*np + kk)
//   B: plane p, batch k: k-packed (np/8) x np x 8     (B[kk][j] at ((kk/8)*np + j)*8 + kk%8)
// so that the eight consecutive kk one lane feeds to an MFMA are 16 bytes.
// Output: row-major N x N complex64.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

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

// The copy of A for this step (see kADither): bf16 only, the fp16 form keeps one.
template <int E>
__device__ inline const uint16_t *a_copy(const uint16_t *A, const int64_t *lev_ctr, size_t plane) {
  if constexpr (E != 0) return A;
  const int lev = lev_ctr != nullptr ? (int)(*lev_ctr % kADither) : kADither / 2;
  return A + (size_t)lev * 4 * plane;
}

constexpr int BM = 64, BN = 64, BK = 32;   // workgroup tile; 4 wavefronts of 32x32
constexpr int NT = 256;
constexpr int APAD = 40;                    // 16-bit values per LDS row of A (32 + 8 pad)

template <int E>
__global__ __launch_bounds__(NT) void k_cgemm_split16(const uint16_t *__restrict__ A0,
                                                     const uint16_t *__restrict__ B,
                                                     float2 *__restrict__ Y, int n, int np,
                                                     int batch_count, int tiles_m, int tiles_n,
                                                     const float *__restrict__ sa,
                                                     const float *__restrict__ sb,
                                                     const int64_t *__restrict__ lev_ctr) {
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
  const uint16_t *__restrict__ A = a_copy<E>(A0, lev_ctr, plane);
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
    const bool flip = (kt & 1) != 0;   // odd stages accumulate -Im
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const u32x4 nih = negate8(fa[a][2]), nil = negate8(fa[a][3]);
      const u32x4 i0 = flip ? negate8(fa[a][0]) : fa[a][0], i1 = flip ? negate8(fa[a][1]) : fa[a][1];
      const u32x4 i2 = flip ? nih : fa[a][2], i3 = flip ? nil : fa[a][3];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        v4f r = cr[a][b], m = flip ? -ci[a][b] : ci[a][b];
        // Re += ar br - ai bi
        r = mma<E>(fa[a][0], fb[b][0], r);
        r = mma<E>(fa[a][0], fb[b][1], r);
        r = mma<E>(fa[a][1], fb[b][0], r);
        r = mma<E>(nih, fb[b][2], r);
        r = mma<E>(nih, fb[b][3], r);
        r = mma<E>(nil, fb[b][2], r);
        // Im += ar bi + ai br (its negative in odd stages)
        m = mma<E>(i0, fb[b][2], m);
        m = mma<E>(i0, fb[b][3], m);
        m = mma<E>(i1, fb[b][2], m);
        m = mma<E>(i2, fb[b][0], m);
        m = mma<E>(i2, fb[b][1], m);
        m = mma<E>(i3, fb[b][0], m);
        cr[a][b] = r;
        ci[a][b] = flip ? -m : m;
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

// The main loop of one 128 x 128 tile (rows bm.., columns bn.. of the batch
// entry at element offset boff): zeroes and fills the accumulators cr, ci of
// this wavefront.  Ends with a workgroup barrier, after which LDS is free.
template <int E, int WGM, int WGN>
__device__ __forceinline__ void split128_accumulate(
    const uint16_t *__restrict__ A, const uint16_t *__restrict__ B, int np, size_t plane, size_t boff,
    int bm, int bn, u32x4 (&As)[2][4][BM2][APAD / 8], u32x4 (&Bs)[2][4][BK / 8][BN2],
    v4f (&cr)[BM2 / WGM / 16][BN2 / WGN / 16], v4f (&ci)[BM2 / WGM / 16][BN2 / WGN / 16]) {
  constexpr int NT2 = 64 * WGM * WGN;
  constexpr int TM = BM2 / WGM / 16, TN = BN2 / WGN / 16;
  constexpr int LD = 2048 / NT2;             // u32x4 per thread per operand and stage
  // An opaque copy of the thread index: a kernel that runs this loop twice
  // must not keep the lane offsets of the second loop live through the first.
  int tid;
  asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"((int)threadIdx.x));
  const int lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WGN) * (BM2 / WGM), wn0 = (wave % WGN) * (BN2 / WGN);
  const int lr = lane & 15, lg = lane >> 4;
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
  // FLIP: the stage accumulates -Im into ci (the caller negates ci around it);
  // its imaginary-part operands are then -A: the two im planes of A are needed
  // only negated (nf2, nf3), so fa[a][2], fa[a][3] take -re_hi, -re_lo.
  auto stage = [&](int kt, int cur, u32x4 (&ra)[LD], u32x4 (&rb)[LD], auto flip_tag) {
    constexpr bool FLIP = decltype(flip_tag)::value;
    u32x4 fa[TM][4], nf2[TM], nf3[TM], fb0[TN], fb1[TN];
#pragma unroll
    for (int a = 0; a < TM; ++a) {
#pragma unroll
      for (int p = 0; p < 4; ++p) fa[a][p] = As[cur][p][wm0 + a * 16 + lr][lg];
      nf2[a] = negate8(fa[a][2]);
      nf3[a] = negate8(fa[a][3]);
      if (FLIP) {
        fa[a][2] = negate8(fa[a][0]);
        fa[a][3] = negate8(fa[a][1]);
      }
    }
    // Operands of the imaginary part: ai (with B re planes), ar (with B im planes).
    auto ai_hi = [&](int a) -> const u32x4 & { return FLIP ? nf2[a] : fa[a][2]; };
    auto ai_lo = [&](int a) -> const u32x4 & { return FLIP ? nf3[a] : fa[a][3]; };
    auto ar_hi = [&](int a) -> const u32x4 & { return FLIP ? fa[a][2] : fa[a][0]; };
    auto ar_lo = [&](int a) -> const u32x4 & { return FLIP ? fa[a][3] : fa[a][1]; };
    VG_READB(fb0, cur, 0);
    VG_READB(fb1, cur, 1);
    // B plane 0 (re_hi): Re += Ar_hi Br_hi + Ar_lo Br_hi;  Im += Ai_hi Br_hi + Ai_lo Br_hi
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        cr[a][b] = mma<E>(fa[a][0], fb0[b], cr[a][b]);
        ci[a][b] = mma<E>(ai_hi(a), fb0[b], ci[a][b]);
        cr[a][b] = mma<E>(fa[a][1], fb0[b], cr[a][b]);
        ci[a][b] = mma<E>(ai_lo(a), fb0[b], ci[a][b]);
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
        ci[a][b] = mma<E>(ai_hi(a), fb1[b], ci[a][b]);
      }
    VG_READB(fb1, cur, 3);
    // B plane 2 (im_hi): Re -= Ai_hi Bi_hi + Ai_lo Bi_hi;  Im += Ar_hi Bi_hi + Ar_lo Bi_hi
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        cr[a][b] = mma<E>(nf2[a], fb0[b], cr[a][b]);
        ci[a][b] = mma<E>(ar_hi(a), fb0[b], ci[a][b]);
        cr[a][b] = mma<E>(nf3[a], fb0[b], cr[a][b]);
        ci[a][b] = mma<E>(ar_lo(a), fb0[b], ci[a][b]);
      }
    // B plane 3 (im_lo): Re -= Ai_hi Bi_lo;  Im += Ar_hi Bi_lo
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        cr[a][b] = mma<E>(nf2[a], fb1[b], cr[a][b]);
        ci[a][b] = mma<E>(ar_hi(a), fb1[b], ci[a][b]);
      }
    __syncthreads();
  };

  VG_LOAD128(ra0, rb0, 0);
  VG_STORE128(ra0, rb0, 0);
  __syncthreads();
  if (nkt > 1) VG_LOAD128(ra0, rb0, BK);                 // stage 1, stored during stage 0
  if (PF == 2 && nkt > 2) VG_LOAD128(ra1, rb1, 2 * BK);  // stage 2, stored during stage 1
  // Even stages accumulate +Im, odd ones -Im (ci negated around them).
  auto negate_ci = [&] {
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b) ci[a][b] = -ci[a][b];
  };
  for (int kt = 0; kt < nkt; kt += 2) {
    stage(kt, 0, ra0, rb0, std::false_type{});
    negate_ci();
    if (PF == 2) stage(kt + 1, 1, ra1, rb1, std::true_type{});
    else stage(kt + 1, 1, ra0, rb0, std::true_type{});
    negate_ci();
  }
#undef VG_LOAD128
#undef VG_STORE128
#undef VG_READB
#undef AROW
#undef ACOL

}

template <int E, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void k_cgemm_split16_128(const uint16_t *__restrict__ A0,
                                                                     const uint16_t *__restrict__ B,
                                                                     float2 *__restrict__ Y, int n,
                                                                     int np, int batch_count,
                                                                     int tiles_m, int tiles_n,
                                                                     const float *__restrict__ sa,
                                                                     const float *__restrict__ sb,
                                                                     const int64_t *__restrict__ lev_ctr) {
  constexpr int TM = BM2 / WGM / 16, TN = BN2 / WGN / 16;
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
  const uint16_t *__restrict__ A = a_copy<E>(A0, lev_ctr, plane);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm0 = (wave / WGN) * (BM2 / WGM), wn0 = (wave % WGN) * (BN2 / WGN);
  const int lr = lane & 15, lg = lane >> 4;

  v4f cr[TM][TN], ci[TM][TN];
  split128_accumulate<E, WGM, WGN>(A, B, np, plane, boff, bm, bn, As, Bs, cr, ci);

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

// The dense product fused with the leapfrog update of the deviation form
// (Eq. 13 on Eq. 6): D_out = D_base - i fac (Y - Y^dag) (+ fac m0) with
// Y = G + W in FP64, G = (S^-1 - I) W the reduced product.  Y - Y^dag pairs
// element (i, j) with (j, i), so the unit of work is a pair of mirrored
// 128 x 128 tiles: a workgroup computes G of tile (I, J) (I < J), writes it to
// Y, computes G of tile (J, I) in registers, and then forms both tiles of
// D_out; a diagonal tile (I, I) is a unit of its own.  Only the workgroup of a
// unit touches its tiles of Y and D, so no workgroup waits for another.  Per
// batch entry the T (T - 1) / 2 pairs come first, then the T diagonal tiles
// (the dispatch then balances eight tiles per CU on a 16 x 16 tile grid); with
// a multiple of eight batch entries each XCD takes whole batch entries.  The
// arithmetic of every output element is that of k_update (same FP64 sums in
// the same order), so the results are the same bits.
//
// Epilogue of one 16 x 16 MFMA tile (a, b) of a wavefront: own elements
// (R0 + 4 lg + j, C0 + lr) from the registers, mirror elements
// (C0 + 4 lg + j, R0 + lr) from Y; each is formed in FP64 and passed through
// per-wavefront LDS buffers to the lane that needs it transposed.
template <int E, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void k_cgemm_split16_128_update(
    const uint16_t *__restrict__ A0, const uint16_t *__restrict__ B, float2 *__restrict__ Y,
    const float2 *__restrict__ W, const double2 *__restrict__ m0, const double2 *dbase,
    double2 *dout, int n, int np, int batch_count, int T, double fac, const float *__restrict__ sa,
    const float *__restrict__ sb, const int64_t *__restrict__ lev_ctr) {
  constexpr int TM = BM2 / WGM / 16, TN = BN2 / WGN / 16;
  __shared__ u32x4 As[2][4][BM2][APAD / 8];
  __shared__ u32x4 Bs[2][4][BK / 8][BN2];

  const int units = T * (T + 1) / 2, npairs = T * (T - 1) / 2;
  const int lin = xcd_slot(blockIdx.x, units * batch_count);
  const int batch = lin / units;
  const int u = lin % units;
  // Pairs in blocks of four tile rows, column-major within a block (like
  // grouped_tile), so that the units resident together share operand panels.
  int ti = 0, tj = 0;
  const bool pair = u < npairs;
  if (pair) {
    int rem = u;
    for (int g0 = 0; g0 < T; g0 += 4) {
      const int g1 = min(g0 + 4, T);
      int cnt = 0;   // pairs (I, J) with I in [g0, g1), J > I
      for (int i = g0; i < g1; ++i) cnt += T - 1 - i;
      if (rem >= cnt) {
        rem -= cnt;
        continue;
      }
      for (int j = g0 + 1; j < T; ++j) {
        const int rows = min(g1, j) - g0;   // I in [g0, min(g1, j))
        if (rem < rows) {
          ti = g0 + rem;
          tj = j;
          break;
        }
        rem -= rows;
      }
      break;
    }
  } else {
    ti = tj = u - npairs;
  }

  const size_t plane = (size_t)batch_count * np * np;
  const size_t boff = (size_t)batch * np * np;
  const uint16_t *__restrict__ A = a_copy<E>(A0, lev_ctr, plane);
  const size_t base = (size_t)batch * n * n;
  float2 *Yb = Y + base;
  const float2 *Wb = W + base;
  const float us = unscale(sa, sb, batch);
  // The lane-dependent indices of the stores are formed after each main loop
  // from an opaque copy of the thread index, so that the compiler does not keep
  // them live through the loops (the 16-wavefront tile has no registers to spare).
  auto opaque_tid = [] {
    int t;
    asm volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
    return t;
  };

  v4f cr[TM][TN], ci[TM][TN];
  // Tile (I, J): G to Y.
  split128_accumulate<E, WGM, WGN>(A, B, np, plane, boff, ti * BM2, tj * BN2, As, Bs, cr, ci);
  {
    const int tid = opaque_tid(), lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave / WGN) * (BM2 / WGM), wn0 = (wave % WGN) * (BN2 / WGN);
    const int lr = lane & 15, lg = lane >> 4;
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = ti * BM2 + wm0 + a * 16 + 4 * lg + j;
          const int col = tj * BN2 + wn0 + b * 16 + lr;
          if (row < n && col < n)
            Yb[(size_t)row * n + col] = make_float2(us * cr[a][b][j], us * ci[a][b][j]);
        }
  }
  // Own tile in registers: (J, I) for a pair, else (I, I) (the accumulators as they are).
  if (pair) split128_accumulate<E, WGM, WGN>(A, B, np, plane, boff, tj * BM2, ti * BN2, As, Bs, cr, ci);
  __syncthreads();   // every wavefront's stores to Y are visible to the workgroup; LDS is free
  const int tid = opaque_tid(), lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WGN) * (BM2 / WGM), wn0 = (wave % WGN) * (BN2 / WGN);
  const int lr = lane & 15, lg = lane >> 4;
  const int obm = tj * BM2, obn = ti * BN2;   // own tile rows, columns
  // Per wavefront: own Y values (16 x 17 doubles2, in the A stages) and mirror
  // Y values (16 x 16, rotated by the row so that transposed reads hit
  // distinct banks, in the B stages).
  double2 *yob = reinterpret_cast<double2 *>(&As[0][0][0][0]) + wave * (16 * 17);
  double2 *ymb = reinterpret_cast<double2 *>(&Bs[0][0][0][0]) + wave * (16 * 16);
  auto ym_at = [&](int p, int q) -> double2 & { return ymb[p * 16 + ((p + q) & 15)]; };

  auto out = [&](int row, int col, double2 yv, double2 yt) {
    const size_t idx = base + (size_t)row * n + col;
    const double xr = yv.x - yt.x;           // X = Y - conj(Y^T)
    const double xi = yv.y + yt.y;
    const double2 bv = dbase[idx];
    double2 o = make_double2(bv.x + fac * xi, bv.y - fac * xr);
    if (m0 != nullptr) {
      const double2 mv = m0[idx];
      o.x += fac * mv.x;
      o.y += fac * mv.y;
    }
    dout[idx] = o;
  };
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int R0 = obm + wm0 + a * 16, C0 = obn + wn0 + b * 16;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = 4 * lg + j;
        double2 yo = make_double2(0.0, 0.0);            // own element (R0 + r, C0 + lr)
        if (R0 + r < n && C0 + lr < n) {
          const float2 w = Wb[(size_t)(R0 + r) * n + C0 + lr];
          yo = make_double2((double)(us * cr[a][b][j]), (double)(us * ci[a][b][j]));
          yo.x += (double)w.x;
          yo.y += (double)w.y;
        }
        yob[r * 17 + lr] = yo;
        double2 ym = make_double2(0.0, 0.0);            // mirror element (C0 + r, R0 + lr)
        if (C0 + r < n && R0 + lr < n) {
          const size_t mi = (size_t)(C0 + r) * n + R0 + lr;
          const float2 g = Yb[mi];
          const float2 w = Wb[mi];
          ym = make_double2((double)g.x, (double)g.y);
          ym.x += (double)w.x;
          ym.y += (double)w.y;
        }
        ym_at(r, lr) = ym;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = 4 * lg + j, c = lr;
        // Own output (R0 + r, C0 + c), paired with Y(C0 + c, R0 + r).
        if (R0 + r < n && C0 + c < n) out(R0 + r, C0 + c, yob[r * 17 + c], ym_at(c, r));
        // Mirror output (C0 + r, R0 + c), paired with Y(R0 + c, C0 + r); a
        // diagonal tile is its own mirror and writes its own outputs only.
        if (pair && C0 + r < n && R0 + c < n) out(C0 + r, R0 + c, ym_at(r, c), yob[c * 17 + r]);
      }
      __syncthreads();
    }
}

// tile: 1 = 64 x 64 (four wavefronts); 128 x 128 (np a multiple of 128 only)
// with 2 = sixteen wavefronts of 32 x 32, 3 = eight of 64 x 32, 4 = eight of
// 32 x 64, 5 = four of 64 x 64 (fewer LDS fragment reads per matrix
// instruction, fewer wavefronts to cover stalls); 0 = 2 where allowed from
// np = 512 up, else 1.
template <int E>
static void launch_e(const uint16_t *a, const uint16_t *b, float2 *y, int n, int np, int batch,
                     hipStream_t s, int tile, const float *sa, const float *sb,
                     const int64_t *lev_ctr) {
  if (tile == 0) tile = split16_default_tile(np);
  if (tile >= 2 && tile <= 5 && np % BM2 == 0) {
    const int tm = np / BM2, tn = np / BN2;
    const dim3 grid(tm * tn, batch);
    if (tile == 2)
      hipLaunchKernelGGL((k_cgemm_split16_128<E, 4, 4>), grid, dim3(64 * 16), 0, s, a, b, y, n, np, batch, tm, tn, sa, sb, lev_ctr);
    else if (tile == 3)
      hipLaunchKernelGGL((k_cgemm_split16_128<E, 2, 4>), grid, dim3(64 * 8), 0, s, a, b, y, n, np, batch, tm, tn, sa, sb, lev_ctr);
    else if (tile == 4)
      hipLaunchKernelGGL((k_cgemm_split16_128<E, 4, 2>), grid, dim3(64 * 8), 0, s, a, b, y, n, np, batch, tm, tn, sa, sb, lev_ctr);
    else
      hipLaunchKernelGGL((k_cgemm_split16_128<E, 2, 2>), grid, dim3(64 * 4), 0, s, a, b, y, n, np, batch, tm, tn, sa, sb, lev_ctr);
  } else {
    const int tm = np / BM, tn = np / BN;
    hipLaunchKernelGGL((k_cgemm_split16<E>), dim3(tm * tn, batch), dim3(NT), 0, s, a, b, y, n, np, batch,
                       tm, tn, sa, sb, lev_ctr);
  }
}

template <int E>
static bool launch_update_e(const uint16_t *a, const uint16_t *b, float2 *y, const float2 *w,
                            const double2 *m0, const double2 *dbase, double2 *dout, int n, int np,
                            int batch, double fac, int64_t *ctr, hipStream_t s, int tile,
                            const float *sa, const float *sb) {
  if (tile == 0) tile = split16_default_tile(np);
  if (tile < 2 || tile > 5 || np % BM2 != 0) return false;
  const int T = np / BM2;
  const dim3 grid(T * (T + 1) / 2 * batch);
#define VG_UPD(WGM, WGN)                                                                           \
  hipLaunchKernelGGL((k_cgemm_split16_128_update<E, WGM, WGN>), grid, dim3(64 * WGM * WGN), 0, s, a, b, y, \
                     w, m0, dbase, dout, n, np, batch, T, fac, sa, sb, ctr)
  if (tile == 2) VG_UPD(4, 4);
  else if (tile == 3) VG_UPD(2, 4);
  else if (tile == 4) VG_UPD(4, 2);
  else VG_UPD(2, 2);
#undef VG_UPD
  // The step is done once the product and update have run: advance the device
  // step index (a launch of its own: every workgroup reads it for its copy of A).
  if (ctr != nullptr) launch_advance_counter(ctr, s);
  return true;
}

}  // namespace

int split16_default_tile(int np) { return (np % BM2 == 0 && np >= 512) ? 2 : 1; }

bool launch_cgemm_update_split16(int fmt, const uint16_t *a, const uint16_t *b, float2 *y,
                                 const float2 *w, const double2 *m0, const double2 *dbase,
                                 double2 *dout, int n, int np, int batch, double fac, int64_t *ctr,
                                 const float *sa, const float *sb, hipStream_t s, int tile) {
  if (fmt == 3) return launch_update_e<1>(a, b, y, w, m0, dbase, dout, n, np, batch, fac, ctr, s, tile, sa, sb);
  return launch_update_e<0>(a, b, y, w, m0, dbase, dout, n, np, batch, fac, ctr, s, tile, nullptr, nullptr);
}

void launch_cgemm_bf16x3(const uint16_t *a, const uint16_t *b, float2 *y, int n, int np, int batch,
                         hipStream_t s, int tile, const int64_t *lev_ctr) {
  launch_e<0>(a, b, y, n, np, batch, s, tile, nullptr, nullptr, lev_ctr);
}

void launch_cgemm_f16x3(const uint16_t *a, const uint16_t *b, float2 *y, int n, int np, int batch,
                        const float *sa, const float *sb, hipStream_t s, int tile) {
  launch_e<1>(a, b, y, n, np, batch, s, tile, sa, sb, nullptr);
}

}  // namespace vgtb
