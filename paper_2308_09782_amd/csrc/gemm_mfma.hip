// Batched complex GEMM C = A * B (row-major N x N per batch entry) on the
// gfx950 matrix cores: the dense product S_k^-1 (H_k D_k) of Eq. 6, in
// complex128 (v_mfma_f64_16x16x4f64) or complex64 (v_mfma_f32_16x16x4f32).
//
// Each complex multiply-accumulate is four real MFMAs on interleaved
// (re, im) operands: Cr += ar br - ai bi, Ci += ar bi + ai br.
// A workgroup owns a BM x BN output tile (XCD-aware, grouped tile order); its
// WM x WN wavefronts each own a
// (BM/WM) x (BN/WN) sub-tile made of 16 x 16 MFMA tiles.  Operand tiles of
// depth BK are staged through LDS (A stored k-major so that the sixteen
// lanes of an MFMA row group read consecutive addresses), double-buffered
// with a register prefetch of the next tile.  Ragged edges are zero-filled.
#include <hip/hip_runtime.h>

#include "vgtb_internal.h"

namespace vgtb {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Element traits: complex type, accumulator, one 16x16x4 MFMA, and the row
// of accumulator element j of a lane (the f64 and f32 forms differ).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  using C2 = double2;
  using Acc = v4d;
  static __device__ inline Acc mac(double a, double b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lk, int j) { return lk + 4 * j; }
  static __device__ inline C2 make(double x, double y) { return make_double2(x, y); }
};
template <> struct Mfma<float> {
  using C2 = float2;
  using Acc = v4f;
  static __device__ inline Acc mac(float a, float b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lk, int j) { return 4 * lk + j; }
  static __device__ inline C2 make(float x, float y) { return make_float2(x, y); }
};

template <typename T, int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(WM *WN * 64) void k_zgemm(const typename Mfma<T>::C2 *__restrict__ A,
                                                      const typename Mfma<T>::C2 *__restrict__ B,
                                                      typename Mfma<T>::C2 *__restrict__ C, int n,
                                                      int tiles_m, int tiles_n) {
  using M = Mfma<T>;
  using C2 = typename M::C2;
  using Acc = typename M::Acc;
  constexpr int NT = WM * WN * 64;
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  constexpr int LA = BM * BK / NT;   // complex elements of A per thread per stage
  constexpr int LB = BN * BK / NT;
  static_assert(LA * NT == BM * BK && LB * NT == BN * BK, "tile / thread mismatch");
  __shared__ C2 As[2][BK][BM + 1];
  __shared__ C2 Bs[2][BK][BN + 1];

  // XCD-aware tile order: consecutive workgroup ids land on different XCDs,
  // so give each XCD a contiguous run of tiles (same A rows, same batch).
  const int tiles = tiles_m * tiles_n;
  const int lin = xcd_slot(blockIdx.x + blockIdx.y * tiles, tiles * gridDim.y);
  const int batch = lin / tiles;
  int tm, tn;
  grouped_tile(lin % tiles, tiles_m, tiles_n, 8, tm, tn);
  const int bm = tm * BM;
  const int bn = tn * BN;

  const size_t boff = (size_t)batch * n * n;
  const C2 *Ab = A + boff;
  const C2 *Bb = B + boff;
  C2 *Cb = C + boff;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave / WN) * (BM / WM);
  const int wn0 = (wave % WN) * (BN / WN);

  Acc cr[TM][TN], ci[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      cr[a][b] = Acc{0, 0, 0, 0};
      ci[a][b] = Acc{0, 0, 0, 0};
    }

  C2 ra[LA], rb[LB];
  // Global -> registers for the stage at depth k0 (zero outside the matrix).
#define VG_LOAD(k0)                                                                   \
  do {                                                                                \
    _Pragma("unroll") for (int i = 0; i < LA; ++i) {                                  \
      const int L = tid + i * NT;                                                     \
      const int gm = bm + L / BK, gk = (k0) + L % BK;                                 \
      if (gm < n && gk < n) ra[i] = Ab[(size_t)gm * n + gk];                          \
      else ra[i] = M::make(0, 0);                                                     \
    }                                                                                 \
    _Pragma("unroll") for (int i = 0; i < LB; ++i) {                                  \
      const int L = tid + i * NT;                                                     \
      const int gk = (k0) + L / BN, gc = bn + L % BN;                                 \
      if (gk < n && gc < n) rb[i] = Bb[(size_t)gk * n + gc];                          \
      else rb[i] = M::make(0, 0);                                                     \
    }                                                                                 \
  } while (0)
  // Registers -> LDS buffer buf (A stored k-major).
#define VG_STORE(buf)                                                                 \
  do {                                                                                \
    _Pragma("unroll") for (int i = 0; i < LA; ++i) {                                  \
      const int L = tid + i * NT;                                                     \
      As[buf][L % BK][L / BK] = ra[i];                                                \
    }                                                                                 \
    _Pragma("unroll") for (int i = 0; i < LB; ++i) {                                  \
      const int L = tid + i * NT;                                                     \
      Bs[buf][L / BN][L % BN] = rb[i];                                                \
    }                                                                                 \
  } while (0)

  const int nkt = (n + BK - 1) / BK;
  VG_LOAD(0);
  VG_STORE(0);
  __syncthreads();
  int buf = 0;
  const int lr = lane & 15, lk = lane >> 4;
  for (int kt = 0; kt < nkt; ++kt) {
    if (kt + 1 < nkt) VG_LOAD((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      C2 fa[TM], fb[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) fa[a] = As[buf][ks + lk][wm0 + a * 16 + lr];
#pragma unroll
      for (int b = 0; b < TN; ++b) fb[b] = Bs[buf][ks + lk][wn0 + b * 16 + lr];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          cr[a][b] = M::mac(fa[a].x, fb[b].x, cr[a][b]);
          ci[a][b] = M::mac(fa[a].x, fb[b].y, ci[a][b]);
        }
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          cr[a][b] = M::mac(-fa[a].y, fb[b].y, cr[a][b]);
          ci[a][b] = M::mac(fa[a].y, fb[b].x, ci[a][b]);
        }
    }
    if (kt + 1 < nkt) VG_STORE(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // Output layout: element j of a lane is row M::row(lane/16, j), column lane%16
  // (f64: lane/16 + 4j; f32: 4 (lane/16) + j).
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = bm + wm0 + a * 16 + M::row(lk, j);
        const int col = bn + wn0 + b * 16 + lr;
        if (row < n && col < n) Cb[(size_t)row * n + col] = M::make(cr[a][b][j], ci[a][b][j]);
      }
#undef VG_LOAD
#undef VG_STORE
}

template <typename T, int BM, int BN, int BK, int WM, int WN>
void run(const typename Mfma<T>::C2 *a, const typename Mfma<T>::C2 *b, typename Mfma<T>::C2 *c,
         int n, int batch, hipStream_t s) {
  const int tm = (n + BM - 1) / BM, tn = (n + BN - 1) / BN;
  hipLaunchKernelGGL((k_zgemm<T, BM, BN, BK, WM, WN>), dim3(tm * tn, batch), dim3(WM * WN * 64),
                     0, s, a, b, c, n, tm, tn);
}

}  // namespace

int zgemm_default_tile(int n) { return n >= 1024 ? 2 : 1; }

// tile: 1 = 32 x 32, 2 = 64 x 64 (four wavefronts), 3 = 128 x 64 (eight);
// 0 = 64 x 64 from N = 1024 up, else 32 x 32.
template <typename T>
static void run_tile(const typename Mfma<T>::C2 *a, const typename Mfma<T>::C2 *b,
                     typename Mfma<T>::C2 *c, int n, int batch, int tile, hipStream_t s) {
  if (tile == 0) tile = zgemm_default_tile(n);
  if (tile == 3) run<T, 128, 64, 16, 4, 2>(a, b, c, n, batch, s);
  else if (tile == 2) run<T, 64, 64, 16, 2, 2>(a, b, c, n, batch, s);
  else run<T, 32, 32, 16, 2, 2>(a, b, c, n, batch, s);
}

void launch_zgemm_f64(const double2 *a, const double2 *b, double2 *c, int n, int batch,
                      hipStream_t s, int tile) {
  run_tile<double>(a, b, c, n, batch, tile, s);
}

void launch_cgemm_f32(const float2 *a, const float2 *b, float2 *c, int n, int batch,
                      hipStream_t s, int tile) {
  run_tile<float>(a, b, c, n, batch, tile, s);
}

}  // namespace vgtb
