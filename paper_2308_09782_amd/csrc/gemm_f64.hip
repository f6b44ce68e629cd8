// Batched complex128 GEMM C = A * B (row-major N x N per batch entry) on the
// gfx950 FP64 matrix cores: the dense product S_k^-1 (H_k D_k) of Eq. 6.
//
// Each complex multiply-accumulate is four real v_mfma_f64_16x16x4f64 on
// interleaved (re, im) operands: Cr += ar br - ai bi, Ci += ar bi + ai br.
// A workgroup owns a BM x BN output tile; its WM x WN wavefronts each own a
// (BM/WM) x (BN/WN) sub-tile made of 16 x 16 MFMA tiles.  Operand tiles of
// depth BK are staged through LDS (A stored k-major so that the sixteen
// lanes of an MFMA row group read consecutive addresses), double-buffered
// with a register prefetch of the next tile.  Ragged edges are zero-filled.
#include <hip/hip_runtime.h>

#include "vgtb_internal.h"

namespace vgtb {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

template <int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(WM *WN * 64) void k_zgemm_f64(const double2 *__restrict__ A,
                                                          const double2 *__restrict__ B,
                                                          double2 *__restrict__ C, int n,
                                                          int tiles_m, int tiles_n) {
  constexpr int NT = WM * WN * 64;
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  constexpr int LA = BM * BK / NT;   // complex elements of A per thread per stage
  constexpr int LB = BN * BK / NT;
  static_assert(LA * NT == BM * BK && LB * NT == BN * BK, "tile / thread mismatch");
  __shared__ double2 As[2][BK][BM + 1];
  __shared__ double2 Bs[2][BK][BN + 1];

  // XCD-aware tile order: consecutive workgroup ids land on different XCDs,
  // so give each XCD a contiguous run of tiles (same A rows, same batch).
  const int tiles = tiles_m * tiles_n;
  const int nwg = tiles * gridDim.y;
  int lin = blockIdx.x + blockIdx.y * tiles;
  if ((nwg & 7) == 0) lin = (lin & 7) * (nwg >> 3) + (lin >> 3);
  const int batch = lin / tiles;
  const int tile = lin % tiles;
  const int bm = (tile / tiles_n) * BM;
  const int bn = (tile % tiles_n) * BN;

  const size_t boff = (size_t)batch * n * n;
  const double2 *Ab = A + boff;
  const double2 *Bb = B + boff;
  double2 *Cb = C + boff;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave / WN) * (BM / WM);
  const int wn0 = (wave % WN) * (BN / WN);

  v4d cr[TM][TN], ci[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      cr[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
      ci[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    }

  double2 ra[LA], rb[LB];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int L = tid + i * NT;
      const int m = L / BK, kk = L % BK;
      const int gm = bm + m, gk = k0 + kk;
      ra[i] = (gm < n && gk < n) ? Ab[(size_t)gm * n + gk] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int L = tid + i * NT;
      const int kk = L / BN, c = L % BN;
      const int gk = k0 + kk, gc = bn + c;
      rb[i] = (gk < n && gc < n) ? Bb[(size_t)gk * n + gc] : make_double2(0.0, 0.0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int L = tid + i * NT;
      As[buf][L % BK][L / BK] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int L = tid + i * NT;
      Bs[buf][L / BN][L % BN] = rb[i];
    }
  };

  const int nkt = (n + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  int buf = 0;
  const int lr = lane & 15, lk = lane >> 4;
  for (int kt = 0; kt < nkt; ++kt) {
    if (kt + 1 < nkt) load((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double2 fa[TM], fb[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) fa[a] = As[buf][ks + lk][wm0 + a * 16 + lr];
#pragma unroll
      for (int b = 0; b < TN; ++b) fb[b] = Bs[buf][ks + lk][wn0 + b * 16 + lr];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a].x, fb[b].x, cr[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a].x, fb[b].y, ci[a][b], 0, 0, 0);
        }
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-fa[a].y, fb[b].y, cr[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a].y, fb[b].x, ci[a][b], 0, 0, 0);
        }
    }
    if (kt + 1 < nkt) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // Output layout of the 16x16 f64 MFMA: element j of a lane is row lane/16 + 4*j,
  // column lane%16.
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = bm + wm0 + a * 16 + lk + 4 * j;
        const int col = bn + wn0 + b * 16 + lr;
        if (row < n && col < n) Cb[(size_t)row * n + col] = make_double2(cr[a][b][j], ci[a][b][j]);
      }
}

template <int BM, int BN, int BK, int WM, int WN>
void run(const double2 *a, const double2 *b, double2 *c, int n, int batch, hipStream_t s) {
  const int tm = (n + BM - 1) / BM, tn = (n + BN - 1) / BN;
  hipLaunchKernelGGL((k_zgemm_f64<BM, BN, BK, WM, WN>), dim3(tm * tn, batch), dim3(WM * WN * 64),
                     0, s, a, b, c, n, tm, tn);
}

}  // namespace

void launch_zgemm_f64(const double2 *a, const double2 *b, double2 *c, int n, int batch,
                      hipStream_t s) {
  if (n >= 1024)
    run<64, 64, 16, 2, 2>(a, b, c, n, batch, s);
  else
    run<32, 32, 16, 2, 2>(a, b, c, n, batch, s);
}

}  // namespace vgtb
