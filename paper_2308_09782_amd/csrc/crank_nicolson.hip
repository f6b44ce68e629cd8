// Crank-Nicolson propagation of the coefficient vectors (Eq. 5), the unitary
// scheme the paper names beside the density leapfrog:
//
//   (S_k + i tau H_k) C(t + dt) = (S_k - i tau H_k) C(t),   tau = dt / 2,
//
// solved as X = (S + i tau H)^-1 S C and C(t + dt) = 2 X - C(t).  The matrix
// A = S + i tau H has the positive-definite Hermitian part S, so Gaussian
// elimination needs no pivoting (every leading block is invertible).  It is
// done recursively on the augmented matrix [A | S C] (cn_solve): halve the
// block, solve the top half against everything to its right, form the Schur
// complement, solve the bottom half, and back-substitute into the top half;
// after which the S C columns hold X.  The kCnBlock x kCnBlock blocks at the
// leaves are inverted in registers (Gauss-Jordan, one workgroup per k-point);
// every other flop is a strided complex FP64 GEMM on the matrix cores, half of
// them with a depth of N/2.
//
// Observables need D = sum_n f_n C_n C_n^dag (the definition after Eq. 6) only
// on the pair pattern; k_cn_pattern samples it there, and the density-form
// kernels then form charges, current and energy from it unchanged.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "vgtb_internal.h"

namespace vgtb {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline double wave_reduce(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// C = beta C + alpha A B for M x K times K x N operands, each batch entry at
// its own stride; row-major with leading dimensions lda, ldb, ldc.  Complex
// products as four real 16x16x4 FP64 MFMAs on interleaved (re, im) values.
// B may alias C when every workgroup owns whole columns of C (M <= BM) and
// reads only those columns of B (the K rows of B are the M rows of C): each
// workgroup reads its whole slab before it writes it.
template <int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(WM *WN * 64) void k_zgemm_strided(
    const double2 *__restrict__ A, int lda, size_t sa, const double2 *B, int ldb, size_t sb,
    double2 *C, int ldc, size_t sc, int M, int N, int K, double alpha, int beta_one, int tiles_m,
    int tiles_n) {
  constexpr int NT = WM * WN * 64;
  constexpr int TM = BM / WM / 16;
  constexpr int TN = BN / WN / 16;
  constexpr int LA = BM * BK / NT;
  constexpr int LB = BN * BK / NT;
  static_assert(LA * NT == BM * BK && LB * NT == BN * BK, "tile / thread mismatch");
  __shared__ double2 As[2][BK][BM + 1];
  __shared__ double2 Bs[2][BK][BN + 1];

  const int tiles = tiles_m * tiles_n;
  const int lin = xcd_slot(blockIdx.x + blockIdx.y * tiles, tiles * gridDim.y);
  const int batch = lin / tiles;
  int tm, tn;
  grouped_tile(lin % tiles, tiles_m, tiles_n, 8, tm, tn);
  const int bm = tm * BM, bn = tn * BN;
  const double2 *Ab = A + (size_t)batch * sa;
  const double2 *Bb = B + (size_t)batch * sb;
  double2 *Cb = C + (size_t)batch * sc;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave / WN) * (BM / WM);
  const int wn0 = (wave % WN) * (BN / WN);
  v4d cr[TM][TN], ci[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      cr[a][b] = v4d{0, 0, 0, 0};
      ci[a][b] = v4d{0, 0, 0, 0};
    }
  double2 ra[LA], rb[LB];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int L = tid + i * NT;
      const int gm = bm + L / BK, gk = k0 + L % BK;
      ra[i] = (gm < M && gk < K) ? Ab[(size_t)gm * lda + gk] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int L = tid + i * NT;
      const int gk = k0 + L / BN, gc = bn + L % BN;
      rb[i] = (gk < K && gc < N) ? Bb[(size_t)gk * ldb + gc] : make_double2(0.0, 0.0);
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
  const int nkt = (K + BK - 1) / BK;
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
  // Accumulator element j of a lane: row lane/16 + 4j, column lane%16.
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = bm + wm0 + a * 16 + lk + 4 * j;
        const int col = bn + wn0 + b * 16 + lr;
        if (row < M && col < N) {
          double2 *o = Cb + (size_t)row * ldc + col;
          double2 v = make_double2(alpha * cr[a][b][j], alpha * ci[a][b][j]);
          if (beta_one) {
            const double2 old = *o;
            v.x += old.x;
            v.y += old.y;
          }
          *o = v;
        }
      }
}

template <int BM, int BN, int WM, int WN>
void gemm_tile(const double2 *a, int lda, size_t sa, const double2 *b, int ldb, size_t sb, double2 *c,
               int ldc, size_t sc, int m, int n, int k, double alpha, bool beta_one, int batch,
               hipStream_t s) {
  const int tm = (m + BM - 1) / BM, tn = (n + BN - 1) / BN;
  hipLaunchKernelGGL((k_zgemm_strided<BM, BN, 16, WM, WN>), dim3(tm * tn, batch), dim3(WM * WN * 64),
                     0, s, a, lda, sa, b, ldb, sb, c, ldc, sc, m, n, k, alpha, beta_one ? 1 : 0, tm, tn);
}

// Tile shape of the large products (trailing update, back substitution):
// 1 = 64 x 64 (4 waves), 2 = 128 x 64 (8), 3 = 128 x 128 (16); the leaf
// products (small_m) always use 64 x 64.
void gemm_strided(const double2 *a, int lda, size_t sa, const double2 *b, int ldb, size_t sb,
                  double2 *c, int ldc, size_t sc, int m, int n, int k, double alpha, bool beta_one,
                  int batch, hipStream_t s, int big_tile, bool small_m = false) {
  if (m <= 0 || n <= 0 || k <= 0) return;
  const int tile = small_m ? 1 : big_tile;
  if (tile == 3 && m > 64)
    gemm_tile<128, 128, 4, 4>(a, lda, sa, b, ldb, sb, c, ldc, sc, m, n, k, alpha, beta_one, batch, s);
  else if (tile == 2 && m > 64)
    gemm_tile<128, 64, 4, 2>(a, lda, sa, b, ldb, sb, c, ldc, sc, m, n, k, alpha, beta_one, batch, s);
  else
    gemm_tile<64, 64, 2, 2>(a, lda, sa, b, ldb, sb, c, ldc, sc, m, n, k, alpha, beta_one, batch, s);
}

// Inverse of the nb x nb diagonal block at (j0, j0) of each k's augmented
// matrix, by Gauss-Jordan elimination without pivoting; written to inv[k]
// (kCnBlock x kCnBlock, identity outside nb x nb).  The block lives in
// registers: thread t of kInvThreads owns column t % B and rows t / B + W r (four
// rows each, sixteen wavefronts: while one waits, the others issue).  Each pivot step
// publishes the old pivot row and column through LDS (double-buffered, so one
// barrier per step).  With b = 0 on the pivot row and column (else a_ij),
// c = -1 on the pivot row (else a_ip) and t_j = 1/a_pp at j = p (else
// a_pj/a_pp), every entry takes the same update a_ij <- b - c t_j, which is
//   a_pp <- 1/a_pp,  a_pj <- a_pj/a_pp,  a_ip <- -a_ip/a_pp,
//   a_ij <- a_ij - a_ip a_pj / a_pp,
// written with selects only (no branches, no indexed register arrays).
constexpr int kInvThreads = 1024;
__global__ __launch_bounds__(kInvThreads) void k_blk_inv(const double2 *__restrict__ aug, int ld,
                                                         size_t sa, int j0, int nb,
                                                         double2 *__restrict__ inv) {
  constexpr int B = kCnBlock;
  constexpr int W = kInvThreads / B;   // row groups
  constexpr int R = B / W;       // rows per thread
  __shared__ double2 rowb[2][B], colb[2][B];
  const int k = blockIdx.x, tid = threadIdx.x;
  const int j = tid % B, w = tid / B;
  const double2 *src = aug + (size_t)k * sa + (size_t)j0 * ld + j0;
  double ar[R], ai[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = w + W * r;
    const bool in = i < nb && j < nb;
    const double2 v = in ? src[(size_t)i * ld + j] : make_double2(0.0, 0.0);
    ar[r] = in ? v.x : (i == j ? 1.0 : 0.0);
    ai[r] = in ? v.y : 0.0;
  }
  for (int p = 0; p < nb; ++p) {
    const int buf = p & 1;
    const int rp = p / W;
    if (w == p % W) {
      double xr = ar[0], xi = ai[0];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        xr = (r == rp) ? ar[r] : xr;
        xi = (r == rp) ? ai[r] : xi;
      }
      rowb[buf][j] = make_double2(xr, xi);
    }
    if (j == p) {
#pragma unroll
      for (int r = 0; r < R; ++r) colb[buf][w + W * r] = make_double2(ar[r], ai[r]);
    }
    __syncthreads();
    const double2 d = colb[buf][p];
    const double den = 1.0 / (d.x * d.x + d.y * d.y);
    const double pr = d.x * den, pi = -d.y * den;         // 1 / a_pp
    const double2 rv = rowb[buf][j];
    const bool jp = (j == p);
    const double tr = jp ? pr : rv.x * pr - rv.y * pi;    // t_j
    const double ti = jp ? pi : rv.x * pi + rv.y * pr;
    double2 cv[R];   // this thread's rows of the pivot column, all loads in flight at once
#pragma unroll
    for (int r = 0; r < R; ++r) cv[r] = colb[buf][w + W * r];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool ip = (w + W * r == p);
      const double cr = ip ? -1.0 : cv[r].x, ci = ip ? 0.0 : cv[r].y;
      const double br = (ip || jp) ? 0.0 : ar[r], bi = (ip || jp) ? 0.0 : ai[r];
      ar[r] = br - (cr * tr - ci * ti);
      ai[r] = bi - (cr * ti + ci * tr);
    }
  }
  double2 *dst = inv + (size_t)k * B * B;
#pragma unroll
  for (int r = 0; r < R; ++r) dst[(size_t)(w + W * r) * B + j] = make_double2(ar[r], ai[r]);
}

// [A | R] of each k: zeros in A (the pattern is scattered next), R = W[:, :ns].
__global__ void k_cn_fill(double2 *__restrict__ aug, int ld, const double2 *__restrict__ w, int n,
                          int ns) {
  const int k = blockIdx.z, i = blockIdx.y;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n + ns) return;
  const size_t base = (size_t)k * n * ld + (size_t)i * ld;
  aug[base + c] = c < n ? make_double2(0.0, 0.0) : w[((size_t)k * n + i) * n + (c - n)];
}

// A = S + i tau H on the pair pattern (H pair blocks in grouped order q, S in pair order p).
template <int NO>
__global__ void k_cn_scatter(PairGraph g, double2 *__restrict__ aug, int ld, int n,
                             const double2 *__restrict__ hq, const double2 *__restrict__ spk,
                             double tau) {
  constexpr int E2 = NO * NO;
  const int k = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.n_pairs * E2) return;
  const int q = t / E2, e = t % E2;
  const int p = g.gp_pair[q];
  const int I = g.pair_row[p], J = g.pair_col[p];
  const double2 h = hq[((size_t)k * g.n_pairs + q) * E2 + e];
  const double2 sv = spk[((size_t)k * g.n_pairs + p) * E2 + e];
  const size_t at = (size_t)k * n * ld + (size_t)(I * NO + e / NO) * ld + (J * NO + e % NO);
  aug[at] = make_double2(sv.x - tau * h.y, sv.y + tau * h.x);
}

// C(t + dt) = 2 X - C(t), X = the R columns after the solve; the step is done.
__global__ void k_cn_update(const double2 *__restrict__ aug, int ld, double2 *__restrict__ c,
                            int n, int ns, int64_t *ctr) {
  const int k = blockIdx.z, i = blockIdx.y;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < ns) {
    const double2 x = aug[(size_t)k * n * ld + (size_t)i * ld + n + s];
    double2 *o = c + ((size_t)k * n + i) * n + s;
    const double2 old = *o;
    *o = make_double2(2.0 * x.x - old.x, 2.0 * x.y - old.y);
  }
  if (ctr != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0)
    *ctr += 1;
}

// D on the pair pattern: D[I mu][J nu] = sum_s f_s C[I mu][s] conj(C[J nu][s]).
// One wavefront per (pair, k), four pairs per workgroup; each lane sums every
// 64th state (coalesced rows of C), then a shuffle reduction.
template <int NO>
__global__ __launch_bounds__(256) void k_cn_pattern(PairGraph g, const double2 *__restrict__ c,
                                                    const double *__restrict__ occ, int n, int ns,
                                                    double2 *__restrict__ d) {
  constexpr int E2 = NO * NO;
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int k = blockIdx.y;
  if (p >= g.n_pairs) return;   // uniform per wavefront
  const int I = g.pair_row[p], J = g.pair_col[p];
  const double2 *ck = c + (size_t)k * n * n;
  const double *fk = occ + (size_t)k * n;
  double accr[E2], acci[E2];
#pragma unroll
  for (int e = 0; e < E2; ++e) accr[e] = acci[e] = 0.0;
  for (int s = lane; s < ns; s += 64) {
    const double f = fk[s];
    double2 ci[NO], cj[NO];
#pragma unroll
    for (int m = 0; m < NO; ++m) {
      ci[m] = ck[(size_t)(I * NO + m) * n + s];
      const double2 v = ck[(size_t)(J * NO + m) * n + s];
      cj[m] = make_double2(f * v.x, f * v.y);
    }
#pragma unroll
    for (int mu = 0; mu < NO; ++mu)
#pragma unroll
      for (int nu = 0; nu < NO; ++nu) {
        // ci * conj(cj)
        accr[mu * NO + nu] += ci[mu].x * cj[nu].x + ci[mu].y * cj[nu].y;
        acci[mu * NO + nu] += ci[mu].y * cj[nu].x - ci[mu].x * cj[nu].y;
      }
  }
#pragma unroll
  for (int e = 0; e < E2; ++e) {
    accr[e] = wave_reduce(accr[e]);
    acci[e] = wave_reduce(acci[e]);
  }
  if (lane == 0) {
#pragma unroll
    for (int e = 0; e < E2; ++e)
      d[(size_t)k * n * n + (size_t)(I * NO + e / NO) * n + (J * NO + e % NO)] =
          make_double2(accr[e], acci[e]);
  }
}

// SCC potential of the midpoint: (3 V_n - V_{n-1}) / 2, V_{-1} = V_n on the first step.
__global__ void k_cn_vmid(const double *__restrict__ v, double *__restrict__ vprev,
                          double *__restrict__ vmid, int na, int first) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= na) return;
  const double now = v[i];
  vmid[i] = first ? now : 1.5 * now - 0.5 * vprev[i];
  vprev[i] = now;
}

// Coefficients from the eigensolver's vectors (vector s stored conjugated in
// row s): C[i][s] = conj(evec[s][i]) for s < ns; the other columns zero.
__global__ void k_cn_from_vectors(const double2 *__restrict__ evec, double2 *__restrict__ c, int n,
                                  int ns) {
  const int k = blockIdx.z, i = blockIdx.y;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  double2 v = make_double2(0.0, 0.0);
  if (s < ns) {
    const double2 e = evec[(size_t)k * n * n + (size_t)s * n + i];
    v = make_double2(e.x, -e.y);
  }
  c[((size_t)k * n + i) * n + s] = v;
}

// The inverse map (for the dense density): evec[s][i] = conj(C[i][s]), zero for s >= ns.
__global__ void k_cn_to_vectors(const double2 *__restrict__ c, double2 *__restrict__ evec, int n,
                                int ns) {
  const int k = blockIdx.z, s = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double2 v = make_double2(0.0, 0.0);
  if (s < ns) {
    const double2 e = c[((size_t)k * n + i) * n + s];
    v = make_double2(e.x, -e.y);
  }
  evec[(size_t)k * n * n + (size_t)s * n + i] = v;
}

// S pair blocks in the sparse product's grouped order: sq[k][q] = spk[k][gp_pair[q]].
__global__ void k_permute_pairs(PairGraph g, const double2 *__restrict__ spk, double2 *__restrict__ sq) {
  const int e2 = g.norb * g.norb;
  const int k = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.n_pairs * e2) return;
  const int q = t / e2, e = t % e2;
  sq[((size_t)k * g.n_pairs + q) * e2 + e] = spk[((size_t)k * g.n_pairs + g.gp_pair[q]) * e2 + e];
}

int blocks(long long n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

void launch_cn_permute_pairs(const PairGraph &g, const double2 *spk, double2 *sq, int nk, hipStream_t s) {
  const int e2 = g.norb * g.norb;
  hipLaunchKernelGGL(k_permute_pairs, dim3(blocks((long long)g.n_pairs * e2, 256), nk), dim3(256), 0,
                     s, g, spk, sq);
}

void launch_cn_pattern(const PairGraph &g, const double2 *c, const double *occ, int n, int ns, int nk,
                       double2 *d, hipStream_t s) {
  const dim3 grid(blocks(g.n_pairs, 4), nk);
  if (g.norb == 4)
    hipLaunchKernelGGL(k_cn_pattern<4>, grid, dim3(256), 0, s, g, c, occ, n, ns, d);
  else
    hipLaunchKernelGGL(k_cn_pattern<1>, grid, dim3(256), 0, s, g, c, occ, n, ns, d);
}

void launch_cn_vmid(const double *v, double *vprev, double *vmid, int na, bool first, hipStream_t s) {
  hipLaunchKernelGGL(k_cn_vmid, dim3(blocks(na, 256)), dim3(256), 0, s, v, vprev, vmid, na,
                     first ? 1 : 0);
}

void launch_cn_build(const PairGraph &g, const double2 *w, const double2 *hq, const double2 *spk,
                     double tau, int n, int ns, int nk, double2 *aug, hipStream_t s) {
  const int ld = 2 * n;
  hipLaunchKernelGGL(k_cn_fill, dim3(blocks(n + ns, 256), n, nk), dim3(256), 0, s, aug, ld, w, n, ns);
  const int e2 = g.norb * g.norb;
  const dim3 grid(blocks((long long)g.n_pairs * e2, 256), nk);
  if (g.norb == 4)
    hipLaunchKernelGGL(k_cn_scatter<4>, grid, dim3(256), 0, s, g, aug, ld, n, hq, spk, tau);
  else
    hipLaunchKernelGGL(k_cn_scatter<1>, grid, dim3(256), 0, s, g, aug, ld, n, hq, spk, tau);
}

namespace {

// Rows split of a solve of m rows: the first part a whole number of blocks,
// at least half of them.
int cn_split(int m) {
  const int nb = (m + kCnBlock - 1) / kCnBlock;
  return kCnBlock * ((nb + 1) / 2);
}

// A^-1 B in place for the m x m diagonal block A at (r0, r0) of every k's
// augmented matrix and B = all columns to its right (width n + ns - r0 - m):
//   m <= kCnBlock: B <- A^-1 B with A^-1 from k_blk_inv;
//   else, A = [A11 A12; A21 A22] split at h:
//     [A12 | B1] <- A11^-1 [A12 | B1]            (recursion)
//     [A22 | B2] -= A21 [A12 | B1]               (Schur complement, K = h)
//     B2 <- A22^-1 B2                            (recursion)
//     B1 -= A12 B2                               (K = m - h)
// Most of the work is in the two products, whose depth K is half the block.
void cn_solve(double2 *aug, double2 *inv, int r0, int m, int n, int ns, int nk, int tile,
              hipStream_t s) {
  const int ld = 2 * n;
  const size_t sa = (size_t)n * ld;
  const int w = n + ns - (r0 + m);
  auto at = [&](int r, int c) { return aug + (size_t)r * ld + c; };
  if (m <= kCnBlock) {
    hipLaunchKernelGGL(k_blk_inv, dim3(nk), dim3(kInvThreads), 0, s, aug, ld, sa, r0, m, inv);
    // In place: the product's tile holds all m rows of each column it owns.
    gemm_strided(inv, kCnBlock, (size_t)kCnBlock * kCnBlock, at(r0, r0 + m), ld, sa, at(r0, r0 + m),
                 ld, sa, m, w, m, 1.0, false, nk, s, tile, true);
    return;
  }
  const int h = cn_split(m);
  cn_solve(aug, inv, r0, h, n, ns, nk, tile, s);
  gemm_strided(at(r0 + h, r0), ld, sa, at(r0, r0 + h), ld, sa, at(r0 + h, r0 + h), ld, sa, m - h,
               (m - h) + w, h, -1.0, true, nk, s, tile);
  cn_solve(aug, inv, r0 + h, m - h, n, ns, nk, tile, s);
  gemm_strided(at(r0, r0 + h), ld, sa, at(r0 + h, r0 + m), ld, sa, at(r0, r0 + m), ld, sa, h, w,
               m - h, -1.0, true, nk, s, tile);
}

}  // namespace

void launch_cn_solve(double2 *aug, double2 *inv, int n, int ns, int nk, int tile, hipStream_t s) {
  cn_solve(aug, inv, 0, n, n, ns, nk, (tile >= 1 && tile <= 3) ? tile : 2, s);
}

void launch_cn_update(const double2 *aug, double2 *c, int n, int ns, int nk, int64_t *ctr,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_cn_update, dim3(blocks(ns, 256), n, nk), dim3(256), 0, s, aug, 2 * n, c, n, ns,
                     ctr);
}

void launch_cn_from_vectors(const double2 *evec, double2 *c, int n, int ns, int nk, hipStream_t s) {
  hipLaunchKernelGGL(k_cn_from_vectors, dim3(blocks(n, 256), n, nk), dim3(256), 0, s, evec, c, n, ns);
}

void launch_cn_to_vectors(const double2 *c, double2 *evec, int n, int ns, int nk, hipStream_t s) {
  hipLaunchKernelGGL(k_cn_to_vectors, dim3(blocks(n, 256), n, nk), dim3(256), 0, s, c, evec, n, ns);
}

void launch_zgemm_strided(const double2 *a, int lda, size_t sa, const double2 *b, int ldb, size_t sb,
                          double2 *c, int ldc, size_t sc, int m, int n, int k, double alpha,
                          bool beta_one, int batch, hipStream_t s) {
  gemm_strided(a, lda, sa, b, ldb, sb, c, ldc, sc, m, n, k, alpha, beta_one, batch, s, 2);
}

}  // namespace vgtb
