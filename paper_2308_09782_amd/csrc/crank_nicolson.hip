// Crank-Nicolson propagation of the coefficient vectors (Eq. 5), the unitary
// scheme the paper names beside the density leapfrog:
//
//   (S_k + i tau H_k) C(t + dt) = (S_k - i tau H_k) C(t),   tau = dt / 2,
//
// solved as X = (S + i tau H)^-1 S C and C(t + dt) = 2 X - C(t).  The matrix
// A = S + i tau H has the positive-definite Hermitian part S, so Gaussian
// elimination needs no pivoting (every leading block is invertible).  It is
// done by blocks of kCnBlock rows on the augmented matrix [A | S C]:
//   for each diagonal block j:  Z_j = A_jj^-1 [A_j,>j | R_j]   (in place)
//                               [A_>j,>j | R_>j] -= A_>j,j Z_j
//   then, right-looking back substitution over the R columns:
//                               R_<j -= Z_<j,j X_j
// after which the R columns hold X.  The diagonal blocks are inverted in LDS
// (Gauss-Jordan, one workgroup per k-point); every other flop is a strided
// complex FP64 GEMM on the matrix cores.
//
// Observables need D = sum_n f_n C_n C_n^dag (the definition after Eq. 6) only
// on the pair pattern; k_cn_pattern samples it there, and the density-form
// kernels then form charges, current and energy from it unchanged.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "vgtb_internal.h"

namespace vgtb {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

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

constexpr int kGemmBM = 64, kGemmBN = 64;

void gemm_strided(const double2 *a, int lda, size_t sa, const double2 *b, int ldb, size_t sb,
                  double2 *c, int ldc, size_t sc, int m, int n, int k, double alpha, bool beta_one,
                  int batch, hipStream_t s) {
  if (m <= 0 || n <= 0 || k <= 0) return;
  const int tm = (m + kGemmBM - 1) / kGemmBM, tn = (n + kGemmBN - 1) / kGemmBN;
  hipLaunchKernelGGL((k_zgemm_strided<kGemmBM, kGemmBN, 16, 2, 2>), dim3(tm * tn, batch), dim3(256),
                     0, s, a, lda, sa, b, ldb, sb, c, ldc, sc, m, n, k, alpha, beta_one ? 1 : 0, tm, tn);
}

// Inverse of the nb x nb diagonal block at (j0, j0) of each k's augmented
// matrix, by Gauss-Jordan elimination without pivoting in LDS; written to
// inv[k] (kCnBlock x kCnBlock, identity outside nb x nb).
__global__ __launch_bounds__(256) void k_blk_inv(const double2 *__restrict__ aug, int ld, size_t sa,
                                                 int j0, int nb, double2 *__restrict__ inv) {
  constexpr int B = kCnBlock;
  constexpr int PER = B * B / 256;
  __shared__ double2 a[B][B + 1];
  const int k = blockIdx.x, tid = threadIdx.x;
  const double2 *src = aug + (size_t)k * sa + (size_t)j0 * ld + j0;
  for (int e = tid; e < B * B; e += 256) {
    const int i = e / B, j = e % B;
    a[i][j] = (i < nb && j < nb) ? src[(size_t)i * ld + j] : make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int p = 0; p < nb; ++p) {
    const double2 d = a[p][p];
    const double den = d.x * d.x + d.y * d.y;
    const double2 piv = make_double2(d.x / den, -d.y / den);
    double2 nv[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + 256 * r;
      const int i = e / B, j = e % B;
      const double2 aij = a[i][j], aip = a[i][p], apj = a[p][j];
      if (i == p && j == p) {
        nv[r] = piv;
      } else if (i == p) {
        nv[r] = cmul(apj, piv);
      } else if (j == p) {
        const double2 t = cmul(aip, piv);
        nv[r] = make_double2(-t.x, -t.y);
      } else {
        const double2 t = cmul(aip, cmul(apj, piv));
        nv[r] = make_double2(aij.x - t.x, aij.y - t.y);
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = tid + 256 * r;
      a[e / B][e % B] = nv[r];
    }
    __syncthreads();
  }
  double2 *dst = inv + (size_t)k * B * B;
  for (int e = tid; e < B * B; e += 256) dst[e] = a[e / B][e % B];
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

// D on the pair pattern: D[I mu][J nu] = sum_s f_s C[I mu][s] conj(C[J nu][s]),
// one workgroup per (pair, k), the state sum split over its threads.
template <int NO>
__global__ __launch_bounds__(256) void k_cn_pattern(PairGraph g, const double2 *__restrict__ c,
                                                    const double *__restrict__ occ, int n, int ns,
                                                    double2 *__restrict__ d) {
  constexpr int E2 = NO * NO;
  __shared__ double red[4][2 * E2];
  const int p = blockIdx.x, k = blockIdx.y, tid = threadIdx.x;
  const int I = g.pair_row[p], J = g.pair_col[p];
  const double2 *ck = c + (size_t)k * n * n;
  const double *fk = occ + (size_t)k * n;
  double2 acc[E2];
#pragma unroll
  for (int e = 0; e < E2; ++e) acc[e] = make_double2(0.0, 0.0);
  for (int s = tid; s < ns; s += 256) {
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
        acc[mu * NO + nu].x += ci[mu].x * cj[nu].x + ci[mu].y * cj[nu].y;
        acc[mu * NO + nu].y += ci[mu].y * cj[nu].x - ci[mu].x * cj[nu].y;
      }
  }
  const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int e = 0; e < E2; ++e) {
    const double xr = wave_reduce(acc[e].x), xi = wave_reduce(acc[e].y);
    if (lane == 0) {
      red[wave][2 * e] = xr;
      red[wave][2 * e + 1] = xi;
    }
  }
  __syncthreads();
  if (tid < E2) {
    const int e = tid;
    const double xr = (red[0][2 * e] + red[1][2 * e]) + (red[2][2 * e] + red[3][2 * e]);
    const double xi = (red[0][2 * e + 1] + red[1][2 * e + 1]) + (red[2][2 * e + 1] + red[3][2 * e + 1]);
    d[(size_t)k * n * n + (size_t)(I * NO + e / NO) * n + (J * NO + e % NO)] = make_double2(xr, xi);
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
  if (g.norb == 4)
    hipLaunchKernelGGL(k_cn_pattern<4>, dim3(g.n_pairs, nk), dim3(256), 0, s, g, c, occ, n, ns, d);
  else
    hipLaunchKernelGGL(k_cn_pattern<1>, dim3(g.n_pairs, nk), dim3(256), 0, s, g, c, occ, n, ns, d);
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

void launch_cn_eliminate(double2 *aug, double2 *inv, int n, int ns, int nk, hipStream_t s) {
  const int ld = 2 * n;
  const size_t sa = (size_t)n * ld;
  const size_t si = (size_t)kCnBlock * kCnBlock;
  for (int j0 = 0; j0 < n; j0 += kCnBlock) {
    const int nb = std::min(kCnBlock, n - j0);
    hipLaunchKernelGGL(k_blk_inv, dim3(nk), dim3(256), 0, s, aug, ld, sa, j0, nb, inv);
    // Z = A_jj^-1 [A_j,>j | R_j], in place (M = nb <= the tile's 64 rows).
    double2 *row = aug + (size_t)j0 * ld + (j0 + nb);
    gemm_strided(inv, kCnBlock, si, row, ld, sa, row, ld, sa, nb, (n - j0 - nb) + ns, nb, 1.0, false,
                 nk, s);
    const int m = n - j0 - nb;
    if (m > 0)
      gemm_strided(aug + (size_t)(j0 + nb) * ld + j0, ld, sa, row, ld, sa,
                   aug + (size_t)(j0 + nb) * ld + (j0 + nb), ld, sa, m, m + ns, nb, -1.0, true, nk, s);
  }
}

void launch_cn_back(double2 *aug, int n, int ns, int nk, hipStream_t s) {
  const int ld = 2 * n;
  const size_t sa = (size_t)n * ld;
  const int last = ((n - 1) / kCnBlock) * kCnBlock;
  for (int j0 = last; j0 > 0; j0 -= kCnBlock) {
    const int nb = std::min(kCnBlock, n - j0);
    gemm_strided(aug + j0, ld, sa, aug + (size_t)j0 * ld + n, ld, sa, aug + n, ld, sa, j0, ns, nb,
                 -1.0, true, nk, s);
  }
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
  gemm_strided(a, lda, sa, b, ldb, sb, c, ldc, sc, m, n, k, alpha, beta_one, batch, s);
}

}  // namespace vgtb
