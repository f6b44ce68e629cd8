// HIP kernels (gfx950) for everything except the dense matrix-core product:
// Bloch sums over the pair graph, fused Peierls assembly + block-sparse
// product W = H_k D_k, Mulliken / energy / current sweeps, the single-block
// reduction with the SCC shift, and the leapfrog update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>

#include "vgtb_internal.h"

namespace vgtb {
namespace {

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void k_fill_zero(double2 *p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = make_double2(0.0, 0.0);
}

// S_k restricted to the pair graph: spk[k][p][e] = sum_images exp(i k.d) S(e)  (Eq. 7).
__global__ void k_pair_bloch_s(PairGraph g, const double *kpts, double2 *spk) {
  const int e2 = g.norb * g.norb;
  const int k = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.n_pairs * e2) return;
  const int p = t / e2, e = t % e2;
  const double kx = kpts[3 * k], ky = kpts[3 * k + 1], kz = kpts[3 * k + 2];
  double2 acc = make_double2(0.0, 0.0);
  for (int m = g.img_ptr[p]; m < g.img_ptr[p + 1]; ++m) {
    const double th = kx * g.img_d[3 * m] + ky * g.img_d[3 * m + 1] + kz * g.img_d[3 * m + 2];
    double sn, cs;
    sincos(th, &sn, &cs);
    const double s = g.img_s[(size_t)m * e2 + e];
    acc.x += cs * s;
    acc.y += sn * s;
  }
  spk[((size_t)k * g.n_pairs + p) * e2 + e] = acc;
}

// Momentum coupling: the k-dependent, time-independent pair blocks
// h0k[k][p][e] = sum_images exp(i k.d) H0 and ppk[k][p][a][e] = sum_images
// exp(i k.d) i dS/dd^a (Eq. 12: <phi_mu|p|phi_nu> = i dS/dR_J).
__global__ void k_pair_bloch_momentum(PairGraph g, const double *kpts, double2 *h0k, double2 *ppk) {
  const int e2 = g.norb * g.norb;
  const int k = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.n_pairs * e2) return;
  const int p = t / e2, e = t % e2;
  const double kx = kpts[3 * k], ky = kpts[3 * k + 1], kz = kpts[3 * k + 2];
  double2 h = make_double2(0.0, 0.0), pa[3] = {h, h, h};
  for (int m = g.img_ptr[p]; m < g.img_ptr[p + 1]; ++m) {
    const double th = kx * g.img_d[3 * m] + ky * g.img_d[3 * m + 1] + kz * g.img_d[3 * m + 2];
    double sn, cs;
    sincos(th, &sn, &cs);
    const double hv = g.img_h0[(size_t)m * e2 + e];
    h.x += cs * hv;
    h.y += sn * hv;
    for (int a = 0; a < 3; ++a) {
      const double gv = g.img_ds[((size_t)m * 3 + a) * e2 + e];
      pa[a].x -= sn * gv;      // i exp(i th) = -sin th + i cos th
      pa[a].y += cs * gv;
    }
  }
  const size_t pe = (size_t)k * g.n_pairs + p;
  h0k[pe * e2 + e] = h;
  for (int a = 0; a < 3; ++a) ppk[(pe * 3 + a) * e2 + e] = pa[a];
}

// Scatter pair values into a dense N x N matrix per k.  which = 0: S_k from
// spk; which = 1: H0_k at A = 0 (Eq. 8), Bloch-summed here.
__global__ void k_scatter_pairs(PairGraph g, const double *kpts, const double2 *spk, int which,
                                double2 *dense, int n) {
  const int e2 = g.norb * g.norb;
  const int k = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.n_pairs * e2) return;
  const int p = t / e2, e = t % e2;
  // row atom of pair p: binary search in row_ptr
  int lo = 0, hi = g.n_atoms - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g.row_ptr[mid] <= p) lo = mid; else hi = mid - 1;
  }
  const int I = lo, J = g.pair_col[p];
  const int mu = e / g.norb, nu = e % g.norb;
  double2 val;
  if (which == 0) {
    val = spk[((size_t)k * g.n_pairs + p) * e2 + e];
  } else {
    const double kx = kpts[3 * k], ky = kpts[3 * k + 1], kz = kpts[3 * k + 2];
    val = make_double2(0.0, 0.0);
    for (int m = g.img_ptr[p]; m < g.img_ptr[p + 1]; ++m) {
      const double th = kx * g.img_d[3 * m] + ky * g.img_d[3 * m + 1] + kz * g.img_d[3 * m + 2];
      double sn, cs;
      sincos(th, &sn, &cs);
      const double h = g.img_h0[(size_t)m * e2 + e];
      val.x += cs * h;
      val.y += sn * h;
    }
  }
  dense[(size_t)k * n * n + (size_t)(I * g.norb + mu) * n + (J * g.norb + nu)] = val;
}

// A(t_n)/c of the step the device counter names, from the ring of kStepRing
// slots (slot = step mod kStepRing); a null ring means A = 0.
__device__ inline StepField step_field(StepSource src) {
  if (src.ring == nullptr) return StepField{0.0, 0.0, 0.0};
  const int64_t st = src.ctr ? *src.ctr : 0;
  const double *a = src.ring + 3 * (st % kStepRing);
  return StepField{a[0], a[1], a[2]};
}

__global__ void k_store_ring(FieldChunk f, int64_t step0, int ns, double *ring) {
  const int i = threadIdx.x;
  if (i < 3 * ns) ring[3 * ((step0 + i / 3) % kStepRing) + i % 3] = f.a[i];
}

__global__ void k_set_counter(int64_t *ctr, int64_t v) { *ctr = v; }
__global__ void k_advance_counter(int64_t *ctr) { *ctr += 1; }

// One wavefront per (atom I, k): sweep the pair blocks of row I of D_k and
// accumulate  q = Re sum D conj(S)  (Mulliken, row I),  E = Re sum conj(D) H0,
// J^a = Re sum conj(D) Pi^a  with Pi^a = sum_images i d^a exp(i(k+A/c).d) H0.
template <int NO>
__global__ __launch_bounds__(64) void k_observe(PairGraph g, const double2 *__restrict__ d, int n,
                                                const double *kpts, StepSource src,
                                                const double2 *__restrict__ spk,
                                                const double2 *__restrict__ h0k,
                                                const double2 *__restrict__ ppk,
                                                double *__restrict__ part) {
  constexpr int E2 = NO * NO;
  constexpr int P = 64 / E2;
  const int I = blockIdx.x, k = blockIdx.y;
  const int lane = threadIdx.x;
  const int e = lane % E2, slot = lane / E2;
  const int mu = e / NO, nu = e % NO;
  const StepField f = step_field(src);
  const double kx = kpts[3 * k] + f.ax, ky = kpts[3 * k + 1] + f.ay, kz = kpts[3 * k + 2] + f.az;
  const size_t base = (size_t)k * n * n;
  double q = 0.0, en = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  const int p1 = g.row_ptr[I + 1];
  for (int p = g.row_ptr[I] + slot; p < p1; p += P) {
    const int J = g.pair_col[p];
    const size_t idx = base + (size_t)(I * NO + mu) * n + (J * NO + nu);
    const double2 dv = d[idx];
    const double2 s = spk[((size_t)k * g.n_pairs + p) * E2 + e];
    q += dv.x * s.x + dv.y * s.y;
    if (h0k != nullptr) {
      // Momentum coupling: H = H0_k + a.P_k + |a|^2/2 S_k, Pi = P_k + a S_k (a = A/c);
      // Re Tr(D X) over the pair block is sum Re(D conj(X)) for Hermitian X.
      const size_t pe = (size_t)k * g.n_pairs + p;
      const double2 h0 = h0k[pe * E2 + e];
      const double2 px = ppk[(pe * 3 + 0) * E2 + e], py = ppk[(pe * 3 + 1) * E2 + e],
                    pz = ppk[(pe * 3 + 2) * E2 + e];
      const double a2 = 0.5 * (f.ax * f.ax + f.ay * f.ay + f.az * f.az);
      const double hr = h0.x + f.ax * px.x + f.ay * py.x + f.az * pz.x + a2 * s.x;
      const double hi = h0.y + f.ax * px.y + f.ay * py.y + f.az * pz.y + a2 * s.y;
      en += dv.x * hr + dv.y * hi;
      jx += dv.x * (px.x + f.ax * s.x) + dv.y * (px.y + f.ax * s.y);
      jy += dv.x * (py.x + f.ay * s.x) + dv.y * (py.y + f.ay * s.y);
      jz += dv.x * (pz.x + f.az * s.x) + dv.y * (pz.y + f.az * s.y);
      continue;
    }
    for (int m = g.img_ptr[p]; m < g.img_ptr[p + 1]; ++m) {
      const double dx = g.img_d[3 * m], dy = g.img_d[3 * m + 1], dz = g.img_d[3 * m + 2];
      double sn, cs;
      sincos(kx * dx + ky * dy + kz * dz, &sn, &cs);
      const double h = g.img_h0[(size_t)m * E2 + e];
      const double re = (dv.x * cs + dv.y * sn) * h;   // Re(conj(D) e^{i th} h)
      const double im = (dv.x * sn - dv.y * cs) * h;   // Im(conj(D) e^{i th} h)
      en += re;
      jx -= dx * im;
      jy -= dy * im;
      jz -= dz * im;
    }
  }
  q = wave_sum(q);
  en = wave_sum(en);
  jx = wave_sum(jx);
  jy = wave_sum(jy);
  jz = wave_sum(jz);
  if (lane == 0) {
    double *o = part + ((size_t)k * g.n_atoms + I) * 5;
    o[0] = q;
    o[1] = en;
    o[2] = jx;
    o[3] = jy;
    o[4] = jz;
  }
}

// Reduction of the per-(k, atom) partials, in three short kernels with a
// fixed summation order (repeated runs agree bit for bit):
//  1. per atom I: q_I = sum_k w_k q(k,I) (Mulliken), and the atom's shares
//     of the band energy and the current, each summed over k with the
//     weights w_k (Eq. 14's 1/N_k is the equal-weight mesh);
//  2. SCC only, one wavefront per row: V_I = sum_K gamma_IK (q_K - Z_K)
//     (Eq. 10) and the atom's share 1/2 dq_I V_I of the SCC energy;
//  3. one workgroup: sums over atoms into the history row
//     [Jx Jy Jz E Tr q_0 .. q_{na-1}] (current of Eq. 14, Tr = sum_I q_I).
__global__ __launch_bounds__(256) void k_reduce_atoms(const double *__restrict__ part, int nk,
                                                      int na, const double *__restrict__ kw,
                                                      double *__restrict__ qbuf,
                                                      double *__restrict__ rowpart,
                                                      double *__restrict__ hist, int cap,
                                                      const int64_t *ctr) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= na) return;
  double *hist_row = hist + (size_t)(ctr ? *ctr % cap : 0) * (5 + na);
  double q = 0.0, en = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  for (int k = 0; k < nk; ++k) {
    const double *o = part + ((size_t)k * na + I) * 5;
    q += kw[k] * o[0];
    en += kw[k] * o[1];
    jx += kw[k] * o[2];
    jy += kw[k] * o[3];
    jz += kw[k] * o[4];
  }
  qbuf[I] = q;
  hist_row[5 + I] = q;
  double *r = rowpart + (size_t)I * 5;
  r[0] = en;
  r[1] = jx;
  r[2] = jy;
  r[3] = jz;
  r[4] = 0.0;
}

__global__ __launch_bounds__(1024) void k_reduce_scc(int na, const double *__restrict__ gamma,
                                                     const double *__restrict__ z,
                                                     const double *__restrict__ qbuf,
                                                     double *__restrict__ v,
                                                     double *__restrict__ rowpart) {
  const int lane = threadIdx.x & 63;
  const int I = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (I >= na) return;
  const double *gr = gamma + (size_t)I * na;
  double acc = 0.0;
  for (int K = lane; K < na; K += 64) acc += gr[K] * (qbuf[K] - z[K]);
  acc = wave_sum(acc);
  if (lane == 0) {
    v[I] = acc;
    rowpart[(size_t)I * 5 + 4] = 0.5 * (qbuf[I] - z[I]) * acc;
  }
}

constexpr int kReduceThreads = 1024;
constexpr int kReduceWaves = kReduceThreads / 64;

__global__ __launch_bounds__(kReduceThreads) void k_reduce_final(int na, double jscale,
                                                                 const double *__restrict__ qbuf,
                                                                 const double *__restrict__ rowpart,
                                                                 double *__restrict__ hist, int cap,
                                                                 const int64_t *ctr, int *flag) {
  __shared__ double red[6][kReduceWaves];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double *hist_row = hist + (size_t)(ctr ? *ctr % cap : 0) * (5 + na);
  double c[6] = {0, 0, 0, 0, 0, 0};
  for (int I = t; I < na; I += kReduceThreads) {
    const double *r = rowpart + (size_t)I * 5;
    c[0] += r[0];
    c[1] += r[1];
    c[2] += r[2];
    c[3] += r[3];
    c[4] += r[4];
    c[5] += qbuf[I];
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    c[i] = wave_sum(c[i]);
    if (lane == 0) red[i][wave] = c[i];
  }
  __syncthreads();
  if (t == 0) {
    double o[6] = {0, 0, 0, 0, 0, 0};
    for (int w = 0; w < kReduceWaves; ++w)
      for (int i = 0; i < 6; ++i) o[i] += red[i][w];
    hist_row[0] = o[1] * jscale;
    hist_row[1] = o[2] * jscale;
    hist_row[2] = o[3] * jscale;
    hist_row[3] = o[0] + o[4];
    hist_row[4] = o[5];
    if (!isfinite(o[5]) || !isfinite(o[0])) *flag = 1;
  }
}

// Round-to-nearest-even float -> bf16 bits, and back.
__device__ inline uint16_t to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
// x = hi + lo with hi = bf16(x), lo = bf16(x - hi).
__device__ inline void split_bf16(double x, uint16_t &hi, uint16_t &lo) {
  const float xf = (float)x;
  hi = to_bf16(xf);
  lo = to_bf16(xf - from_bf16(hi));
}
// The lo part of the bf16 split of S^-1 - I in copy `level` of the dithered
// representation (see kADither): r the remainder after hi.
__device__ inline uint16_t dithered_bf16(float r, int level) {
  if (r == 0.0f) return to_bf16(r);
  const double ar = fabs((double)r);
  const double d = dither_offset(level);
  int e;
  frexp(ar, &e);   // ar = m 2^e, m in [0.5, 1): the bf16 grid step there is 2^(e - 8)
  const float t = d == 0.0 ? (float)ar : (float)(ar + d * ldexp(1.0, e - 8));
  const uint16_t m = to_bf16(t);
  return r < 0.0f ? (uint16_t)(m ^ 0x8000u) : m;
}
// x sc = hi + lo with hi = f16(x sc), lo = f16(x sc - hi); sc a power of two
// chosen so that the largest |x sc| of the matrix lies in [2^13, 2^14).
__device__ inline void split_f16(double x, float sc, uint16_t &hi, uint16_t &lo) {
  const float xs = (float)x * sc;
  hi = __builtin_bit_cast(uint16_t, (_Float16)xs);
  lo = __builtin_bit_cast(uint16_t, (_Float16)(xs - (float)__builtin_bit_cast(_Float16, hi)));
}
// Largest |re|, |im| the lanes of a wave have written, into *dst as float bits
// (non-negative floats order like their bit patterns).  NaNs are skipped.
__device__ inline void wave_max_to(float m, unsigned *dst) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(dst, __float_as_uint(m));
}

// Block-sparse product W = H_k D_k (Eqs. 8-10) over the pair blocks
//   H_k(I,J) = sum_images exp(i(k+A/c).d) H0 + 1/2 (V_I + V_J) S_k(I,J)
// that k_assemble writes in grouped order.
//
// A workgroup owns the rows of KG consecutive atoms and one chunk of
// columns (one column per thread).  It walks the union of those atoms'
// neighbours once: each neighbour's D rows are loaded a single time and
// applied to every group atom that pairs with it (mask bits, uniform
// branches, accumulators indexed at compile time).  Pair blocks of H are
// built in LDS kEntChunk neighbours at a time.
//
// OUT selects the operand format of the dense product that consumes W:
//   0: complex128 row-major; 1: complex64 row-major;
//   2: four bf16 planes (re_hi, re_lo, im_hi, im_lo), k-packed with padded
//      size np: W[r][c] at ((r/8)*np + c)*8 + r%8 of each plane; plus a
//      complex64 copy (w32) for the identity part of S^-1 W.
//   3: as 2 with fp16 planes of W wscale[k]; the largest |re|, |im| of each
//      k-point also goes to its slots of wmax (the caller checks that wscale[k]
//      is the scale this maximum calls for and splits the k-point again if not).
constexpr int kEntChunk = 8;

template <int NO, int OUT>
__device__ inline void store_rows(const double2 (&acc)[NO], int r0, int col, int k, int n, int np,
                                  int nk, void *wout, float2 *w32, float sc, float &m) {
  const size_t base = (size_t)k * n * n;
  if (OUT == 0) {
    double2 *w = static_cast<double2 *>(wout);
#pragma unroll
    for (int mu = 0; mu < NO; ++mu) w[base + (size_t)(r0 + mu) * n + col] = acc[mu];
  } else if (OUT == 1) {
    float2 *w = static_cast<float2 *>(wout);
#pragma unroll
    for (int mu = 0; mu < NO; ++mu)
      w[base + (size_t)(r0 + mu) * n + col] = make_float2((float)acc[mu].x, (float)acc[mu].y);
  } else {
#pragma unroll
    for (int mu = 0; mu < NO; ++mu)
      w32[base + (size_t)(r0 + mu) * n + col] = make_float2((float)acc[mu].x, (float)acc[mu].y);
    uint16_t *w = static_cast<uint16_t *>(wout);
    const size_t plane = (size_t)nk * np * np;
    uint16_t h[4][NO];
#pragma unroll
    for (int mu = 0; mu < NO; ++mu) {
      if (OUT == 2) {
        split_bf16(acc[mu].x, h[0][mu], h[1][mu]);
        split_bf16(acc[mu].y, h[2][mu], h[3][mu]);
      } else {
        split_f16(acc[mu].x, sc, h[0][mu], h[1][mu]);
        split_f16(acc[mu].y, sc, h[2][mu], h[3][mu]);
        m = fmaxf(m, fmaxf(fabsf((float)acc[mu].x), fabsf((float)acc[mu].y)));
      }
    }
    const size_t off = (size_t)k * np * np + ((size_t)(r0 >> 3) * np + col) * 8 + (r0 & 7);
    if (NO == 4) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        uint2 pk = make_uint2((uint32_t)h[p][0] | ((uint32_t)h[p][NO > 1 ? 1 : 0] << 16),
                              (uint32_t)h[p][NO > 2 ? 2 : 0] | ((uint32_t)h[p][NO > 3 ? 3 : 0] << 16));
        *reinterpret_cast<uint2 *>(w + p * plane + off) = pk;
      }
    } else {
#pragma unroll
      for (int p = 0; p < 4; ++p) w[p * plane + off] = h[p][0];
    }
  }
}

// Peierls assembly of the pair blocks of H_k(t) in the grouped pair order q
// of the sparse product: hq[k][q][e].
template <int NO>
__global__ __launch_bounds__(256) void k_assemble(PairGraph g, const double *kpts, StepSource src,
                                                  const double2 *__restrict__ spk,
                                                  const double *__restrict__ v,
                                                  double2 *__restrict__ hq,
                                                  const double2 *__restrict__ h0k,
                                                  const double2 *__restrict__ ppk) {
  constexpr int E2 = NO * NO;
  const int k = blockIdx.y;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.n_pairs * E2) return;
  const int q = t / E2, e = t % E2;
  const int p = g.gp_pair[q];
  const StepField f = step_field(src);
  const double k0x = kpts[3 * k], k0y = kpts[3 * k + 1], k0z = kpts[3 * k + 2];
  double2 h = make_double2(0.0, 0.0);
  if (h0k != nullptr) {
    // Momentum coupling (Eq. 12): H0_k + a.P_k + |a|^2/2 S_k with a = A/c.
    const size_t pe = (size_t)k * g.n_pairs + p;
    const double2 h0 = h0k[pe * E2 + e], sv = spk[pe * E2 + e];
    const double2 px = ppk[(pe * 3 + 0) * E2 + e], py = ppk[(pe * 3 + 1) * E2 + e],
                  pz = ppk[(pe * 3 + 2) * E2 + e];
    const double a2 = 0.5 * (f.ax * f.ax + f.ay * f.ay + f.az * f.az);
    h.x = h0.x + f.ax * px.x + f.ay * py.x + f.az * pz.x + a2 * sv.x;
    h.y = h0.y + f.ax * px.y + f.ay * py.y + f.az * pz.y + a2 * sv.y;
  } else
  for (int m = g.img_ptr[p]; m < g.img_ptr[p + 1]; ++m) {
    const double dx = g.img_d[3 * m], dy = g.img_d[3 * m + 1], dz = g.img_d[3 * m + 2];
    const double hv = g.img_h0[(size_t)m * E2 + e];
    double sn, cs;
    sincos((k0x + f.ax) * dx + (k0y + f.ay) * dy + (k0z + f.az) * dz, &sn, &cs);
    h.x += cs * hv;
    h.y += sn * hv;
  }
  if (v != nullptr) {
    const double vs = 0.5 * (v[g.pair_row[p]] + v[g.pair_col[p]]);
    const double2 sv = spk[((size_t)k * g.n_pairs + p) * E2 + e];
    h.x += vs * sv.x;
    h.y += vs * sv.y;
  }
  hq[((size_t)k * g.n_pairs + q) * E2 + e] = h;
}

// DELTA: W = H_k D - C0 with the constant C0 = H0_k(A=0) D0 of a reference
// density D0, i.e. H (D - D0) + (H - H0) D0 in one product; FP64 keeps the
// cancellation harmless.
// KG atoms per row group; CPT columns per thread (stride blockDim), which
// reuses each H value read from LDS CPT times.
template <int NO, bool DELTA, int OUT, int KG, int CPT>
__global__ __launch_bounds__(256) void k_spmm(PairGraph g, const double2 *__restrict__ d, int n,
                                              const double2 *__restrict__ hq,
                                              const double2 *__restrict__ c0,
                                              void *__restrict__ wout, int np, int nk,
                                              float2 *__restrict__ w32,
                                              const float *__restrict__ wscale,
                                              unsigned *__restrict__ wmax) {
  constexpr int E2 = NO * NO;
  constexpr int CP = kEntChunk * KG;           // pair blocks per chunk, at most
  __shared__ double2 hs[CP * E2];
  __shared__ int s_j[kEntChunk], s_mask[kEntChunk], s_pp[kEntChunk];
  const int grp = blockIdx.y, k = blockIdx.z;
  const int I0 = grp * KG;
  const int tid = threadIdx.x;
  int col[CPT], cl[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    col[c] = blockIdx.x * blockDim.x * CPT + c * blockDim.x + tid;
    cl[c] = col[c] < n ? col[c] : n - 1;       // clamped column for loads
  }
  const size_t base = (size_t)k * n * n;
  double2 acc[KG][NO][CPT];
#pragma unroll
  for (int il = 0; il < KG; ++il)
#pragma unroll
    for (int mu = 0; mu < NO; ++mu)
#pragma unroll
      for (int c = 0; c < CPT; ++c) acc[il][mu][c] = make_double2(0.0, 0.0);
  const int e0 = g.grp_ptr[grp], e1 = g.grp_ptr[grp + 1];
  for (int ec = e0; ec < e1; ec += kEntChunk) {
    const int ne = min(kEntChunk, e1 - ec);
    const int q0 = g.ent_pp[ec];
    const int nq = g.ent_pp[ec + ne] - q0;     // <= ne * KG
    const size_t hoff = ((size_t)k * g.n_pairs + q0) * E2;
    for (int t = tid; t < nq * E2; t += blockDim.x) hs[t] = hq[hoff + t];
    if (tid < ne) {
      s_j[tid] = g.ent_j[ec + tid];
      s_mask[tid] = g.ent_mask[ec + tid];
      s_pp[tid] = g.ent_pp[ec + tid] - q0;
    }
    __syncthreads();
    // Software pipeline: the D rows of neighbour el+1 load while el is applied.
    double2 dv[NO][CPT], dn[NO][CPT];
    {
      const int J = s_j[0];
#pragma unroll
      for (int nu = 0; nu < NO; ++nu)
#pragma unroll
        for (int c = 0; c < CPT; ++c) dn[nu][c] = d[base + (size_t)(J * NO + nu) * n + cl[c]];
    }
    for (int el = 0; el < ne; ++el) {
#pragma unroll
      for (int nu = 0; nu < NO; ++nu)
#pragma unroll
        for (int c = 0; c < CPT; ++c) dv[nu][c] = dn[nu][c];
      if (el + 1 < ne) {
        const int J = s_j[el + 1];
#pragma unroll
        for (int nu = 0; nu < NO; ++nu)
#pragma unroll
          for (int c = 0; c < CPT; ++c) dn[nu][c] = d[base + (size_t)(J * NO + nu) * n + cl[c]];
      }
      const int mask = s_mask[el];
      int slot = s_pp[el];
#pragma unroll
      for (int il = 0; il < KG; ++il) {
        if (mask & (1 << il)) {
          const double2 *h = hs + slot * E2;
#pragma unroll
          for (int mu = 0; mu < NO; ++mu)
#pragma unroll
            for (int nu = 0; nu < NO; ++nu) {
              const double2 hv = h[mu * NO + nu];
#pragma unroll
              for (int c = 0; c < CPT; ++c) {
                acc[il][mu][c].x = fma(hv.x, dv[nu][c].x, acc[il][mu][c].x);
                acc[il][mu][c].x = fma(-hv.y, dv[nu][c].y, acc[il][mu][c].x);
                acc[il][mu][c].y = fma(hv.x, dv[nu][c].y, acc[il][mu][c].y);
                acc[il][mu][c].y = fma(hv.y, dv[nu][c].x, acc[il][mu][c].y);
              }
            }
          ++slot;
        }
      }
    }
    __syncthreads();
  }
  const float sc = OUT == 3 ? wscale[k] : 1.0f;
  float wm = 0.0f;
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    if (col[c] >= n) continue;
#pragma unroll
    for (int il = 0; il < KG; ++il) {
      if (I0 + il < g.n_atoms) {
        double2 out[NO];
#pragma unroll
        for (int mu = 0; mu < NO; ++mu) {
          out[mu] = acc[il][mu][c];
          if (DELTA) {
            const double2 cv = c0[base + (size_t)((I0 + il) * NO + mu) * n + col[c]];
            out[mu].x -= cv.x;
            out[mu].y -= cv.y;
          }
        }
        store_rows<NO, OUT>(out, (I0 + il) * NO, col[c], k, n, np, nk, wout, w32, sc, wm);
      }
    }
  }
  if (OUT == 3) {
    const int slot = ((blockIdx.y * gridDim.x + blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)) % kMaxSlots;
    wave_max_to(wm, wmax + ((size_t)k * kMaxSlots + slot) * kMaxStride);
  }
}

// The same product on the FP64 matrix cores (four orbitals per atom).  One
// v_mfma_f64_4x4x4_4b multiplies a 4x4 pair block by 16 consecutive columns
// of the neighbour's four D rows, the four blocks of the instruction being
// four 4-column slices that share the pair block.  It is issued transposed,
// A = D^T and B = H^T, so that
//   A operand of lane l: D[4J + (l >> 4)][c0 + (l & 15)]   (coalesced rows)
//   B operand of lane l: H[I][l & 3][l >> 4]               (one LDS read)
//   result of lane l:    W[4I + (l & 3)][c0 + 4((l >> 2) & 3) + (l >> 4)]
// with the four rows of an atom in four neighbouring lanes.  A wave owns CB
// such 16-column slices; complex arithmetic is four real products per slice
// (re += Dr Hr - Di Hi, im += Di Hr + Dr Hi) into separate accumulators.
// Compared with the vector form, one LDS read of H now feeds 16 matrix
// instructions instead of four FMAs, and no zero blocks are multiplied.
// G3: the complex product in three real products per slice instead of four,
// P1 = Dr Hr, P2 = Di Hi, P3 = (Dr + Di)(Hr + Hi), with re = P1 - P2 and
// im = P3 - P1 - P2 formed in the epilogue (one accumulator more per slice).
// Lane q of each quad of lanes holds row q of a 4 x 4 matrix M of 16-bit
// values as x0 = M[q][0] | M[q][1] << 16, x1 = M[q][2] | M[q][3] << 16; the
// result is column q, (M[0][q] | M[1][q] << 16, M[2][q] | M[3][q] << 16).
// Two quad permutations (DPP, no LDS traffic): first the 2 x 2 blocks are
// exchanged between lanes q and q ^ 2, then single values between q and q ^ 1.
// Every lane of the quad must be active.
__device__ inline uint2 quad_transpose16(uint32_t x0, uint32_t x1, int q) {
  const bool upper = (q & 2) != 0;
  const uint32_t ra = (uint32_t)__builtin_amdgcn_mov_dpp((int)(upper ? x0 : x1), 0x4E, 0xF, 0xF, false);
  // a: row q & 1 of columns 2 (q >> 1) and 2 (q >> 1) + 1; b: row (q & 1) + 2 of the same.
  const uint32_t a = upper ? ra : x0;
  const uint32_t b = upper ? x1 : ra;
  const bool odd = (q & 1) != 0;
  const uint32_t send = odd ? ((a & 0xFFFFu) | (b << 16)) : ((a >> 16) | (b & 0xFFFF0000u));
  const uint32_t rb = (uint32_t)__builtin_amdgcn_mov_dpp((int)send, 0xB1, 0xF, 0xF, false);
  if (odd) return make_uint2((rb & 0xFFFFu) | (a & 0xFFFF0000u), (rb >> 16) | (b & 0xFFFF0000u));
  return make_uint2((a & 0xFFFFu) | (rb << 16), (b & 0xFFFFu) | (rb & 0xFFFF0000u));
}

__device__ inline double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// The four-slice three-product form of row groups up to 8 atoms is held to
// two wavefronts per SIMD (256 registers): its independent accumulators, not
// occupancy, cover the latencies, and left to itself the compiler moves the
// deviation form's epilogue into one wave per SIMD.
template <bool DELTA, int OUT, int KG, int CB, bool G3>
__global__ __launch_bounds__(256, (G3 && CB == 4 && KG <= 8) ? 2 : 1) void k_spmm_mfma(PairGraph g, const double2 *__restrict__ d,
                                                   int n, const double2 *__restrict__ hq,
                                                   const double2 *__restrict__ c0,
                                                   void *__restrict__ wout, int np, int nk,
                                                   float2 *__restrict__ w32,
                                                   const float *__restrict__ wscale,
                                                   unsigned *__restrict__ wmax) {
  constexpr int E2 = 16;
  constexpr int CP = kEntChunk * KG;
  __shared__ double2 hs[CP * E2];
  __shared__ int s_j[kEntChunk], s_mask[kEntChunk], s_pp[kEntChunk];
  const int grp = blockIdx.y, k = blockIdx.z;
  const int I0 = grp * KG;
  const int tid = threadIdx.x, lane = tid & 63;
  const int cw = (blockIdx.x * (blockDim.x >> 6) + (tid >> 6)) * 16 * CB;   // first column of the wave
  const int nu = lane >> 4;                   // D row (orbital of J) of the A operand
  const int hsel = (lane & 3) * 4 + nu;       // H[mu][nu] of the B operand
  int lcol[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) lcol[cb] = min(cw + cb * 16 + (lane & 15), n - 1);
  const size_t base = (size_t)k * n * n;
  double accr[KG][CB], acci[KG][CB], accs[G3 ? KG : 1][G3 ? CB : 1];
#pragma unroll
  for (int il = 0; il < KG; ++il)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      accr[il][cb] = acci[il][cb] = 0.0;
      if (G3) accs[il][cb] = 0.0;
    }
  // Every atom has at least its on-site block (checked when the graph is
  // built), so a group has at least one entry and the loop runs at least
  // once; saying so keeps the accumulators in place up to the epilogue.
  const int e0 = g.grp_ptr[grp], e1 = max(g.grp_ptr[grp + 1], e0 + 1);
  int ec = e0;
  do {
    const int ne = min(kEntChunk, e1 - ec);
    const int q0 = g.ent_pp[ec];
    const int nq = g.ent_pp[ec + ne] - q0;
    const size_t hoff = ((size_t)k * g.n_pairs + q0) * E2;
    for (int t = tid; t < nq * E2; t += blockDim.x) hs[t] = hq[hoff + t];
    if (tid < ne) {
      s_j[tid] = g.ent_j[ec + tid];
      s_mask[tid] = g.ent_mask[ec + tid];
      s_pp[tid] = g.ent_pp[ec + tid] - q0;
    }
    __syncthreads();
    // The D rows of neighbour el + 1 load while el is applied.
    double2 dv[CB], dn[CB];
    {
      const size_t roff = base + (size_t)(s_j[0] * 4 + nu) * n;
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) dn[cb] = d[roff + lcol[cb]];
    }
    for (int el = 0; el < ne; ++el) {
      double dsum[G3 ? CB : 1];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        dv[cb] = dn[cb];
        if (G3) dsum[cb] = dv[cb].x + dv[cb].y;
      }
      if (el + 1 < ne) {
        const size_t roff = base + (size_t)(s_j[el + 1] * 4 + nu) * n;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) dn[cb] = d[roff + lcol[cb]];
      }
      const int mask = __builtin_amdgcn_readfirstlane(s_mask[el]);
      int slot = __builtin_amdgcn_readfirstlane(s_pp[el]);
#pragma unroll
      for (int il = 0; il < KG; ++il) {
        if (mask & (1 << il)) {
          const double2 h = hs[slot * E2 + hsel];
          if (G3) {
            const double hsum = h.x + h.y;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
              accr[il][cb] = mfma4(dv[cb].x, h.x, accr[il][cb]);
              acci[il][cb] = mfma4(dv[cb].y, h.y, acci[il][cb]);
              accs[il][cb] = mfma4(dsum[cb], hsum, accs[il][cb]);
            }
          } else {
            const double nhi = -h.y;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
              accr[il][cb] = mfma4(dv[cb].x, h.x, accr[il][cb]);
              acci[il][cb] = mfma4(dv[cb].y, h.x, acci[il][cb]);
              accr[il][cb] = mfma4(dv[cb].y, nhi, accr[il][cb]);
              acci[il][cb] = mfma4(dv[cb].x, h.y, acci[il][cb]);
            }
          }
          ++slot;
        }
      }
    }
    __syncthreads();
    ec += kEntChunk;
  } while (ec < e1);
  const int mu = lane & 3;
  const float sc = OUT == 3 ? wscale[k] : 1.0f;
  float wm = 0.0f;
  // C0 of the deviation form is read one column slice ahead of its use, so
  // that the loads of slice cb + 1 are in flight while slice cb is stored.
  auto c0_at = [&](int cb, int il) -> double2 {
    const int col = cw + cb * 16 + 4 * ((lane >> 2) & 3) + (lane >> 4);
    if (col < n && I0 + il < g.n_atoms) return c0[base + (size_t)((I0 + il) * 4 + mu) * n + col];
    return make_double2(0.0, 0.0);
  };
  double2 cpre[DELTA ? KG : 1];
  if (DELTA) {
#pragma unroll
    for (int il = 0; il < KG; ++il) cpre[il] = c0_at(0, il);
  }
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int col = cw + cb * 16 + 4 * ((lane >> 2) & 3) + (lane >> 4);
#pragma unroll
    for (int il = 0; il < KG; ++il) {
      const int r = (I0 + il) * 4 + mu;
      const bool ok = col < n && I0 + il < g.n_atoms;
      double2 out = make_double2(accr[il][cb], acci[il][cb]);
      if (G3) out = make_double2(accr[il][cb] - acci[il][cb], accs[il][cb] - accr[il][cb] - acci[il][cb]);
      if (DELTA) {
        const double2 cv = cpre[il];
        if (cb + 1 < CB) cpre[il] = c0_at(cb + 1, il);
        out.x -= cv.x;
        out.y -= cv.y;
      }
      if (OUT == 0) {
        if (ok) static_cast<double2 *>(wout)[base + (size_t)r * n + col] = out;
      } else if (OUT == 1) {
        if (ok) static_cast<float2 *>(wout)[base + (size_t)r * n + col] = make_float2((float)out.x, (float)out.y);
      } else {
        if (ok) w32[base + (size_t)r * n + col] = make_float2((float)out.x, (float)out.y);
        // 16-bit planes: the four rows of the atom sit in lanes 4m..4m+3, and
        // lane 4m + p writes the four rows of plane p as one 8-byte word.
        uint16_t hv[4];
        if (OUT == 2) {
          split_bf16(out.x, hv[0], hv[1]);
          split_bf16(out.y, hv[2], hv[3]);
        } else {
          split_f16(out.x, sc, hv[0], hv[1]);
          split_f16(out.y, sc, hv[2], hv[3]);
          if (ok) wm = fmaxf(wm, fmaxf(fabsf((float)out.x), fabsf((float)out.y)));
        }
        // Lane mu of the quad holds the four plane values of row mu; after the
        // transpose it holds the four rows of plane mu, one 8-byte word.
        const uint2 pk = quad_transpose16((uint32_t)hv[0] | ((uint32_t)hv[1] << 16),
                                          (uint32_t)hv[2] | ((uint32_t)hv[3] << 16), mu);
        uint16_t *w = static_cast<uint16_t *>(wout);
        const size_t plane = (size_t)nk * np * np;
        const int r0 = r - mu;   // first row of the atom (a multiple of 4)
        const size_t off = (size_t)k * np * np + ((size_t)(r0 >> 3) * np + col) * 8 + (r0 & 7);
        if (ok) *reinterpret_cast<uint2 *>(w + mu * plane + off) = pk;
      }
      // One atom's results at a time: keeps the accumulators from being
      // moved out of the matrix registers all at once.
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  if (OUT == 3) {
    const int slot = ((blockIdx.y * gridDim.x + blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)) % kMaxSlots;
    wave_max_to(wm, wmax + ((size_t)k * kMaxSlots + slot) * kMaxStride);
  }
}

// ---- Small systems: a block of steps in one launch ---------------------------
// Without the SCC shift the k-points do not interact within a step, so for
// N <= kSmallN one workgroup per k keeps S_k^-1, both leapfrog levels, H_k(t)
// and W in LDS (5 N^2 complex128, 125 KB at N = 40), with the Peierls phase of
// each periodic image computed once per step (at most kSmallImages), and takes up to
// kSmallChunk steps per launch: per step the observables of D_n (the same
// lane mapping and arithmetic as k_observe, written per step to `part`), the
// Peierls assembly of H_k(t_n) (Eqs. 8-9) as a dense matrix, W = H D and
// Y = S^-1 W in LDS, and the leapfrog D_{n+1} = D_{n-1} - 2i dt (Y - Y^dag)
// (Eqs. 6, 13; forward Euler when there is no previous level).

// C = A B for complex n x n matrices in LDS on the FP64 matrix cores
// (v_mfma_f64_16x16x4: A operand of lane l = A[l % 16][l / 16], B operand =
// B[l / 16][l % 16], result element j at row l / 16 + 4 j, column l % 16).
// A is given transposed (At[k n + r] = A[r][k]) so that both operand reads are
// sixteen consecutive elements; one wavefront per 16 x 16 output tile, edges
// zero-filled.  Complex MAC: Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br.
__device__ inline void lds_zgemm(const double2 *At, const double2 *B, double2 *C, int n) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
  const int nt = (n + 15) >> 4;
  const double2 z = make_double2(0.0, 0.0);
  for (int tile = threadIdx.x >> 6; tile < nt * nt; tile += blockDim.x >> 6) {
    const int r0 = (tile / nt) * 16, c0 = (tile % nt) * 16;
    const int r = r0 + lr, c = c0 + lr;
    v4d cr = {0.0, 0.0, 0.0, 0.0}, ci = cr;
    for (int k0 = 0; k0 < n; k0 += 4) {
      const int kk = k0 + lk;
      const double2 a = (r < n && kk < n) ? At[kk * n + r] : z;
      const double2 b = (c < n && kk < n) ? B[kk * n + c] : z;
      cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, ci, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, ci, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = r0 + lk + 4 * j;
      if (row < n && c < n) C[row * n + c] = make_double2(cr[j], ci[j]);
    }
  }
}

// (cos, sin) of (k + A/c).d for every periodic image, into ph.
__device__ inline void small_phases(const PairGraph &g, double kx, double ky, double kz, double2 *ph) {
  for (int m = threadIdx.x; m < g.n_images; m += blockDim.x) {
    double sn, cs;
    sincos(kx * g.img_d[3 * m] + ky * g.img_d[3 * m + 1] + kz * g.img_d[3 * m + 2], &sn, &cs);
    ph[m] = make_double2(cs, sn);
  }
}

// H_k from the phase table, dense and transposed (Hm[c n + r] = H[r][c]),
// with the SCC term 1/2 (V_I + V_J) S_k of Eq. 10 when v is given.
template <int NO>
__device__ inline void small_assemble(const PairGraph &g, const double2 *ph, double2 *Hm, int n,
                                      const double *v = nullptr, const double2 *spk = nullptr,
                                      int k = 0) {
  constexpr int E2 = NO * NO;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) Hm[t] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int t = threadIdx.x; t < g.n_pairs * E2; t += blockDim.x) {
    const int p = t / E2, ee = t % E2;
    double2 h = make_double2(0.0, 0.0);
    for (int m = g.img_ptr[p]; m < g.img_ptr[p + 1]; ++m) {
      const double hv = g.img_h0[(size_t)m * E2 + ee];
      h.x += ph[m].x * hv;
      h.y += ph[m].y * hv;
    }
    if (v != nullptr) {
      const double vs = 0.5 * (v[g.pair_row[p]] + v[g.pair_col[p]]);
      const double2 sv = spk[((size_t)k * g.n_pairs + p) * E2 + ee];
      h.x += vs * sv.x;
      h.y += vs * sv.y;
    }
    Hm[(g.pair_col[p] * NO + ee % NO) * n + g.pair_row[p] * NO + ee / NO] = h;
  }
}

// Grid-wide barrier of a cooperative launch: every workgroup adds one arrival
// to *bar and waits until target arrivals are in.  The wait is bounded (about
// a second of sleeps); past it *err is set and false is returned, and the
// caller ends its launch.  Global writes before the barrier are visible to
// every workgroup after it (device-scope release and acquire).
__device__ inline bool small_grid_barrier(unsigned *bar, unsigned target, int *err) {
  __shared__ int ok;
  __threadfence();   // every wavefront's own writes of this step reach device scope
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(bar, 1u);
    int spins = 0;
    ok = 1;
    while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(8);
      if (++spins > (1 << 22) || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        atomicExch(err, 1);
        ok = 0;
        break;
      }
    }
  }
  __syncthreads();
  __threadfence();   // and every wavefront reads the other workgroups' writes
  return ok != 0;
}

// C0 = H0_k D0 (A = 0) of the deviation forms on the small path, with the same
// assembly and LDS product as the step kernel, so that a stationary density
// gives W = H D - C0 = 0 exactly.
template <int NO>
__global__ __launch_bounds__(256) void k_small_c0(PairGraph g, const double *__restrict__ kpts,
                                                  const double2 *__restrict__ d0,
                                                  double2 *__restrict__ c0, int n) {
  __shared__ double2 lds[3 * kSmallN * kSmallN];
  __shared__ double2 ph[kSmallImages];
  const int k = blockIdx.x;
  const int n2 = n * n;
  double2 *Hm = lds, *Dm = lds + n2, *Cm = lds + 2 * n2;
  const size_t base = (size_t)k * n2;
  for (int t = threadIdx.x; t < n2; t += blockDim.x) Dm[t] = d0[base + t];
  small_phases(g, kpts[3 * k] + 0.0, kpts[3 * k + 1] + 0.0, kpts[3 * k + 2] + 0.0, ph);
  __syncthreads();
  small_assemble<NO>(g, ph, Hm, n);
  __syncthreads();
  lds_zgemm(Hm, Dm, Cm, n);
  __syncthreads();
  for (int t = threadIdx.x; t < n2; t += blockDim.x) c0[base + t] = Cm[t];
}

// One complex multiply-add of the reduced product (S^-1 - I) W in the
// arithmetic of each deviation form, as the dense product kernels do it: FP32
// on complex64 operands; 3xBF16 / FP16X3 on hi/lo splits (x = hi + lo) of both
// operands, A_hi B_hi + A_hi B_lo + A_lo B_hi, with fp32 accumulation (products
// of two 16-bit values are exact in fp32); FP16X3 splits x s with the per-k
// powers of two sa, sw.  3xBF16 takes the lo part of S^-1 - I from copy
// `level` of its dithered representation (see kADither), as the per-step path.
template <int FORM>
__device__ inline void small_mac(double2 a, double2 w, float sa, float sw, int level, float &gr,
                                 float &gi) {
  if (FORM == 1) {
    const float ar = (float)a.x, ai = (float)a.y, wr = (float)w.x, wi = (float)w.y;
    gr = fmaf(ar, wr, gr);
    gr = fmaf(-ai, wi, gr);
    gi = fmaf(ar, wi, gi);
    gi = fmaf(ai, wr, gi);
    return;
  }
  float arh, arl, aih, ail, wrh, wrl, wih, wil;
  // W as the sparse product splits it; S^-1 - I as it is split once at creation
  // (the scaled value in FP64, then hi = fp16(x s), lo = fp16(x s - hi)).
  auto split = [&](double x, float sc, bool a_operand, float &hi, float &lo) {
    uint16_t h, l;
    if (FORM == 2) {
      if (a_operand) {
        const float xf = (float)x;
        h = to_bf16(xf);
        l = dithered_bf16(xf - from_bf16(h), level);
      } else {
        split_bf16(x, h, l);
      }
      hi = from_bf16(h);
      lo = from_bf16(l);
    } else if (a_operand) {
      const double xs = x * (double)sc;
      hi = (float)(_Float16)(float)xs;
      lo = (float)(_Float16)(float)(xs - (double)hi);
    } else {
      split_f16(x, sc, h, l);
      hi = (float)__builtin_bit_cast(_Float16, h);
      lo = (float)__builtin_bit_cast(_Float16, l);
    }
  };
  split(a.x, sa, true, arh, arl);
  split(a.y, sa, true, aih, ail);
  split(w.x, sw, false, wrh, wrl);
  split(w.y, sw, false, wih, wil);
  gr = fmaf(arh, wrh, gr);
  gr = fmaf(arh, wrl, gr);
  gr = fmaf(arl, wrh, gr);
  gr = fmaf(-aih, wih, gr);
  gr = fmaf(-aih, wil, gr);
  gr = fmaf(-ail, wih, gr);
  gi = fmaf(arh, wih, gi);
  gi = fmaf(arh, wil, gi);
  gi = fmaf(arl, wih, gi);
  gi = fmaf(aih, wrh, gi);
  gi = fmaf(aih, wrl, gi);
  gi = fmaf(ail, wrh, gi);
}

// Block-wide sum (thread 0's value valid for every thread after the call).
__device__ inline double block_sum_small(double v, double *red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  __syncthreads();
  return s;
}

// Deviation form of the product on the small path: W <- H D - C0 (FP64, in
// place), then Y = W + (S^-1 - I) W with the second term in the form's
// arithmetic (per element: complex64 W plus the complex64 product, summed in
// FP64, as the update of the per-step path reads them).  St = (S^-1)^T.
template <int FORM>
__device__ void small_deviation_product(const double2 *St, double2 *Wm, double2 *Y, int n,
                                        const SmallDeviation &dev, int k, size_t base, int level,
                                        double *red) {
  const int n2 = n * n;
  float m = 0.0f;
  for (int t = threadIdx.x; t < n2; t += blockDim.x) {
    double2 w = Wm[t];
    const double2 c = dev.c0[base + t];
    w.x -= c.x;
    w.y -= c.y;
    Wm[t] = w;
    if (FORM == 3) m = fmaxf(m, fmaxf(fabsf((float)w.x), fabsf((float)w.y)));
  }
  float sw = 1.0f, sa = 1.0f;
  if (FORM == 3) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = (double)m;
    __syncthreads();
    float mm = 0.0f;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) mm = fmaxf(mm, (float)red[w]);
    sw = f16_pow2_scale(mm);
    sa = dev.scale_a[k];
  }
  __syncthreads();
  const float us = FORM == 3 ? 1.0f / (sa * sw) : 1.0f;
  for (int t = threadIdx.x; t < n2; t += blockDim.x) {
    const int i = t / n, j = t - i * n;
    float gr = 0.0f, gi = 0.0f;
    for (int kk = 0; kk < n; ++kk) {
      double2 a = St[kk * n + i];             // S^-1[i][kk]
      if (kk == i) a.x -= 1.0;
      small_mac<FORM>(a, Wm[kk * n + j], sa, sw, level, gr, gi);
    }
    const double2 w = Wm[t];
    const float2 g = make_float2(us * gr, us * gi);
    double2 y = make_double2((double)g.x, (double)g.y);
    y.x += (double)(float)w.x;
    y.y += (double)(float)w.y;
    Y[t] = y;
  }
  __syncthreads();
}

// Rescale of the deviation forms on the small path: both levels
// D <- c 1/2 (D + D^dag) with c = target / Re Tr(D S_k) (S on the pair pattern).
template <int NO>
__device__ void small_rescale(const PairGraph &g, const double2 *__restrict__ spk, double2 *Da,
                              double2 *Db, int n, int k, double target, double *red) {
  constexpr int E2 = NO * NO;
  double ta = 0.0, tb = 0.0;
  for (int q = threadIdx.x; q < g.n_pairs * E2; q += blockDim.x) {
    const int p = q / E2, e = q - p * E2;
    const int idx = (g.pair_row[p] * NO + e / NO) * n + g.pair_col[p] * NO + e % NO;
    const double2 sv = spk[((size_t)k * g.n_pairs + p) * E2 + e];
    ta += Da[idx].x * sv.x + Da[idx].y * sv.y;
    tb += Db[idx].x * sv.x + Db[idx].y * sv.y;
  }
  const double ca = target / block_sum_small(ta, red);
  const double cb = target / block_sum_small(tb, red);
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int i = t / n, j = t - i * n;
    if (i > j) continue;
    for (int lev = 0; lev < 2; ++lev) {
      double2 *d = lev ? Db : Da;
      const double c = lev ? cb : ca;
      const double2 a = d[i * n + j], m = d[j * n + i];
      d[i * n + j] = make_double2(c * 0.5 * (a.x + m.x), c * 0.5 * (a.y - m.y));
      if (i != j) d[j * n + i] = make_double2(c * 0.5 * (m.x + a.x), c * 0.5 * (m.y - a.y));
    }
  }
  __syncthreads();
}

// The block of steps of k-point k (of nk) of one system, run by the calling
// workgroup; fa holds A(t_n)/c of the block's steps, three per step.  Shared
// by the one-system launch and the launch of several systems.
template <int NO, int FORM, bool SCC>
__device__ __forceinline__ void small_steps_body(const PairGraph &g, const double *__restrict__ kpts,
                                                 const double2 *__restrict__ spk,
                                                 const double2 *__restrict__ sinv, double2 *dlev0,
                                                 double2 *dlev1, int cur, int have_prev, int n,
                                                 const double *__restrict__ fa, int nsteps, double dt,
                                                 double *part, const SmallDeviation &dev, int k,
                                                 int nk) {
  constexpr int E2 = NO * NO;
  constexpr int P = 64 / E2;
  __shared__ double2 lds[5 * kSmallN * kSmallN];
  __shared__ double2 ph[kSmallImages];        // (cos, sin) of (k + A/c).d per image
  __shared__ double red[8];
  __shared__ double qv[SCC ? kSmallN : 1], vv[SCC ? kSmallN : 1];   // charges, SCC shift
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
  const int n2 = n * n;
  // St = (S_k^-1)^T; Hm holds H_k(t)^T, then Y = S^-1 W (row-major).
  double2 *St = lds, *Dc = lds + n2, *Dp = lds + 2 * n2, *Hm = lds + 3 * n2, *Wm = lds + 4 * n2;
  const size_t base = (size_t)k * n2;
  {
    const double2 *dc = cur ? dlev1 : dlev0, *dp = cur ? dlev0 : dlev1;
    for (int t = tid; t < n2; t += blockDim.x) {
      St[t] = sinv[base + (size_t)(t % n) * n + t / n];
      Dc[t] = dc[base + t];
      Dp[t] = have_prev ? dp[base + t] : make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  const int e = lane % E2, slot = lane / E2, mu = e / NO, nu = e % NO;
  bool hp = have_prev != 0;
  for (int s = 0; s < nsteps; ++s) {
    const double kx = kpts[3 * k] + fa[3 * s], ky = kpts[3 * k + 1] + fa[3 * s + 1],
                 kz = kpts[3 * k + 2] + fa[3 * s + 2];
    small_phases(g, kx, ky, kz, ph);   // Peierls phases of step n, once per image
    __syncthreads();
    // Observables of D_n: Mulliken row sums, band energy and current.
    for (int I = wave; I < g.n_atoms; I += nwaves) {
      double q = 0.0, en = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
      for (int p = g.row_ptr[I] + slot; p < g.row_ptr[I + 1]; p += P) {
        const int J = g.pair_col[p];
        const double2 dv = Dc[(I * NO + mu) * n + (J * NO + nu)];
        const double2 sv = spk[((size_t)k * g.n_pairs + p) * E2 + e];
        q += dv.x * sv.x + dv.y * sv.y;
        for (int m = g.img_ptr[p]; m < g.img_ptr[p + 1]; ++m) {
          const double dx = g.img_d[3 * m], dy = g.img_d[3 * m + 1], dz = g.img_d[3 * m + 2];
          const double cs = ph[m].x, sn = ph[m].y;
          const double h = g.img_h0[(size_t)m * E2 + e];
          const double re = (dv.x * cs + dv.y * sn) * h;
          const double im = (dv.x * sn - dv.y * cs) * h;
          en += re;
          jx -= dx * im;
          jy -= dy * im;
          jz -= dz * im;
        }
      }
      q = wave_sum(q);
      en = wave_sum(en);
      jx = wave_sum(jx);
      jy = wave_sum(jy);
      jz = wave_sum(jz);
      if (lane == 0) {
        double *o = part + (((size_t)s * nk + k) * g.n_atoms + I) * 5;
        o[0] = q;
        o[1] = en;
        o[2] = jx;
        o[3] = jy;
        o[4] = jz;
      }
    }
    if (SCC) {
      // Mulliken charges of D_n summed over every k-point (Eq. 10): wait for all
      // workgroups' partials of this step, then dq = q - Z and V = gamma dq.
      if (!small_grid_barrier(dev.bar, dev.bar_base + (unsigned)(s + 1) * (unsigned)nk, dev.err)) {
        nsteps = s;   // ends the launch with the state of this step
        break;
      }
      const int na = g.n_atoms;
      for (int I = tid; I < na; I += blockDim.x) {
        double q = 0.0;
        for (int kk = 0; kk < nk; ++kk) q += dev.kw[kk] * part[(((size_t)s * nk + kk) * na + I) * 5];
        qv[I] = q - dev.z[I];
      }
      __syncthreads();
      for (int I = tid; I < na; I += blockDim.x) {
        double v = 0.0;
        for (int K = 0; K < na; ++K) v += dev.gamma[(size_t)I * na + K] * qv[K];
        vv[I] = v;
      }
      __syncthreads();
      if (k == 0 && tid == 0) {
        double e = 0.0;
        for (int I = 0; I < na; ++I) e += 0.5 * qv[I] * vv[I];
        dev.escc[s] = e;
      }
      small_assemble<NO>(g, ph, Hm, n, vv, spk, k);   // H_k(t_n) with the SCC term
    } else {
      small_assemble<NO>(g, ph, Hm, n);  // H_k(t_n), dense and transposed
    }
    __syncthreads();
    lds_zgemm(Hm, Dc, Wm, n);     // W = H D_n
    __syncthreads();
    if (FORM == 0) {
      lds_zgemm(St, Wm, Hm, n);   // Y = S^-1 W (H no longer needed)
      __syncthreads();
    } else {
      small_deviation_product<FORM>(St, Wm, Hm, n, dev, k, base, (int)((dev.step0 + s) % kADither),
                                    red);
    }
    const double fac = hp ? 2.0 * dt : dt;
    const double2 *Db = hp ? Dp : Dc;
    for (int t = tid; t < n2; t += blockDim.x) {
      const int i = t / n, j = t - i * n;
      const double2 y = Hm[t], yt = Hm[j * n + i];
      const double xr = y.x - yt.x;           // X = Y - conj(Y^T)
      const double xi = y.y + yt.y;
      const double2 b = Db[t];
      double2 o = make_double2(b.x + fac * xi, b.y - fac * xr);
      if (FORM != 0 && dev.m0 != nullptr) {
        const double2 mv = dev.m0[base + t];
        o.x += fac * mv.x;
        o.y += fac * mv.y;
      }
      Dp[t] = o;
    }
    __syncthreads();
    double2 *tmp = Dc;
    Dc = Dp;
    Dp = tmp;
    hp = true;
    if (FORM != 0 && dev.rescale_every > 0 && (dev.step0 + s + 1) % dev.rescale_every == 0)
      small_rescale<NO>(g, spk, Dc, Dp, n, k, dev.trace0[k], red);
  }
  double2 *dc = ((cur ^ (nsteps & 1)) != 0) ? dlev1 : dlev0;
  double2 *dp = ((cur ^ (nsteps & 1)) != 0) ? dlev0 : dlev1;
  for (int t = tid; t < n2; t += blockDim.x) {
    dc[base + t] = Dc[t];
    if (hp) dp[base + t] = Dp[t];
  }
}

template <int NO, int FORM, bool SCC>
__global__ __launch_bounds__(256) void k_small_steps(PairGraph g, const double *__restrict__ kpts,
                                                     const double2 *__restrict__ spk,
                                                     const double2 *__restrict__ sinv,
                                                     double2 *dlev0, double2 *dlev1, int cur,
                                                     int have_prev, int n, FieldChunk f,
                                                     int nsteps, double dt,
                                                     double *part, SmallDeviation dev) {
  small_steps_body<NO, FORM, SCC>(g, kpts, spk, sinv, dlev0, dlev1, cur, have_prev, n, f.a, nsteps, dt,
                                  part, dev, blockIdx.x, gridDim.x);
}

// Several systems in one launch: workgroup w runs k-point w - wg0 of system
// wg_job[w].  With the SCC shift each system's workgroups meet at that
// system's own grid-wide barrier (the launch is cooperative, so all are
// resident).
template <int NO, int FORM, bool SCC>
__global__ __launch_bounds__(256) void k_small_group(const SmallJob *__restrict__ jobs,
                                                     const int *__restrict__ wg_job, int nsteps) {
  const SmallJob &J = jobs[wg_job[blockIdx.x]];
  small_steps_body<NO, FORM, SCC>(J.g, J.kpts, J.spk, J.sinv, J.dlev0, J.dlev1, J.cur, J.have_prev, J.n,
                                  J.field, nsteps, J.dt, J.part, J.dev, (int)blockIdx.x - J.wg0, J.nk);
}

// History rows of a block of steps from the per-(step, k, atom) partials of
// k_small_steps: for each step the same sums, in the same order, as
// k_reduce_atoms followed by k_reduce_final; with the SCC term the energy of
// each step adds the SCC energy the step kernel wrote to escc.
__device__ __forceinline__ void reduce_step_row(const double *__restrict__ part, int nk, int na,
                                                const double *__restrict__ kw, double jscale,
                                                double *hist, int64_t step0, int cap, int *flag,
                                                const double *__restrict__ escc, int s) {
  __shared__ double red[6][kReduceWaves];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  double *row = hist + (size_t)((step0 + s) % cap) * (5 + na);
  const double *ps = part + (size_t)s * nk * na * 5;
  double c[6] = {0, 0, 0, 0, 0, 0};
  for (int I = t; I < na; I += kReduceThreads) {
    double q = 0.0, en = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int k = 0; k < nk; ++k) {
      const double *o = ps + ((size_t)k * na + I) * 5;
      q += kw[k] * o[0];
      en += kw[k] * o[1];
      jx += kw[k] * o[2];
      jy += kw[k] * o[3];
      jz += kw[k] * o[4];
    }
    row[5 + I] = q;
    c[0] += en;
    c[1] += jx;
    c[2] += jy;
    c[3] += jz;
    c[4] += 0.0;
    c[5] += q;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    c[i] = wave_sum(c[i]);
    if (lane == 0) red[i][wave] = c[i];
  }
  __syncthreads();
  if (t == 0) {
    double o[6] = {0, 0, 0, 0, 0, 0};
    for (int w = 0; w < kReduceWaves; ++w)
      for (int i = 0; i < 6; ++i) o[i] += red[i][w];
    row[0] = o[1] * jscale;
    row[1] = o[2] * jscale;
    row[2] = o[3] * jscale;
    row[3] = o[0] + (escc != nullptr ? escc[s] : o[4]);
    row[4] = o[5];
    if (!isfinite(o[5]) || !isfinite(o[0])) *flag = 1;
  }
}

__global__ __launch_bounds__(kReduceThreads) void k_reduce_steps(const double *__restrict__ part,
                                                                 int nk, int na,
                                                                 const double *__restrict__ kw,
                                                                 double jscale, double *hist,
                                                                 int64_t step0, int cap,
                                                                 int *flag,
                                                                 const double *__restrict__ escc) {
  reduce_step_row(part, nk, na, kw, jscale, hist, step0, cap, flag, escc, blockIdx.x);
}

// History rows of several systems' blocks: step blockIdx.x of system blockIdx.y.
__global__ __launch_bounds__(kReduceThreads) void k_reduce_group(const SmallJob *__restrict__ jobs) {
  const SmallJob &J = jobs[blockIdx.y];
  reduce_step_row(J.part, J.nk, J.na, J.kw, J.jscale, J.hist, J.step0, J.cap, J.flag, J.dev.escc,
                  blockIdx.x);
}

// Leapfrog (Eq. 13) in the form D_out = D_base - i fac (Y - Y^dag), Y = S^-1 H D,
// so that dD/dt = -i (Y - Y^dag) is anti-Hermitian bit for bit.  One workgroup
// takes the pair of 32x32 tiles (I, J), (J, I) with I <= J: both tiles of Y are
// staged in LDS once and both tiles of D_out are written from them, so every
// element of Y (and W) is read once per step.  D_out may be D_base (each
// element is read and written by the same thread).
// SPLIT: the product is Y = W + G with G = (S^-1 - I) W computed separately;
// both are complex64 and are summed in FP64 here.
// m0 (may be null): a constant term -i X0 added as fac * m0, where
// X0 = S^-1 H0 D0 - D0 H0 S^-1 is the part of dD/dt the deviation form leaves
// out when the reference density D0 is not stationary.
// Y at rows r0 + ty + 8q, column c0 + tx (q = 0..3) into v; zero outside n.
template <typename YT, bool SPLIT>
__device__ inline void update_load(const YT *__restrict__ y, const float2 *__restrict__ wsplit,
                                   size_t base, int n, int r0, int c0, double2 (&v)[4]) {
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int c = c0 + tx;
  YT yv[4];
  float2 wv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = r0 + ty + 8 * q;
    const bool in = row < n && c < n;
    const size_t idx = base + (size_t)(in ? row : 0) * n + (in ? c : 0);
    yv[q] = y[idx];
    if (SPLIT) wv[q] = wsplit[idx];
    if (!in) {
      yv[q].x = 0;
      yv[q].y = 0;
      if (SPLIT) wv[q] = make_float2(0.0f, 0.0f);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    v[q] = make_double2((double)yv[q].x, (double)yv[q].y);
    if (SPLIT) {
      v[q].x += (double)wv[q].x;
      v[q].y += (double)wv[q].y;
    }
  }
}

// Rows r0.., columns c0.. of D_out from `own` (this tile of Y) and `other`
// (the tile at the mirrored position: other[c][r] = Y[c0 + c][r0 + r]).
__device__ inline void update_store(const double2 (*own)[33], const double2 (*other)[33],
                                    const double2 *__restrict__ m0, const double2 *dbase,
                                    double2 *dout, size_t base, int n, int r0, int c0, double fac) {
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = ty + 8 * q;
    const int i = r0 + r, j = c0 + tx;
    if (i < n && j < n) {
      const size_t idx = base + (size_t)i * n + j;
      const double2 yv = own[r][tx];
      const double2 yt = other[tx][r];         // Y[j][i]
      const double xr = yv.x - yt.x;           // X = Y - conj(Y^T)
      const double xi = yv.y + yt.y;
      const double2 b = dbase[idx];
      double2 o = make_double2(b.x + fac * xi, b.y - fac * xr);
      if (m0 != nullptr) {
        const double2 mv = m0[idx];
        o.x += fac * mv.x;
        o.y += fac * mv.y;
      }
      dout[idx] = o;
    }
  }
}

template <typename YT, bool SPLIT>
__global__ __launch_bounds__(256) void k_update(const YT *__restrict__ y,
                                                const float2 *__restrict__ wsplit,
                                                const double2 *__restrict__ m0,
                                                const double2 *dbase, double2 *dout, int n,
                                                double fac, int64_t *ctr) {
  __shared__ double2 ta[32][33], tb[32][33];   // Y(I, J), Y(J, I)
  const int k = blockIdx.z;
  const size_t base = (size_t)k * n * n;
  // Pair p = tj (tj + 1) / 2 + ti with ti <= tj.
  const int p = blockIdx.x;
  int tj = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
  while ((tj + 1) * (tj + 2) / 2 <= p) ++tj;
  while (tj * (tj + 1) / 2 > p) --tj;
  const int ti = p - tj * (tj + 1) / 2;
  const int bi = ti * 32, bj = tj * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  double2 va[4], vb[4];
  // All global loads of both tiles are issued before the first LDS write.
  update_load<YT, SPLIT>(y, wsplit, base, n, bi, bj, va);
  if (ti != tj) update_load<YT, SPLIT>(y, wsplit, base, n, bj, bi, vb);
#pragma unroll
  for (int q = 0; q < 4; ++q) ta[ty + 8 * q][tx] = va[q];
  if (ti != tj) {
#pragma unroll
    for (int q = 0; q < 4; ++q) tb[ty + 8 * q][tx] = vb[q];
  }
  __syncthreads();
  update_store(ta, ti != tj ? tb : ta, m0, dbase, dout, base, n, bi, bj, fac);
  if (ti != tj) update_store(tb, ta, m0, dbase, dout, base, n, bj, bi, fac);
  // The step is done once this kernel has run: advance the device step index
  // (no other thread of this kernel reads it).
  if (ctr != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0)
    *ctr += 1;
}

// After a lower-triangle result (row-major): m[i][j] = conj(m[j][i]) for i < j,
// diagonal made real.
__global__ void k_hermitian_from_lower(double2 *m, int n) {
  const int k = blockIdx.z;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= n || j >= n) return;
  double2 *mk = m + (size_t)k * n * n;
  if (i < j) {
    const double2 lo = mk[(size_t)j * n + i];
    mk[(size_t)i * n + j] = make_double2(lo.x, -lo.y);
  } else if (i == j) {
    mk[(size_t)i * n + i].y = 0.0;
  }
}

// D[i][j] = sum_n occ[n] c_n[i] conj(c_n[j]) where row n of evec holds conj(c_n)
// (the column-major eigenvectors of the conjugated problem seen row-major).
// Lower triangle computed, upper mirrored: exactly Hermitian.
__global__ __launch_bounds__(256) void k_density_from_vectors(const double2 *__restrict__ evec,
                                                              const double *__restrict__ occ,
                                                              double2 *__restrict__ d, int n) {
  __shared__ double2 ei[16][17];
  __shared__ double2 ej[16][17];
  const int k = blockIdx.z;
  const int bi = blockIdx.y * 16, bj = blockIdx.x * 16;
  if (bj > bi + 15) return;   // tile strictly above the diagonal
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const double2 *ek = evec + (size_t)k * n * n;
  const double *ok = occ + (size_t)k * n;
  const int i = bi + ty, j = bj + tx;
  double2 acc = make_double2(0.0, 0.0);
  for (int n0 = 0; n0 < n; n0 += 16) {
    const int nn = n0 + ty;
    const double f = (nn < n) ? ok[nn] : 0.0;
    ei[ty][tx] = (nn < n && bi + tx < n) ? ek[(size_t)nn * n + bi + tx] : make_double2(0.0, 0.0);
    const double2 vj = (nn < n && bj + tx < n) ? ek[(size_t)nn * n + bj + tx] : make_double2(0.0, 0.0);
    ej[ty][tx] = make_double2(f * vj.x, f * vj.y);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const double2 a = ei[s][ty];    // conj(c_n[i])
      const double2 b = ej[s][tx];    // f conj(c_n[j])
      // c_n[i] conj(c_n[j]) = conj(a) * b
      acc.x += a.x * b.x + a.y * b.y;
      acc.y += a.x * b.y - a.y * b.x;
    }
    __syncthreads();
  }
  if (i < n && j < n && i >= j) {
    double2 *dk = d + (size_t)k * n * n;
    if (i == j) {
      dk[(size_t)i * n + i] = make_double2(acc.x, 0.0);
    } else {
      dk[(size_t)i * n + j] = acc;
      dk[(size_t)j * n + i] = make_double2(acc.x, -acc.y);
    }
  }
}

// S^-1 - I in the operand format of the reduced-precision product (the
// identity part of S^-1 W is added back exactly in the update).
// fmt 1: complex64 row-major (n); fmt 2: four bf16 planes row-major, padded np.
__global__ void k_convert_operand(const double2 *__restrict__ src, void *__restrict__ dst, int n,
                                  int np, int nk, int fmt) {
  const int k = blockIdx.z;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (fmt == 1) {
    if (j >= n) return;
    double2 v = src[(size_t)k * n * n + (size_t)i * n + j];
    if (i == j) v.x -= 1.0;
    static_cast<float2 *>(dst)[(size_t)k * n * n + (size_t)i * n + j] = make_float2((float)v.x, (float)v.y);
  } else {
    if (j >= np) return;
    double2 v = make_double2(0.0, 0.0);
    if (i < n && j < n) v = src[(size_t)k * n * n + (size_t)i * n + j];
    if (i == j && i < n) v.x -= 1.0;
    uint16_t rh, ih;
    float rr, ri;   // remainders after hi (exact in float)
    {
      const float xr = (float)v.x, xi = (float)v.y;
      rh = to_bf16(xr);
      ih = to_bf16(xi);
      rr = xr - from_bf16(rh);
      ri = xi - from_bf16(ih);
    }
    uint16_t *o = static_cast<uint16_t *>(dst);
    const size_t plane = (size_t)nk * np * np;
    const size_t idx = (size_t)k * np * np + (size_t)i * np + j;
    for (int lev = 0; lev < kADither; ++lev) {
      uint16_t *ol = o + (size_t)lev * 4 * plane;
      ol[idx] = rh;
      ol[plane + idx] = dithered_bf16(rr, lev);
      ol[2 * plane + idx] = ih;
      ol[3 * plane + idx] = dithered_bf16(ri, lev);
    }
  }
}

// Per-row partial traces Re sum_{pairs of I} D_{mu nu} conj(S_{mu nu}) of one level.
template <int NO>
__global__ __launch_bounds__(64) void k_trace_rows(PairGraph g, const double2 *__restrict__ da,
                                                   const double2 *__restrict__ db, int n,
                                                   const double2 *__restrict__ spk, double *tpart) {
  constexpr int E2 = NO * NO;
  constexpr int P = 64 / E2;
  const int I = blockIdx.x, k = blockIdx.y, lev = blockIdx.z;
  const double2 *d = lev ? db : da;
  const int lane = threadIdx.x, e = lane % E2, slot = lane / E2, mu = e / NO, nu = e % NO;
  const size_t base = (size_t)k * n * n;
  double q = 0.0;
  for (int p = g.row_ptr[I] + slot; p < g.row_ptr[I + 1]; p += P) {
    const size_t idx = base + (size_t)(I * NO + mu) * n + (g.pair_col[p] * NO + nu);
    const double2 a = d[idx], sv = spk[((size_t)k * g.n_pairs + p) * E2 + e];
    q += a.x * sv.x + a.y * sv.y;
  }
  q = wave_sum(q);
  if (lane == 0) tpart[((size_t)lev * gridDim.y + k) * g.n_atoms + I] = q;
}

// mode 0: fac[lev*nk+k] = target[k] / trace(lev, k);  mode 1: target[k] = trace(0, k).
__global__ void k_trace_factors(const double *__restrict__ tpart, double *target, double *fac,
                                int nk, int na, int mode) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * nk) return;
  double s = 0.0;
  for (int I = 0; I < na; ++I) s += tpart[(size_t)t * na + I];
  if (mode == 1) {
    if (t < nk) target[t] = s;
  } else {
    fac[t] = target[t % nk] / s;
  }
}

// Both levels: D <- c * 1/2 (D + D^dag).  A tile pair (bi <= bj) is handled by
// one block so the in-place update never races with its mirror; the grid holds
// only the pairs (blockIdx.x = bj (bj + 1) / 2 + bi, as in k_update), and each
// thread issues all its loads of both tiles before the first LDS write.
__global__ __launch_bounds__(256) void k_rescale(double2 *da, double2 *db,
                                                 const double *__restrict__ fac, int n) {
  __shared__ double2 t1[32][33], t2[32][33];
  const int p = blockIdx.x;
  int tj = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
  while ((tj + 1) * (tj + 2) / 2 <= p) ++tj;
  while (tj * (tj + 1) / 2 > p) --tj;
  const int bi = p - tj * (tj + 1) / 2, bj = tj;
  const int k = blockIdx.y, lev = blockIdx.z;
  double2 *d = lev ? db : da;
  const double c = fac[lev * gridDim.y + k];
  const size_t base = (size_t)k * n * n;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const double2 z = make_double2(0.0, 0.0);
  double2 v1[4], v2[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = ty + 8 * q;
    const int i1 = bi * 32 + r, j1 = bj * 32 + tx;
    const int i2 = bj * 32 + r, j2 = bi * 32 + tx;
    v1[q] = (i1 < n && j1 < n) ? d[base + (size_t)i1 * n + j1] : z;   // tile (bi, bj)
    v2[q] = (bi != bj && i2 < n && j2 < n) ? d[base + (size_t)i2 * n + j2] : z;   // tile (bj, bi)
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    t1[ty + 8 * q][tx] = v1[q];
    t2[ty + 8 * q][tx] = v2[q];
  }
  __syncthreads();
  // On the diagonal the mirror of tile (bi, bi) is itself.
  auto mirror = [&](int r, int cc) -> const double2 & { return bi != bj ? t2[cc][r] : t1[cc][r]; };
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = ty + 8 * q;
    const int i1 = bi * 32 + r, j1 = bj * 32 + tx;
    if (i1 < n && j1 < n) {
      const double2 a = t1[r][tx], m = mirror(r, tx);        // D[i][j], D[j][i]
      d[base + (size_t)i1 * n + j1] = make_double2(c * 0.5 * (a.x + m.x), c * 0.5 * (a.y - m.y));
    }
    if (bi != bj) {
      const int i2 = bj * 32 + r, j2 = bi * 32 + tx;
      if (i2 < n && j2 < n) {
        const double2 b = t2[r][tx], m = t1[tx][r];
        d[base + (size_t)i2 * n + j2] = make_double2(c * 0.5 * (b.x + m.x), c * 0.5 * (b.y - m.y));
      }
    }
  }
}

// Filtered Fourier transform of the current (Eq. 15) and the dielectric
// function (Eq. 16): one wavefront per frequency, fixed-order lane sums.
inline unsigned blocks_for(size_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void launch_fill_zero(double2 *p, size_t n, hipStream_t s) {
  unsigned b = blocks_for(n, 256);
  if (b > 65536u) b = 65536u;
  if (b == 0) return;
  hipLaunchKernelGGL(k_fill_zero, dim3(b), dim3(256), 0, s, p, n);
}

void launch_pair_bloch_s(const PairGraph &g, const double *kpts, int nk, double2 *spk,
                         hipStream_t s) {
  const size_t tot = (size_t)g.n_pairs * g.norb * g.norb;
  hipLaunchKernelGGL(k_pair_bloch_s, dim3(blocks_for(tot, 256), nk), dim3(256), 0, s, g, kpts,
                     spk);
}

void launch_scatter_pairs(const PairGraph &g, const double *kpts, int nk, const double2 *spk,
                          int which, double2 *dense, int n, hipStream_t s) {
  const size_t tot = (size_t)g.n_pairs * g.norb * g.norb;
  hipLaunchKernelGGL(k_scatter_pairs, dim3(blocks_for(tot, 256), nk), dim3(256), 0, s, g, kpts,
                     spk, which, dense, n);
}

void launch_observe(const PairGraph &g, const double2 *d, int n, const double *kpts, int nk,
                    StepSource src, const double2 *spk, const double2 *h0k, const double2 *ppk,
                    double *part, hipStream_t s) {
  dim3 grid(g.n_atoms, nk);
  if (g.norb == 4)
    hipLaunchKernelGGL(k_observe<4>, grid, dim3(64), 0, s, g, d, n, kpts, src, spk, h0k, ppk, part);
  else
    hipLaunchKernelGGL(k_observe<1>, grid, dim3(64), 0, s, g, d, n, kpts, src, spk, h0k, ppk, part);
}

void launch_pair_bloch_momentum(const PairGraph &g, const double *kpts, int nk, double2 *h0k,
                                double2 *ppk, hipStream_t s) {
  dim3 grid(blocks_for((size_t)g.n_pairs * g.norb * g.norb, 256), nk);
  hipLaunchKernelGGL(k_pair_bloch_momentum, grid, dim3(256), 0, s, g, kpts, h0k, ppk);
}

void launch_store_ring(const FieldChunk &f, int64_t step0, int ns, double *ring, hipStream_t s) {
  hipLaunchKernelGGL(k_store_ring, dim3(1), dim3(3 * kSmallChunk), 0, s, f, step0, ns, ring);
}

void launch_advance_counter(int64_t *ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_advance_counter, dim3(1), dim3(1), 0, s, ctr);
}

void launch_set_counter(int64_t *ctr, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, s, ctr, v);
}

void launch_reduce(const double *part, int nk, int na, const double *kw, double jscale,
                   const double *gamma, const double *z, double *v, double *qbuf,
                   double *rowpart, double *hist, int cap, const int64_t *ctr, int *flag,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_atoms, dim3(blocks_for(na, 256)), dim3(256), 0, s, part, nk, na, kw,
                     qbuf, rowpart, hist, cap, ctr);
  if (gamma != nullptr)
    hipLaunchKernelGGL(k_reduce_scc, dim3(blocks_for(na, 16)), dim3(1024), 0, s, na, gamma, z, qbuf,
                       v, rowpart);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kReduceThreads), 0, s, na, jscale, qbuf, rowpart,
                     hist, cap, ctr, flag);
}

template <int NO, bool DELTA, int OUT>
static void spmm_launch(int threads, hipStream_t s, const PairGraph &g, const double2 *d,
                        int n, const double2 *hq, const double2 *c0, void *w,
                        int np, int nk, float2 *w32, int cpt, int ncols, const float *wscale,
                        unsigned *wmax) {
  const int ng = g.n_groups;
  if (g.group_size == 8 && cpt == 1)
    hipLaunchKernelGGL((k_spmm<NO, DELTA, OUT, 8, 1>), dim3(blocks_for(ncols, threads), ng, nk),
                       dim3(threads), 0, s, g, d, n, hq, c0, w, np, nk, w32, wscale, wmax);
  else if (g.group_size == 4 && cpt == 2)
    hipLaunchKernelGGL((k_spmm<NO, DELTA, OUT, 4, 2>), dim3(blocks_for(ncols, 2 * threads), ng, nk),
                       dim3(threads), 0, s, g, d, n, hq, c0, w, np, nk, w32, wscale, wmax);
  else if (g.group_size == 4 && cpt == 1)
    hipLaunchKernelGGL((k_spmm<NO, DELTA, OUT, 4, 1>), dim3(blocks_for(ncols, threads), ng, nk),
                       dim3(threads), 0, s, g, d, n, hq, c0, w, np, nk, w32, wscale, wmax);
  else
    hipLaunchKernelGGL((k_spmm<NO, DELTA, OUT, 8, 2>), dim3(blocks_for(ncols, 2 * threads), ng, nk),
                       dim3(threads), 0, s, g, d, n, hq, c0, w, np, nk, w32, wscale, wmax);
}

void launch_assemble(const PairGraph &g, const double *kpts, int nk, StepSource src,
                     const double2 *spk, const double *v, double2 *hq, const double2 *h0k,
                     const double2 *ppk, hipStream_t s) {
  const size_t tot = (size_t)g.n_pairs * g.norb * g.norb;
  dim3 grid(blocks_for(tot, 256), nk);
  if (g.norb == 4)
    hipLaunchKernelGGL(k_assemble<4>, grid, dim3(256), 0, s, g, kpts, src, spk, v, hq, h0k, ppk);
  else
    hipLaunchKernelGGL(k_assemble<1>, grid, dim3(256), 0, s, g, kpts, src, spk, v, hq, h0k, ppk);
}

template <bool DELTA, int OUT, int CB, bool G3>
static void spmm_mfma_launch_cb(hipStream_t s, const PairGraph &g, const double2 *d, int n,
                                const double2 *hq, const double2 *c0, void *w, int np, int nk,
                                float2 *w32, int ncols, const float *wscale, unsigned *wmax) {
  const int nw = std::max(1, std::min(4, (ncols + 16 * CB - 1) / (16 * CB)));
  dim3 grid(blocks_for(ncols, 16 * CB * nw), g.n_groups, nk);
  if (g.group_size == 16)
    hipLaunchKernelGGL((k_spmm_mfma<DELTA, OUT, 16, CB, G3>), grid, dim3(64 * nw), 0, s, g, d, n, hq,
                       c0, w, np, nk, w32, wscale, wmax);
  else if (g.group_size == 8)
    hipLaunchKernelGGL((k_spmm_mfma<DELTA, OUT, 8, CB, G3>), grid, dim3(64 * nw), 0, s, g, d, n, hq, c0,
                       w, np, nk, w32, wscale, wmax);
  else
    hipLaunchKernelGGL((k_spmm_mfma<DELTA, OUT, 4, CB, G3>), grid, dim3(64 * nw), 0, s, g, d, n, hq, c0,
                       w, np, nk, w32, wscale, wmax);
}

template <bool DELTA, int OUT>
static void spmm_mfma_launch(hipStream_t s, const PairGraph &g, const double2 *d, int n,
                             const double2 *hq, const double2 *c0, void *w, int np, int nk,
                             float2 *w32, int cb, bool g3, int ncols, const float *wscale,
                             unsigned *wmax) {
#define VG_CB(CB, G3) spmm_mfma_launch_cb<DELTA, OUT, CB, G3>(s, g, d, n, hq, c0, w, np, nk, w32, ncols, wscale, wmax)
  if (g3) {
    if (cb == 4) VG_CB(4, true);
    else if (cb == 2) VG_CB(2, true);
    else VG_CB(1, true);
  } else {
    if (cb == 4) VG_CB(4, false);
    else if (cb == 2) VG_CB(2, false);
    else VG_CB(1, false);
  }
#undef VG_CB
}

void launch_spmm(const PairGraph &g, const double2 *d, const double2 *d0, int n, int nk,
                 const double2 *hq, const double2 *c0, void *w, int out_format, int np,
                 float2 *w32, int variant, hipStream_t s, int ncols, const float *wscale,
                 unsigned *wmax) {
  if (ncols <= 0 || ncols > n) ncols = n;
  if (g.norb == 4 && variant < 0) {
    const bool g3 = variant <= -10;   // -11, -12, -14: three real products per complex one
    const int cb = g3 ? -variant - 10 : -variant;
#define VG_SPMM_MFMA(DL, OUT) spmm_mfma_launch<DL, OUT>(s, g, d, n, hq, c0, w, np, nk, w32, cb, g3, ncols, wscale, wmax)
    if (!d0) VG_SPMM_MFMA(false, 0);
    else if (out_format == 0) VG_SPMM_MFMA(true, 0);
    else if (out_format == 1) VG_SPMM_MFMA(true, 1);
    else if (out_format == 2) VG_SPMM_MFMA(true, 2);
    else VG_SPMM_MFMA(true, 3);
#undef VG_SPMM_MFMA
    return;
  }
  const int cpt = variant == 2 ? 2 : 1;
  const int threads = n >= 256 ? 256 : (n > 64 ? 128 : 64);
#define VG_SPMM(NO, DL, OUT) spmm_launch<NO, DL, OUT>(threads, s, g, d, n, hq, c0, w, np, nk, w32, cpt, ncols, wscale, wmax)
  if (g.norb == 4) {
    if (!d0) VG_SPMM(4, false, 0);
    else if (out_format == 0) VG_SPMM(4, true, 0);
    else if (out_format == 1) VG_SPMM(4, true, 1);
    else if (out_format == 2) VG_SPMM(4, true, 2);
    else VG_SPMM(4, true, 3);
  } else {
    if (!d0) VG_SPMM(1, false, 0);
    else if (out_format == 0) VG_SPMM(1, true, 0);
    else if (out_format == 1) VG_SPMM(1, true, 1);
    else if (out_format == 2) VG_SPMM(1, true, 2);
    else VG_SPMM(1, true, 3);
  }
#undef VG_SPMM
}

// Tile pairs (I <= J) of 32x32 tiles: one workgroup each.
static int update_pairs(int n) {
  const int t = blocks_for(n, 32);
  return t * (t + 1) / 2;
}

void launch_update(const double2 *y, const double2 *dbase, double2 *dout, int n, int nk,
                   double fac, int64_t *ctr, hipStream_t s) {
  dim3 grid(update_pairs(n), 1, nk);
  hipLaunchKernelGGL((k_update<double2, false>), grid, dim3(256), 0, s, y, (const float2 *)nullptr,
                     (const double2 *)nullptr, dbase, dout, n, fac, ctr);
}

void launch_update_split(const float2 *g, const float2 *w, const double2 *m0, const double2 *dbase,
                         double2 *dout, int n, int nk, double fac, int64_t *ctr, hipStream_t s) {
  dim3 grid(update_pairs(n), 1, nk);
  hipLaunchKernelGGL((k_update<float2, true>), grid, dim3(256), 0, s, g, w, m0, dbase, dout, n, fac,
                     ctr);
}

void launch_update_const(const double2 *y, const double2 *dbase, double2 *dout, int n, int nk,
                         hipStream_t s) {
  dim3 grid(update_pairs(n), 1, nk);
  hipLaunchKernelGGL((k_update<double2, false>), grid, dim3(256), 0, s, y, (const float2 *)nullptr,
                     (const double2 *)nullptr, dbase, dout, n, 1.0, (int64_t *)nullptr);
}

void launch_convert_operand(const double2 *src, void *dst, int n, int np, int nk, int fmt,
                            hipStream_t s) {
  const int cols = fmt == 1 ? n : np;
  const int rows = fmt == 1 ? n : np;
  hipLaunchKernelGGL(k_convert_operand, dim3(blocks_for(cols, 256), rows, nk), dim3(256), 0, s, src,
                     dst, n, np, nk, fmt);
}

void launch_trace_target(const PairGraph &g, const double2 *dd, int n, int nk, const double2 *spk,
                         double *tpart, double *target, hipStream_t s) {
  dim3 grid(g.n_atoms, nk, 2);
  if (g.norb == 4) hipLaunchKernelGGL(k_trace_rows<4>, grid, dim3(64), 0, s, g, dd, dd, n, spk, tpart);
  else hipLaunchKernelGGL(k_trace_rows<1>, grid, dim3(64), 0, s, g, dd, dd, n, spk, tpart);
  hipLaunchKernelGGL(k_trace_factors, dim3(blocks_for(2 * nk, 64)), dim3(64), 0, s, tpart, target,
                     (double *)nullptr, nk, g.n_atoms, 1);
}

void launch_rescale(const PairGraph &g, double2 *da, double2 *db, int n, int nk, const double2 *spk,
                    double *tpart, const double *target, double *fac, hipStream_t s) {
  dim3 grid(g.n_atoms, nk, 2);
  if (g.norb == 4) hipLaunchKernelGGL(k_trace_rows<4>, grid, dim3(64), 0, s, g, da, db, n, spk, tpart);
  else hipLaunchKernelGGL(k_trace_rows<1>, grid, dim3(64), 0, s, g, da, db, n, spk, tpart);
  hipLaunchKernelGGL(k_trace_factors, dim3(blocks_for(2 * nk, 64)), dim3(64), 0, s, tpart,
                     const_cast<double *>(target), fac, nk, g.n_atoms, 0);
  const int nt = (int)blocks_for(n, 32);
  hipLaunchKernelGGL(k_rescale, dim3(nt * (nt + 1) / 2, nk, 2), dim3(256), 0, s, da, db, fac, n);
}

template <int NO, int FORM, bool SCC>
static hipError_t small_steps_launch(const PairGraph &g, const double *kpts, int nk, const double2 *spk,
                                     const double2 *sinv, double2 *dlev0, double2 *dlev1, int cur,
                                     bool have_prev, int n, const FieldChunk &f, int nsteps, double dt,
                                     double *part, const SmallDeviation &dev, hipStream_t s) {
  if (!SCC) {
    hipLaunchKernelGGL((k_small_steps<NO, FORM, false>), dim3(nk), dim3(256), 0, s, g, kpts, spk, sinv,
                       dlev0, dlev1, cur, have_prev ? 1 : 0, n, f, nsteps, dt, part, dev);
    return hipGetLastError();
  }
  PairGraph ga = g;
  const double *ka = kpts;
  const double2 *sa = spk, *si = sinv;
  double2 *d0 = dlev0, *d1 = dlev1;
  int ca = cur, hpa = have_prev ? 1 : 0, na = n, ns = nsteps;
  FieldChunk fa = f;
  double dta = dt;
  double *pa = part;
  SmallDeviation da = dev;
  void *args[] = {&ga, &ka, &sa, &si, &d0, &d1, &ca, &hpa, &na, &fa, &ns, &dta, &pa, &da};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_small_steps<NO, FORM, true>),
                                    dim3(nk), dim3(256), args, 0, s);
}

template <int NO>
static hipError_t small_steps_form(const PairGraph &g, const double *kpts, int nk, const double2 *spk,
                                   const double2 *sinv, double2 *dlev0, double2 *dlev1, int cur,
                                   bool have_prev, int n, const FieldChunk &f, int nsteps, double dt,
                                   double *part, const SmallDeviation &dev, hipStream_t s) {
#define VG_SMALL(FORM, SCC)                                                                        \
  return small_steps_launch<NO, FORM, SCC>(g, kpts, nk, spk, sinv, dlev0, dlev1, cur, have_prev, n, f, \
                                           nsteps, dt, part, dev, s)
  const bool scc = dev.gamma != nullptr;
  if (dev.form == 1) { if (scc) VG_SMALL(1, true); else VG_SMALL(1, false); }
  if (dev.form == 2) { if (scc) VG_SMALL(2, true); else VG_SMALL(2, false); }
  if (dev.form == 3) { if (scc) VG_SMALL(3, true); else VG_SMALL(3, false); }
  if (scc) VG_SMALL(0, true);
  VG_SMALL(0, false);
#undef VG_SMALL
}

int small_scc_max_kpoints(int norb) {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const void *kfn = norb == 4 ? reinterpret_cast<const void *>(&k_small_steps<4, 0, true>)
                              : reinterpret_cast<const void *>(&k_small_steps<1, 0, true>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, 256, 0) != hipSuccess) return 0;
  return per_cu * cus;
}

template <int NO, int FORM, bool SCC>
static hipError_t small_group_launch(const SmallJob *jobs, const int *wg_job, int n_wg, int nsteps,
                                     hipStream_t s) {
  if (!SCC) {
    hipLaunchKernelGGL((k_small_group<NO, FORM, false>), dim3(n_wg), dim3(256), 0, s, jobs, wg_job, nsteps);
    return hipGetLastError();
  }
  const SmallJob *ja = jobs;
  const int *wa = wg_job;
  int ns = nsteps;
  void *args[] = {&ja, &wa, &ns};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_small_group<NO, FORM, true>),
                                    dim3(n_wg), dim3(256), args, 0, s);
}

template <int NO>
static hipError_t small_group_form(const SmallJob *jobs, const int *wg_job, int n_wg, int form, bool scc,
                                   int nsteps, hipStream_t s) {
#define VG_GROUP(FORM, SCC) return small_group_launch<NO, FORM, SCC>(jobs, wg_job, n_wg, nsteps, s)
  if (form == 1) { if (scc) VG_GROUP(1, true); else VG_GROUP(1, false); }
  if (form == 2) { if (scc) VG_GROUP(2, true); else VG_GROUP(2, false); }
  if (form == 3) { if (scc) VG_GROUP(3, true); else VG_GROUP(3, false); }
  if (scc) VG_GROUP(0, true);
  VG_GROUP(0, false);
#undef VG_GROUP
}

hipError_t launch_small_group(const SmallJob *jobs, const int *wg_job, int n_jobs, int n_wg, int norb,
                              int form, bool scc, int nsteps, hipStream_t s) {
  const hipError_t e = norb == 4 ? small_group_form<4>(jobs, wg_job, n_wg, form, scc, nsteps, s)
                                 : small_group_form<1>(jobs, wg_job, n_wg, form, scc, nsteps, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_group, dim3(nsteps, n_jobs), dim3(kReduceThreads), 0, s, jobs);
  return hipGetLastError();
}

int small_group_max_workgroups(int norb, int form) {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const void *kfn = nullptr;
#define VG_FN(NO, FORM) kfn = reinterpret_cast<const void *>(&k_small_group<NO, FORM, true>)
  if (norb == 4) {
    if (form == 1) VG_FN(4, 1); else if (form == 2) VG_FN(4, 2); else if (form == 3) VG_FN(4, 3); else VG_FN(4, 0);
  } else {
    if (form == 1) VG_FN(1, 1); else if (form == 2) VG_FN(1, 2); else if (form == 3) VG_FN(1, 3); else VG_FN(1, 0);
  }
#undef VG_FN
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, 256, 0) != hipSuccess) return 0;
  return per_cu * cus;
}

void launch_small_c0(const PairGraph &g, const double *kpts, int nk, const double2 *d0, double2 *c0,
                     int n, hipStream_t s) {
  if (g.norb == 4) hipLaunchKernelGGL(k_small_c0<4>, dim3(nk), dim3(256), 0, s, g, kpts, d0, c0, n);
  else hipLaunchKernelGGL(k_small_c0<1>, dim3(nk), dim3(256), 0, s, g, kpts, d0, c0, n);
}

hipError_t launch_small_steps(const PairGraph &g, const double *kpts, int nk, const double2 *spk,
                              const double2 *sinv, double2 *dlev0, double2 *dlev1, int cur,
                              bool have_prev, int n, const FieldChunk &f, int nsteps, double dt,
                              double *part, const SmallDeviation &dev, hipStream_t s) {
  if (g.norb == 4)
    return small_steps_form<4>(g, kpts, nk, spk, sinv, dlev0, dlev1, cur, have_prev, n, f, nsteps, dt,
                               part, dev, s);
  return small_steps_form<1>(g, kpts, nk, spk, sinv, dlev0, dlev1, cur, have_prev, n, f, nsteps, dt,
                             part, dev, s);
}

void launch_reduce_steps(const double *part, int nk, int na, const double *kw, double jscale,
                         double *hist, int64_t step0, int cap, int nsteps, int *flag,
                         const double *escc, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_steps, dim3(nsteps), dim3(kReduceThreads), 0, s, part, nk, na, kw,
                     jscale, hist, step0, cap, flag, escc);
}

void launch_hermitian_from_lower(double2 *m, int n, int nk, hipStream_t s) {
  dim3 grid(blocks_for(n, 16), blocks_for(n, 16), nk);
  hipLaunchKernelGGL(k_hermitian_from_lower, grid, dim3(16, 16), 0, s, m, n);
}

void launch_density_from_vectors(const double2 *evec, const double *occ, double2 *d, int n,
                                 int nk, hipStream_t s) {
  dim3 grid(blocks_for(n, 16), blocks_for(n, 16), nk);
  hipLaunchKernelGGL(k_density_from_vectors, grid, dim3(256), 0, s, evec, occ, d, n);
}

}  // namespace vgtb
