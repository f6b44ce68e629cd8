// Internal declarations of the gfx950 propagator: context layout and the
// host-side launchers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cstdint>
#include <string>
#include <vector>

#include "vgtb.h"

namespace vgtb {

constexpr double kLightSpeed = 137.035999084;


// Workgroup scheduling.  The dispatcher hands consecutive workgroup ids to the
// eight XCDs in turn, and each XCD has its own L2.  xcd_slot() renumbers a
// dispatch id so that each XCD receives a contiguous range of the logical
// index space (when the count divides by 8); grouped_tile() then walks the
// output tiles of one batch entry in blocks of gm row panels, column-major
// within a block, so the workgroups resident on one XCD share A row panels
// and B column panels in its L2.
// The power-of-two scale of the fp16 split: 2^e with m 2^e in [2^13, 2^14)
// for the largest |re|, |im| m; 1 for m zero or non-finite; e clamped to
// [-100, 100] (a float power of two).
__device__ inline float f16_pow2_scale(float m) {
  float sc = 1.0f;
  if (m > 0.0f && isfinite(m)) sc = ldexpf(1.0f, max(-100, min(100, 13 - ilogbf(m))));
  return sc;
}

// The constant S^-1 - I enters the bf16 split product as hi + lo, and the error
// of that representation (about 2^-17 relative) is the same at every step: it
// acts like a slightly different overlap and shifts the response frequencies.
// Its lo part is therefore stored kADither times with dithered rounding, and
// step n uses copy n mod kADither (odd, so that both leapfrog sublattices see
// every copy): copy j rounds |r| + d_j u to the bf16 grid, r the remainder
// after hi, u the grid step at |r|, d_j = (j + 1/2)/kADither - 1/2, so the
// copies average to r within u / (2 kADither).  The middle copy (d = 0) is the
// plain rounding; a remainder of zero stays zero.  Magnitude and sign are
// dithered separately, so the (j, i) copy of a Hermitian matrix stays the
// conjugate of the (i, j) one.  The scaled fp16 split carries 2^-22 and keeps
// one plainly rounded copy.
constexpr int kADither = 5;
__device__ inline double dither_offset(int level) {
  return ((double)level + 0.5) / (double)kADither - 0.5;
}

__device__ inline int xcd_slot(int lin, int total) {
  return (total & 7) == 0 ? (lin & 7) * (total >> 3) + (lin >> 3) : lin;
}
__device__ inline void grouped_tile(int tile, int tiles_m, int tiles_n, int gm, int &tm, int &tn) {
  const int per_group = gm * tiles_n;
  const int g = tile / per_group;
  const int first = g * gm;
  const int rows = min(gm, tiles_m - first);
  const int r = tile % per_group;
  tm = first + r % rows;
  tn = r / rows;
}

// Device view of the real-space blocks, grouped by atom pair (I, J): pairs
// of row atom I are row_ptr[I] .. row_ptr[I+1]-1, sorted by J; the periodic
// images of pair p are img_ptr[p] .. img_ptr[p+1]-1.
//
// Row groups of group_size consecutive atoms (4 or 8): group g's neighbour
// union is entries grp_ptr[g] .. grp_ptr[g+1]-1; entry e is atom ent_j[e]
// with bit il of ent_mask[e] set when atom g*group_size + il pairs with it; its pairs, in il
// order, are gp_pair[ent_pp[e] .. ent_pp[e+1]-1] (local atom gp_il[...]).
struct PairGraph {
  int n_atoms = 0, norb = 0, n_pairs = 0, n_images = 0;
  int group_size = 8, n_groups = 0, n_entries = 0;
  const int *grp_ptr = nullptr;   // n_groups + 1
  const int *ent_j = nullptr;     // n_entries
  const int *ent_mask = nullptr;  // n_entries
  const int *ent_pp = nullptr;    // n_entries + 1
  const int *gp_pair = nullptr;   // n_pairs
  const int *gp_il = nullptr;     // n_pairs
  const int *row_ptr = nullptr;   // n_atoms + 1
  const int *pair_col = nullptr;  // n_pairs
  const int *pair_row = nullptr;  // n_pairs (row atom I of pair p)
  const int *img_ptr = nullptr;   // n_pairs + 1
  const double *img_d = nullptr;  // n_images * 3
  const double *img_h0 = nullptr; // n_images * norb^2
  const double *img_s = nullptr;  // n_images * norb^2
  const double *img_ds = nullptr; // n_images * 3 * norb^2 (momentum coupling), or null
};

// A(t_n) / c.
struct StepField {
  double ax, ay, az;
};

// Where the per-step kernels find the step index and the field, so that every
// step's launches are identical (and can be captured once in a graph):
// ctr = device step counter (advanced by the update kernel), ring = A(t)/c of
// kStepRing consecutive steps at slot step mod kStepRing.  A null ring means
// A = 0, a null counter step 0.
constexpr int kStepRing = 64;
struct StepSource {
  const double *ring;
  const int64_t *ctr;
};

// Small systems: a block of up to kSmallChunk steps per launch, one workgroup
// per k with everything in LDS (N <= kSmallN, at most kSmallImages periodic
// images), in every precision form.  With the SCC shift the k-sum of the
// charges needs every k-point's partials each step: the launch is cooperative
// (at most kSmallSccMaxK workgroups, all resident) with a grid-wide barrier.
constexpr int kSmallN = 40;
constexpr int kSmallSccMaxK = 256;   // k-points (workgroups) of an SCC small-path launch, at most
constexpr int kSmallImages = 1536;
constexpr int kSmallChunk = 64;
struct FieldChunk {
  double a[3 * kSmallChunk];   // A(t_n) / c of the block's steps
};

// ---- launchers (kernels.hip) ------------------------------------------------
void launch_fill_zero(double2 *p, size_t n, hipStream_t s);
void launch_pair_bloch_s(const PairGraph &g, const double *kpts, int nk, double2 *spk,
                         hipStream_t s);
void launch_scatter_pairs(const PairGraph &g, const double *kpts, int nk, const double2 *spk,
                          int which, double2 *dense, int n, hipStream_t s);
// h0k / ppk (both null for the Peierls coupling): H0_k and P_k pair blocks of
// the momentum coupling.
void launch_observe(const PairGraph &g, const double2 *d, int n, const double *kpts, int nk,
                    StepSource src, const double2 *spk, const double2 *h0k, const double2 *ppk,
                    double *part, hipStream_t s);
// h0k[k][p][e] = sum_images exp(i k.d) H0, ppk[k][p][a][e] = sum_images exp(i k.d) i dS/dd^a.
void launch_pair_bloch_momentum(const PairGraph &g, const double *kpts, int nk, double2 *h0k,
                                double2 *ppk, hipStream_t s);
// ring slots of steps [step0, step0 + ns), ns <= kSmallChunk (= kStepRing).
void launch_store_ring(const FieldChunk &f, int64_t step0, int ns, double *ring, hipStream_t s);
void launch_set_counter(int64_t *ctr, int64_t v, hipStream_t s);
void launch_advance_counter(int64_t *ctr, hipStream_t s);   // *ctr += 1
// History row = hist + (step mod cap) (5 + na), step from ctr (row 0 if null).
void launch_reduce(const double *part, int nk, int na, const double *kw, double jscale,
                   const double *gamma, const double *z, double *v, double *qbuf,
                   double *rowpart, double *hist, int cap, const int64_t *ctr, int *flag,
                   hipStream_t s);
// Pair blocks of H_k(t) in grouped pair order.
void launch_assemble(const PairGraph &g, const double *kpts, int nk, StepSource src,
                     const double2 *spk, const double *v, double2 *hq, const double2 *h0k,
                     const double2 *ppk, hipStream_t s);
// W = H D (d0 == null) or W = H D - C0 (d0 != null marks the deviation form);
// out_format: 0 complex128, 1 complex64, 2 bf16 planes (k-packed, padded np)
// + complex64 copy w32, 3 fp16 planes of W wscale[k] + w32, with the largest
// |re|, |im| of each k-point raised into one of its kMaxSlots slots of wmax
// (float bits; zero them first).  variant: -1, -2, -4 = FP64 matrix cores with that
// many 16-column slices per wave (four orbitals per atom only); 1, 2 = vector
// FMAs with that many columns per thread.  ncols (0 = n): only the first
// ncols columns of W are formed (at least those; the rest are left as they were).
void launch_spmm(const PairGraph &g, const double2 *d, const double2 *d0, int n, int nk,
                 const double2 *hq, const double2 *c0, void *w, int out_format, int np,
                 float2 *w32, int variant, hipStream_t s, int ncols = 0,
                 const float *wscale = nullptr, unsigned *wmax = nullptr);
// ctr (may be null): advanced by one when the update has run.
void launch_update(const double2 *y, const double2 *dbase, double2 *dout, int n, int nk,
                   double fac, int64_t *ctr, hipStream_t s);
// D_out = D_base - i fac (Y - Y^dag) + fac m0 with Y = W + G (complex64 each,
// summed in FP64); m0 may be null.
void launch_update_split(const float2 *g, const float2 *w, const double2 *m0, const double2 *dbase,
                         double2 *dout, int n, int nk, double fac, int64_t *ctr, hipStream_t s);
// D_out = D_base - i (Y - Y^dag) (used to form the constant term m0 = -i X0).
void launch_update_const(const double2 *y, const double2 *dbase, double2 *dout, int n, int nk,
                         hipStream_t s);
// fmt 1: S^-1 - I as complex64; fmt 2: its bf16 hi/lo planes in kADither
// copies with dithered lo planes.
void launch_convert_operand(const double2 *src, void *dst, int n, int np, int nk, int fmt,
                            hipStream_t s);
// target[k] = Tr(D_k S_k) of the density dd.
void launch_trace_target(const PairGraph &g, const double2 *dd, int n, int nk, const double2 *spk,
                         double *tpart, double *target, hipStream_t s);
// Both levels: D <- (target / Tr(D S)) 1/2 (D + D^dag), per k.
void launch_rescale(const PairGraph &g, double2 *da, double2 *db, int n, int nk, const double2 *spk,
                    double *tpart, const double *target, double *fac, hipStream_t s);
// ---- spectrum (spectrum.hip) --------------------------------------------------
// Eqs. 15-16 of a host current trace through a device scratch of cap doubles
// (at least spectrum_min_scratch()): trace and frequency grid are streamed
// in chunks; sigma_host / eps_host (host, n_w complex128 each, either may be
// null) receive the results.  Synchronises s.
size_t spectrum_min_scratch();
// The message vgtb_last_error(NULL) returns on this thread (copied into a
// fixed buffer: no allocation).
void set_last_error(const char *m);
hipError_t spectrum_chunked(double *scratch, size_t cap, hipStream_t s, int64_t n_t,
                            const double *j_host, double dt, int64_t n_w, const double *omega_host,
                            double e0, double tau0, bool subtract_mean, void *sigma_host,
                            void *eps_host);
// The deviation (reduced-precision) forms on the small-system path: form 1
// FP32, 2 3xBF16, 3 FP16X3; 0 = the FP64 form (the rest unused).  c0 = H0 D0,
// m0 (may be null) the constant term of a set density, scale_a the per-k
// scale of S^-1 - I (FP16X3), trace0 the per-k target of the rescale every
// rescale_every steps (0 = never) counted from the context's step index step0.
//
// The SCC shift (Eq. 10) on the small path: gamma (na x na) and Z switch it on.
// Its Mulliken charges sum over all k-points, so every step waits at a
// grid-wide barrier (bar: arrival counter; the launch is cooperative, so all
// workgroups are resident) for the per-(k, atom) partials of that step; the
// wait is bounded, and a barrier that times out sets *err and ends the launch
// early.  escc[s] receives the SCC energy 1/2 dq^T gamma dq of block step s.
struct SmallDeviation {
  int form = 0;
  const double2 *c0 = nullptr, *m0 = nullptr;
  const float *scale_a = nullptr;
  const double *trace0 = nullptr;
  int rescale_every = 0;
  int64_t step0 = 0;
  const double *gamma = nullptr, *z = nullptr, *kw = nullptr;
  unsigned *bar = nullptr;
  unsigned bar_base = 0;
  int *err = nullptr;
  double *escc = nullptr;
};
// One system of a launch of several small systems: where its state, its block
// of field values and its history live, and its first workgroup in the launch.
struct SmallJob {
  PairGraph g;
  const double *kpts = nullptr;
  const double2 *spk = nullptr, *sinv = nullptr;
  double2 *dlev0 = nullptr, *dlev1 = nullptr;
  const double *field = nullptr;   // A(t_n)/c of the block's steps, three per step (device)
  double *part = nullptr;          // per-(step, k, atom) partials, as for one system
  SmallDeviation dev;
  const double *kw = nullptr;
  double jscale = 0.0, dt = 0.0;
  double *hist = nullptr;
  int64_t step0 = 0;
  int *flag = nullptr;
  int cap = 1, cur = 0, have_prev = 0, n = 0, nk = 0, na = 0, wg0 = 0;
};
// Steps of several small systems in one launch (one workgroup per system and
// k-point; wg_job maps workgroup to system), then their history rows.  All
// systems share orbitals per atom norb, the precision form and whether the
// SCC shift is on (then the launch is cooperative and n_wg is bounded by
// small_group_max_workgroups).  jobs and wg_job are device memory.
hipError_t launch_small_group(const SmallJob *jobs, const int *wg_job, int n_jobs, int n_wg, int norb,
                              int form, bool scc, int nsteps, hipStream_t s);
int small_group_max_workgroups(int norb, int form);
// C0 = H0_k D0 of the small path (its own assembly and LDS product).
void launch_small_c0(const PairGraph &g, const double *kpts, int nk, const double2 *d0, double2 *c0,
                     int n, hipStream_t s);
// Steps [step, step + nsteps) of a small system (see kSmallN); per-step
// partials [nsteps][nk][na][5] into part, then launch_reduce_steps.
// With the SCC shift the launch is cooperative; it returns its error (a grid
// too large to be resident at once is hipErrorCooperativeLaunchTooLarge).
hipError_t launch_small_steps(const PairGraph &g, const double *kpts, int nk, const double2 *spk,
                              const double2 *sinv, double2 *dlev0, double2 *dlev1, int cur,
                              bool have_prev, int n, const FieldChunk &f, int nsteps, double dt,
                              double *part, const SmallDeviation &dev, hipStream_t s);
// Largest k-point count the SCC small path can run (workgroups resident at once).
int small_scc_max_kpoints(int norb);
// escc (may be null): per-step SCC energy of the block, added to E.
void launch_reduce_steps(const double *part, int nk, int na, const double *kw, double jscale,
                         double *hist, int64_t step0, int cap, int nsteps, int *flag,
                         const double *escc, hipStream_t s);
void launch_hermitian_from_lower(double2 *m, int n, int nk, hipStream_t s);
void launch_density_from_vectors(const double2 *evec, const double *occ, double2 *d, int n,
                                 int nk, hipStream_t s);

// ---- launchers (crank_nicolson.hip) -----------------------------------------
// Coefficients C (nk * n * n, columns s < ns used), augmented [A | R] (nk * n * 2n),
// diagonal-block inverses inv (nk * kCnBlock^2).
constexpr int kCnBlock = 64;
void launch_cn_permute_pairs(const PairGraph &g, const double2 *spk, double2 *sq, int nk,
                             hipStream_t s);
void launch_cn_pattern(const PairGraph &g, const double2 *c, const double *occ, int n, int ns,
                       int nk, double2 *d, hipStream_t s);
void launch_cn_vmid(const double *v, double *vprev, double *vmid, int na, bool first,
                    hipStream_t s);
// [A | R]: A = S + i tau H on the pair pattern (zero elsewhere), R = W[:, :ns].
void launch_cn_build(const PairGraph &g, const double2 *w, const double2 *hq, const double2 *spk,
                     double tau, int n, int ns, int nk, double2 *aug, hipStream_t s);
// X = A^-1 R in the R columns of [A | R] (recursive block elimination); tile
// of the large products: 1 = 64 x 64, 2 = 128 x 64 (0 or other: 2), 3 = 128 x 128.
void launch_cn_solve(double2 *aug, double2 *inv, int n, int ns, int nk, int tile, hipStream_t s);
// C = 2 X - C with X the R columns; ctr (may be null) advanced by one.
void launch_cn_update(const double2 *aug, double2 *c, int n, int ns, int nk, int64_t *ctr,
                      hipStream_t s);
void launch_cn_from_vectors(const double2 *evec, double2 *c, int n, int ns, int nk, hipStream_t s);
void launch_cn_to_vectors(const double2 *c, double2 *evec, int n, int ns, int nk, hipStream_t s);
// C = beta C + alpha A B (M x K by K x N, row-major, per-batch strides).
void launch_zgemm_strided(const double2 *a, int lda, size_t sa, const double2 *b, int ldb,
                          size_t sb, double2 *c, int ldc, size_t sc, int m, int n, int k,
                          double alpha, bool beta_one, int batch, hipStream_t s);

// ---- launchers (gemm_mfma.hip, gemm_split16.hip) ------------------------------
// tile: workgroup tile shape (0 = the size rule; see the definitions).
void launch_zgemm_f64(const double2 *a, const double2 *b, double2 *c, int n, int batch,
                      hipStream_t s, int tile = 0);
void launch_cgemm_f32(const float2 *a, const float2 *b, float2 *c, int n, int batch,
                      hipStream_t s, int tile = 0);
// a holds kADither copies of the four planes of A (each 4 np^2 batch values);
// the product uses copy (*lev_ctr) mod kADither, the plainly rounded middle
// copy when lev_ctr is null.
void launch_cgemm_bf16x3(const uint16_t *a, const uint16_t *b, float2 *y, int n, int np, int batch,
                         hipStream_t s, int tile = 0, const int64_t *lev_ctr = nullptr);
// The same product on fp16 planes scaled per k by sa[k] (A, one copy) and
// sb[k] (B).
void launch_cgemm_f16x3(const uint16_t *a, const uint16_t *b, float2 *y, int n, int np, int batch,
                        const float *sa, const float *sb, hipStream_t s, int tile = 0);
// The 16-bit split product fused with the leapfrog update (fmt 2: bf16, 3:
// scaled fp16): G = (S^-1 - I) W into y for the tiles I <= J, and
// dout = dbase - i fac (Y - Y^dag) + fac m0 (m0 may be null) with Y = G + w,
// the same bits as launch_cgemm_* followed by launch_update_split; the copy of
// the bf16 A is chosen by ctr as there, and ctr (may be null) is then advanced by one
// (by a launch of its own, after the product).  Only for the 128 x 128 tiles
// (tile 2-5, or 0 where the size rule picks them); returns false, launching
// nothing, otherwise.
bool launch_cgemm_update_split16(int fmt, const uint16_t *a, const uint16_t *b, float2 *y,
                                 const float2 *w, const double2 *m0, const double2 *dbase,
                                 double2 *dout, int n, int np, int batch, double fac, int64_t *ctr,
                                 const float *sa, const float *sb, hipStream_t s, int tile);

// Tiles the size rule picks when no tile is given (tile 0): the FP64 / FP32
// complex product at size n, the 16-bit split product at padded size np.
int zgemm_default_tile(int n);
int split16_default_tile(int np);

// ---- launchers (split_f16.hip) ------------------------------------------------
// Power-of-two scale per k putting max(|re|, |im|) in [2^13, 2^14); part holds
// nk * f16_scale_parts() floats.
int f16_scale_parts();
void launch_f16_scale(const double2 *src, int n, int nk, bool minus_identity, float *part,
                      float *scale, hipStream_t s);
// Per-k maximum of W as the sparse product leaves it: kMaxSlots slots per
// k-point (float bits), kMaxStride words apart, so that the wavefronts' atomic
// maxima spread over many L2 lines instead of meeting on one address.
constexpr int kMaxSlots = 64, kMaxStride = 32;
// Sets scale[k] to the scale the maximum over k's slots of wmax calls for,
// flag[k] to whether it changed, and zeroes the slots.
void launch_f16_scale_check(unsigned *wmax, float *scale, int *flag, int nk, hipStream_t s);
// wmax slots = 0, scale = 1 for every k (before the first sparse product).
void launch_f16_scale_init(unsigned *wmax, float *scale, int nk, hipStream_t s);
// Scaled fp16 hi/lo planes: W in the product's k-packed B layout (only the
// k-points with flag[k] != 0 when flag is given), S^-1 - I row-major.
void launch_split_w_f16(const float2 *w, const float *scale, uint16_t *planes, int n, int np,
                        int nk, const int *flag, hipStream_t s);
void launch_split_a_f16(const double2 *sinv, const float *scale, uint16_t *planes, int n, int np,
                        int nk, hipStream_t s);

}  // namespace vgtb

struct vgtb_ctx {
  // sizes
  int na = 0, no = 0, n = 0, nk = 0;
  double volume = 0.0, n_electrons = 0.0, dt = 0.0;
  int precision = 0, rescale_every = 0, hist_cap = 1;
  int spmm_variant = -1;       // sparse-product kernel (see launch_spmm)
  int gemm_tile = 0;           // dense-product tile shape (0: size rule; vgtb_autotune)
  bool scc = false, z_from_ground_state = false;
  bool small_path = false;     // whole blocks of steps per launch (kSmallN)
  bool use_graphs = true;      // replay captured two-step graphs (general path)
  bool fuse_update = false;    // 16-bit split forms: product and update in one launch
                               // (on the 128 x 128 tiles)
  hipStream_t cap_stream = nullptr;            // private stream graphs are captured on
  hipGraphExec_t graph[2] = {nullptr, nullptr};  // two steps, by the parity of cur
  int64_t ring_lo = -1;        // first step whose field is in the ring (-1: none)
  int64_t ctr_step = 0;        // value the device counter has after the queued work

  hipStream_t stream = nullptr;
  rocblas_handle blas = nullptr;
  int device = 0;

  // host copies
  std::vector<double> kpts, kw, field;  // field: n_field * 3 (A, not A/c)
  std::vector<double> z_host;

  // device memory (carved from the caller's arena)
  vgtb::PairGraph g;
  double *kpts_dev = nullptr, *kw_dev = nullptr;
  double2 *spk = nullptr;      // nk * n_pairs * norb^2
  double2 *hq = nullptr;       // nk * n_pairs * norb^2, H_k pair blocks (grouped order)
  double2 *h0k = nullptr;      // momentum coupling: nk * n_pairs * norb^2, H0_k pair blocks
  double2 *ppk = nullptr;      // momentum coupling: nk * n_pairs * 3 * norb^2, P_k pair blocks
  double2 *c0 = nullptr;       // nk * n * n, H0_k(A=0) D0 (deviation forms)
  double2 *sinv = nullptr;     // nk * n * n
  double2 *dlev[2] = {nullptr, nullptr};
  double2 *d0 = nullptr;       // reference density (deviation forms)
  double2 *w = nullptr;        // nk * n * n
  double2 *y = nullptr;        // nk * n * n
  double *part = nullptr;      // nk * na * 5
  double *v = nullptr;         // na
  double *z = nullptr;         // na
  double *qbuf = nullptr;      // na
  double *rowpart = nullptr;   // na * 5 (per-atom shares of E, J, SCC energy)
  double *gamma = nullptr;     // na * na
  double *hist = nullptr;      // hist_cap * (5 + na)
  double *eig = nullptr;       // nk * n
  double *eig_e = nullptr;     // nk * n
  double *occ = nullptr;       // nk * n
  int *info = nullptr;         // nk
  int *flag = nullptr;         // 1
  // deviation (reduced-precision) forms
  int np = 0;                  // padded N of the bf16 planes
  void *sinv_lo = nullptr;     // S^-1 - I as complex64 (n), its 4 fp16 planes, or kADither copies of its 4 bf16 planes (np)
  void *w_lo = nullptr;        // W in the same format
  float2 *y_lo = nullptr;      // nk * n * n, G = (S^-1 - I) W
  float2 *w32 = nullptr;       // nk * n * n, W as complex64 (bf16 and fp16 forms; the fp32 form uses w_lo)
  float *scale_a = nullptr, *scale_w = nullptr;   // fp16 form: per-k scales of S^-1 - I and W
  float *scale_part = nullptr; // fp16 form: nk * f16_scale_parts() partial maxima
  unsigned *wmax = nullptr;    // fp16 form: per-k slots of the largest |re|, |im| of W (float bits)
  int *wflag = nullptr;        // fp16 form: per-k, W's scale changed at this step
  double *tpart = nullptr;     // 2 * nk * na
  double *tfac = nullptr;      // 2 * nk
  double *trace0 = nullptr;    // nk
  double *sm_part = nullptr;   // kSmallChunk * nk * na * 5 per-step partials (small path)
  unsigned *sm_bar = nullptr;  // small path with SCC: grid-barrier arrival counter
  int *sm_err = nullptr;       //   and its time-out flag
  double *sm_escc = nullptr;   //   kSmallChunk per-step SCC energies
  unsigned bar_count = 0;      //   arrivals so far (the next launch's base)
  double *ring = nullptr;      // kStepRing * 3, A(t)/c of the steps in flight
  int64_t *ctr = nullptr;      // device step counter
  double2 *m0 = nullptr;       // nk * n * n, -i (S^-1 H0 D0 - D0 H0 S^-1) for a set density
  bool m0_active = false;
  // Crank-Nicolson propagation of the coefficients (C in dlev[0], the sampled
  // density in dlev[1], S C in w)
  bool cn = false;
  int ns = 0;                  // coefficient vectors per k
  bool have_vprev = false;     // V_{n-1} of the SCC extrapolation is set
  double2 *aug = nullptr;      // nk * n * 2n, [S + i tau H | S C] and the solve
  double2 *cinv = nullptr;     // nk * kCnBlock^2, diagonal-block inverses
  double2 *sq = nullptr;       // nk * n_pairs * norb^2, S_k pair blocks (grouped order)
  double *cocc = nullptr;      // nk * n, occupations of the coefficient vectors
  double *vprev = nullptr, *vmid = nullptr;   // na each
  double *ring_mid = nullptr;  // kStepRing * 3, midpoint A/c of the steps in flight

  // per-kernel event timing (vgtb_profile_*)
  struct EvPair { int id; hipEvent_t a, b; };
  bool profiling = false;
  std::vector<EvPair> ev_pending;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;
  double prof_ms[VGTB_K_COUNT] = {0};
  int64_t prof_n[VGTB_K_COUNT] = {0};

  // propagation state
  int cur = 0;                 // dlev[cur] = D_n
  bool have_density = false, have_prev = false, poisoned = false;
  int64_t step = 0;
  std::string err;
};
