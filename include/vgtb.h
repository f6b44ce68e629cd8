/*
 * vgtb.h - C ABI of the MI355X (gfx950) velocity-gauge real-time TDDFTB
 * density-matrix propagator (Xu et al., arXiv 2308.09782).
 *
 * The library advances the k-dependent density matrices D_k of a periodic
 * tight-binding system under a spatially uniform vector potential A(t):
 *
 *   i dD_k/dt = S_k^-1 H_k D_k - D_k H_k S_k^-1                 (Eq. 6)
 *   D_k(t + dt) = D_k(t - dt) + 2 dt dD_k/dt(t)                 (Eq. 13)
 *
 * with S_k and H_k Bloch sums of real-space two-centre blocks (Eqs. 7-8),
 * the velocity-gauge coupling realised as the phase exp(i (k + A/c) . d) on
 * the H0 blocks, the self-consistent-charge shift of Eq. 10 from Mulliken
 * charges, and the current of Eq. 14.
 *
 * Conventions shared by every call:
 *   - Atomic units (bohr, hartree, atomic time); c = 137.035999084.
 *   - Complex matrices are complex128 (two doubles, real then imaginary),
 *     row-major, N x N per k-point, k-points consecutive: element (k, i, j)
 *     sits at offset (k * N + i) * N + j.  N = n_atoms * orbs_per_atom and
 *     orbital index i = atom * orbs_per_atom + (s, px, py, pz order).
 *   - Pointers named "host" are host memory; pointers named "dev" are device
 *     memory of the GPU that is current when vgtb_create is called.
 *   - Host inputs are copied; the caller keeps ownership of every pointer it
 *     passes.  The device arena passed to vgtb_create belongs to the caller,
 *     must outlive the context, and must not be touched while it is alive.
 *   - Every call returns a vgtb_status; no exception crosses the ABI.  After
 *     VGTB_E_DEVICE or VGTB_E_NONFINITE the context is poisoned: only
 *     vgtb_last_error and vgtb_destroy remain valid.
 *   - A context is not thread-safe; distinct contexts are independent.  All
 *     device work is queued on the stream given at creation.
 */
#ifndef VGTB_H
#define VGTB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vgtb_ctx vgtb_ctx;

typedef enum {
  VGTB_OK = 0,
  VGTB_E_INVAL = 1,      /* bad argument or inconsistent system description      */
  VGTB_E_STATE = 2,      /* call out of order (e.g. step before a density is set) */
  VGTB_E_NOT_PD = 3,     /* the Cholesky factorisation of some S_k failed          */
  VGTB_E_UNSTABLE = 4,   /* |dt| * (spectral width) >= 1: leapfrog would diverge  */
  VGTB_E_NOMEM = 5,      /* the arena is smaller than vgtb_workspace_size          */
  VGTB_E_DEVICE = 6,     /* a HIP / rocSOLVER call failed                          */
  VGTB_E_NONFINITE = 7   /* a non-finite trace was observed during stepping        */
} vgtb_status;

typedef enum {
  VGTB_FP64 = 0,   /* every product in FP64 on the FP64 matrix cores                       */
  VGTB_FP32 = 1,   /* deviation form, S^-1 (H D - H0 D0) product in FP32 on matrix cores   */
  VGTB_BF16X3 = 2, /* deviation form, the same product as three BF16 products (hi/lo split;
                      the lo part of the constant S^-1 - I dithered over five steps, held
                      in five copies)                                                       */
  VGTB_FP16X3 = 3  /* deviation form, three FP16 products of hi/lo splits scaled per k by
                      powers of two (same matrix-core rate, about 16x smaller product error) */
} vgtb_precision;

/*
 * Real-space description of one periodic system (paper Section 2, Eqs. 7-11).
 *
 * Block b couples the orbitals of atom blk_i[b] (rows) with those of the
 * periodic image of atom blk_j[b] (columns) whose bond vector is
 *   d_b = R_J + L - R_I                     (blk_d[3b..3b+2], bohr).
 * blk_h0 / blk_s hold the real orbs_per_atom^2 values of H0 and S of that
 * block, row-major.  On-site blocks have d = 0.  The list must contain, for
 * every block (I, J, d), the partner (J, I, -d) with the transposed values
 * (so that H_k and S_k are Hermitian); vgtb_create checks this.
 *
 * kpts are Cartesian (1/bohr), kw their weights (sum 1); every k-sum (the
 * charges, the energy and the current of Eq. 14, whose 1/N_k is the
 * equal-weight case) uses them.  n_electrons is the
 * electron count per k-point (f = 2 per state, Tr(D_k S_k) = n_electrons).
 * gamma (n_atoms^2, symmetric) switches on the SCC term of Eq. 10; NULL means
 * a non-SCC run.  z_ref is the per-atom reference charge Z_I of dq = q - Z;
 * NULL means "the Mulliken charges of the ground state" (set by
 * vgtb_ground_state), which makes the ground state self-consistent.
 */
typedef struct {
  int32_t n_atoms;
  int32_t orbs_per_atom;       /* 1 (s) or 4 (s, px, py, pz)                   */
  double cell[9];              /* lattice vectors as rows, bohr                 */
  int32_t n_blocks;
  const int32_t *blk_i;        /* host, n_blocks                                */
  const int32_t *blk_j;        /* host, n_blocks                                */
  const double *blk_d;         /* host, n_blocks * 3                            */
  const double *blk_h0;        /* host, n_blocks * orbs^2                       */
  const double *blk_s;         /* host, n_blocks * orbs^2                       */
  int32_t n_k;
  const double *kpts;          /* host, n_k * 3                                 */
  const double *kw;            /* host, n_k                                     */
  double n_electrons;          /* per k-point                                   */
  const double *z_ref;         /* host, n_atoms, or NULL                        */
  const double *gamma;         /* host, n_atoms * n_atoms, or NULL (non-SCC)   */
  const double *blk_ds;        /* host, n_blocks * 3 * orbs^2: dS/dd^alpha, the
                                  gradient of each overlap block with respect to
                                  its bond vector (= with respect to R_J), zero on
                                  site; partner blocks must satisfy
                                  dS(J,I,-d) = -dS(I,J,d)^T.  NULL unless the
                                  momentum coupling is used.                    */
} vgtb_system;

/*
 * How the vector potential enters H_k(t) (the SCC term, Eq. 10, is the same):
 *   PEIERLS:  H0 blocks with the phase exp(i (k + A/c).d), i.e. H0(k + A/c);
 *             current matrix Pi = dH0/dk at k + A/c.
 *   MOMENTUM: the paper's Eq. 12, H0_k + (1/c) A.P_k + |A|^2/(2c^2) S_k with
 *             P_k the Bloch sum of <phi_mu|p|phi_nu> = i dS/dR_J (needs
 *             vgtb_system.blk_ds); current matrix Pi = P_k + (A/c) S_k (the
 *             text after Eq. 14).  Not on the small-system path.
 */
typedef enum { VGTB_COUPLING_PEIERLS = 0, VGTB_COUPLING_MOMENTUM = 1 } vgtb_coupling;

/*
 * What is propagated (Section 2, Eqs. 5, 6 and 13):
 *   LEAPFROG:       the density matrices D_k by leapfrog on Eq. 6 (Eq. 13).
 *   CRANK_NICOLSON: the coefficient vectors C_nk of Eq. 5 by the unitary
 *                   Crank-Nicolson scheme the paper names beside it,
 *                   (S + i dt/2 H) C(t + dt) = (S - i dt/2 H) C(t), with H at
 *                   the midpoint: A = (A(t_n) + A(t_{n+1}))/2 and the SCC
 *                   shift extrapolated as (3 V_n - V_{n-1})/2.  The density
 *                   D_k = sum_n f_n C_nk C_nk^dag is formed on the pair
 *                   pattern for the observables.  FP64 only; the state is set
 *                   by vgtb_ground_state or vgtb_set_coefficients.
 */
typedef enum { VGTB_PROP_LEAPFROG = 0, VGTB_PROP_CRANK_NICOLSON = 1 } vgtb_propagator;

/* Bits of vgtb_options.flags. */
enum {
  VGTB_OPT_NO_GRAPHS = 1,      /* launch every step directly (no captured two-step
                                  graphs); same results bit for bit               */
  VGTB_OPT_NO_SMALL_PATH = 2,  /* no whole-steps-per-launch path for small
                                  systems (N <= 40, Peierls, leapfrog); same
                                  results to rounding.  With the SCC term that
                                  path is one cooperative launch whose workgroups
                                  (one per k-point, at most 256) meet at a
                                  grid-wide barrier every step: it needs them all
                                  resident at once, which kernels of other
                                  streams can prevent; its wait is bounded
                                  (VGTB_E_DEVICE after about a second), so set
                                  this flag for SCC contexts that share the GPU
                                  with concurrent work                           */
  VGTB_OPT_FUSE_UPDATE = 4     /* 3xBF16 / FP16X3 on 128x128 tiles: the dense
                                  product and the leapfrog update as one kernel over
                                  mirrored tile pairs instead of two launches; same
                                  results bit for bit (measured no faster)          */
};

/*
 * Options of one context.  Zero-initialise the struct, then set dt and
 * history_capacity: every other zero is the default.  The kernel choices (tile_override, spmm_variant,
 * spmm_group) change only how the terms of the products are grouped and
 * summed (results agree to rounding), never the method; vgtb_autotune can
 * choose them instead.  No process-wide setting
 * (environment variable, global) is read.
 */
typedef struct {
  double dt;                   /* time step (atomic time units), finite, nonzero */
  int32_t precision;           /* vgtb_precision                                 */
  int32_t rescale_every;       /* deviation forms: re-Hermitise and rescale the
                                  trace every this many steps (0 = never)        */
  int32_t history_capacity;    /* observables ring length in steps (>= 1)        */
  int32_t coupling;            /* vgtb_coupling                                  */
  int32_t propagator;          /* vgtb_propagator                                */
  int32_t tile_override;       /* dense product S^-1 W tile: 0 = size rule; FP64 and
                                  FP32: 1 = 32x32, 2 = 64x64, 3 = 128x64; 3xBF16 and
                                  FP16X3: 1 = 64x64, 2-5 = 128x128 with 16, 8 (64x32),
                                  8 (32x64) or 4 wavefronts (N padded to a multiple of
                                  128, else 64x64); Crank-Nicolson: the solve's large
                                  products, 1 = 64x64, 2 (0) = 128x64, 3 = 128x128   */
  int32_t spmm_variant;        /* sparse product W = H D: 0 = default (-1); -1, -2, -4
                                  = FP64 matrix cores with 1, 2, 4 16-column slices per
                                  wavefront (four orbitals per atom only); -11, -12,
                                  -14 = the same with three real products per complex
                                  one (Dr Hr, Di Hi, (Dr + Di)(Hr + Hi)); 1, 2 =
                                  vector FMAs with 1, 2 columns per thread (always the
                                  vector form for one orbital per atom)              */
  int32_t spmm_group;          /* atoms per row group of the sparse product: 0 (= 8),
                                  4, 8, or 16 (matrix-core variants only)            */
  int32_t flags;               /* VGTB_OPT_* bits                                   */
} vgtb_options;

/* Bytes of device arena vgtb_create needs for this system and options
 * (VGTB_E_INVAL for an invalid system or options, with the reason in
 * vgtb_last_error(NULL)). */
vgtb_status vgtb_workspace_size(const vgtb_system *sys, const vgtb_options *opt,
                                size_t *bytes);

/*
 * Validate the system, copy it to the device arena (dev_arena, arena_bytes,
 * 256-byte aligned), build S_k (Eq. 7) and S_k^-1 by a Cholesky
 * factorisation (VGTB_E_NOT_PD if some S_k is not positive definite), and
 * return a context bound to hip_stream (a hipStream_t; NULL = the null
 * stream).  The caller owns dev_arena and the stream.  *out is set only on
 * VGTB_OK.
 */
vgtb_status vgtb_create(const vgtb_system *sys, const vgtb_options *opt, void *dev_arena,
                        size_t arena_bytes, void *hip_stream, vgtb_ctx **out);

/*
 * Ground state at A = 0, the starting point of every run in Section 3 (the
 * field-free density before the kick or pulse), as the density matrix of the
 * definition after Eq. 6: solve H0_k C = S_k C eps for every k, fill states by
 * aufbau with f = 2 (a degenerate group straddling the Fermi level shares its
 * electrons equally), form D_k(0) = sum_n f_n c_n c_n^dag on the device and
 * make it the current density (step index 0).  If z_ref was NULL, the
 * Mulliken charges of this density become Z.  min_gap_host (may be NULL)
 * receives the smallest HOMO-LUMO gap over k.  Leapfrog contexts: returns
 * VGTB_E_UNSTABLE if |dt| times the largest spectral width over k is >= 1
 * (the density is still set).  Synchronises the stream.  A Crank-Nicolson context keeps the
 * occupied vectors C_nk (and their occupations) as its state instead.
 */
vgtb_status vgtb_ground_state(vgtb_ctx *ctx, double *min_gap_host);

/*
 * Initial condition of Eq. 6 given by the caller (for instance a perturbed or
 * excited density).  Set D_k(0) from n_k * N * N complex128 values (on_device != 0: device
 * pointer read on the context stream; else host).  Resets the step index to
 * 0 and forgets the previous level.  In the deviation forms this density
 * also becomes the reference D0 of the reduced-precision product.
 */
vgtb_status vgtb_set_density(vgtb_ctx *ctx, const void *d, int on_device);

/*
 * Crank-Nicolson contexts only (VGTB_E_STATE otherwise).  Set the state to
 * n_states coefficient vectors per k: c is n_k * N * n_states complex128,
 * element (k, i, s) at offset (k * N + i) * n_states + s (on_device != 0:
 * device pointer read on the context stream; else host); occ_host holds the
 * n_k * n_states occupations f_s (finite, >= 0).  1 <= n_states <= N.  Resets
 * the step index to 0.  vgtb_ground_state sets the occupied ground-state
 * vectors instead (n_states = the largest occupied count over k; a k-point
 * with fewer occupied states carries its next states with f = 0).
 */
vgtb_status vgtb_set_coefficients(vgtb_ctx *ctx, const void *c, const double *occ_host,
                                  int32_t n_states, int on_device);

/* Number of coefficient vectors per k of a Crank-Nicolson context (0 before a
 * state is set, -1 for a null or leapfrog context). */
int32_t vgtb_num_states(const vgtb_ctx *ctx);

/* Copy the current coefficients (layout as in vgtb_set_coefficients, device
 * or host) and, if occ_host is not NULL, the occupations.  Synchronises. */
vgtb_status vgtb_get_coefficients(vgtb_ctx *ctx, void *c_out, double *occ_host, int on_device);

/* The drive as the vector potential of Eq. 3, A(t) = -c int E dt (velocity
 * gauge): A(t_n) for n = 0 .. n-1, t_n = n dt (host, n * 3 doubles, atomic
 * units; copied).  A delta kick E0 delta(t) is the constant A = -c E0 from
 * t = 0; a laser pulse is its A(t) sampled on the step grid.  Steps past the
 * table's end use its last entry.  VGTB_E_INVAL for n < 1 or a non-finite
 * entry (the table in use is then unchanged). */
vgtb_status vgtb_set_field_table(vgtb_ctx *ctx, int64_t n, const double *a_host);

/* A constant vector potential (Eq. 3) from the next step on: a one-entry
 * table, as for a delta kick. */
vgtb_status vgtb_set_field(vgtb_ctx *ctx, const double a_host[3]);

/*
 * The time propagation: queue n_steps leapfrog steps (Eq. 13 applied to
 * Eq. 6) on the context stream (asynchronous).  Step n uses A(t_n),
 * evaluates the SCC shift of Eq. 10 from the Mulliken charges of D_n,
 * records the observables of D_n (current of Eq. 14, energy, Tr(D S),
 * charges) in the history ring, assembles H_k(t_n) from the blocks (Eqs. 8-9,
 * or Eq. 12 in the momentum coupling), then forms D_{n+1} (the first step
 * after a density is set is a forward Euler step).  VGTB_E_STATE before a
 * density is set; VGTB_E_INVAL for n_steps < 0; a non-finite trace is
 * reported by the next vgtb_synchronize.  Deviation forms
 * re-Hermitise and rescale the trace of both levels after every
 * rescale_every-th step.  A Crank-Nicolson context records the observables of
 * C_n with A(t_n), then solves for C_{n+1} (vgtb_propagator).
 */
vgtb_status vgtb_step(vgtb_ctx *ctx, int64_t n_steps);

/* Wait for the stream; VGTB_E_NONFINITE if any recorded trace was not finite. */
vgtb_status vgtb_synchronize(vgtb_ctx *ctx);

/*
 * Copy observables of steps [first, first + count) to host arrays (each may
 * be NULL): J count*3 (Eq. 14, bohr^-2 a.u. current density), E count (band
 * + SCC energy per cell), trace count (sum_k w_k Re Tr(D_k S_k)), q
 * count*n_atoms (Mulliken charges).  Those steps must still be in the ring.
 * Synchronises the stream.
 */
vgtb_status vgtb_read_observables(vgtb_ctx *ctx, int64_t first, int64_t count, double *j_host,
                                  double *e_host, double *trace_host, double *q_host);

/* Copy D at level 0 (= D_n, current) or 1 (= D_{n-1}) to out (device or
 * host), n_k * N * N complex128.  Synchronises the stream.  A Crank-Nicolson
 * context has level 0 only: D = sum_s f_s C_s C_s^dag, formed on the device. */
vgtb_status vgtb_get_density(vgtb_ctx *ctx, int32_t level, void *out, int on_device);

/* Reference charges Z in use (host, n_atoms doubles). */
vgtb_status vgtb_get_reference_charges(vgtb_ctx *ctx, double *z_host);

/* Checkpoint: bytes needed, save both leapfrog levels, the reference density
 * and the step index to host memory, and restore them (Crank-Nicolson: the
 * coefficients, occupations and previous SCC shift).  Resuming continues
 * bit-identically to an uninterrupted run. */
vgtb_status vgtb_state_size(const vgtb_ctx *ctx, size_t *bytes);
vgtb_status vgtb_save_state(vgtb_ctx *ctx, void *host_buf, size_t bytes);
vgtb_status vgtb_load_state(vgtb_ctx *ctx, const void *host_buf, size_t bytes);

/* Steps taken since the density was set. */
int64_t vgtb_step_index(const vgtb_ctx *ctx);

/* Last error message of this context (NUL-terminated, owned by the context;
 * ctx may be NULL for errors raised before a context existed). */
const char *vgtb_last_error(const vgtb_ctx *ctx);

void vgtb_destroy(vgtb_ctx *ctx);

/*
 * Several small systems in one launch.  The paper distributes k-points over
 * processes (Section 3); a small system (N <= 40) has too few k-points to
 * fill a GPU, so a group steps many contexts together: each block of up to
 * 64 steps is one launch with one workgroup per (system, k-point), followed
 * by one launch that writes every system's history rows.  Each system
 * follows exactly the steps vgtb_step takes for it (Eqs. 6 and 13, the SCC
 * shift of Eq. 10 from its own charges, its own field table, dt and
 * rescale cadence), with the same arithmetic, so its state and history are
 * the same as when it is stepped alone.
 *
 * vgtb_group_create: ctxs[0..n_ctx) (1 to 4096 distinct contexts, not
 * copied; the caller keeps them alive until vgtb_group_destroy) must all be
 * on the small-system path (VGTB_K_SMALL), on one device, with the same
 * orbitals per atom, precision form and SCC setting (VGTB_E_INVAL
 * otherwise).  With the SCC term the group's launches are cooperative and the
 * systems' k-points together must fit on the GPU at once (one workgroup per
 * compute unit: 256 on MI355X), VGTB_E_INVAL beyond.  The group allocates a
 * small pinned host buffer and its device copy (four blocks of per-system
 * arguments and field values).
 *
 * vgtb_group_step: queues n_steps steps of every system on the first
 * context's stream, after the work already queued on every context's stream
 * and before any work queued on them later (events join the streams).
 * VGTB_E_STATE if a context has no density or is poisoned; a launch failure
 * poisons every context of the group (VGTB_E_DEVICE).  Observables and
 * densities are read per context as usual.  The group's launches are not
 * recorded in the contexts' profiles.  Errors are reported through
 * vgtb_last_error(NULL).
 */
typedef struct vgtb_group vgtb_group;
vgtb_status vgtb_group_create(vgtb_ctx *const *ctxs, int32_t n_ctx, vgtb_group **out);
vgtb_status vgtb_group_step(vgtb_group *grp, int64_t n_steps);
void vgtb_group_destroy(vgtb_group *grp);

/*
 * Serving: several propagations overlapped on one GPU.
 *
 * A server owns a caller-provided device arena (dev_arena, arena_bytes; the
 * caller keeps it alive until vgtb_server_destroy; 256-byte aligned) and
 * max_active slots (1..64), each a HIP stream the server creates.
 *
 * vgtb_server_run(srv, n, requests, stats, summary) serves n requests and
 * returns when all have finished or failed.  Request i arrives arrival_s
 * seconds after the call starts.  Waiting requests are admitted first come
 * first served when a slot is free and their workspace (vgtb_workspace_size,
 * with the history capacity raised to n_steps) fits in the free part of the
 * arena (first fit); a request larger than the whole arena fails with
 * VGTB_E_NOMEM.  An admitted request is initialised on a worker thread
 * (S_k^-1 and the ground state, the field-free starting point of Section 3;
 * the field table), then stepped in chunks on its own stream, so the kernels
 * of all running requests overlap (its context launches every step directly,
 * VGTB_OPT_NO_GRAPHS).
 * When its n_steps are done, J(t) (n_steps x 3, host j_out, may be NULL) and
 * sigma(omega) of the x current (Eqs. 15-16 with e0 and tau0, n_omega complex
 * values, host sigma_out, may be NULL) are written, and its slot and arena
 * range are released.  The request's system, field table and omega grid must
 * stay valid until the call returns.  stats (n entries) and summary may be
 * NULL.  Results do not depend on the other requests.  A failing request
 * (invalid, too large, a failed initialisation or step) gets its own status
 * and message in stats; the others go on.  The call returns VGTB_OK once every
 * request has finished or failed (VGTB_E_INVAL for a null server or requests).
 */
typedef struct vgtb_server vgtb_server;

typedef struct {
  const vgtb_system *system;
  vgtb_options options;          /* history_capacity is raised to n_steps          */
  int64_t n_steps;
  int64_t n_field;               /* A(t_n), n_field x 3 doubles (host)             */
  const double *field;
  int32_t n_omega;               /* spectrum grid (host), may be 0                 */
  const double *omega;
  double e0, tau0;               /* Eq. 15 normalisation and damping time          */
  double arrival_s;
  double *j_out;                 /* host, n_steps x 3, may be NULL                 */
  double *sigma_out;             /* host, n_omega complex128, may be NULL          */
} vgtb_request;

typedef struct {
  vgtb_status status;
  int32_t slot;                  /* -1 if never admitted                           */
  size_t workspace_bytes;
  double arrival_s, admitted_s, ready_s, finished_s;   /* seconds on the run clock */
  char message[128];             /* why the request failed (NUL-terminated; empty
                                    when status is VGTB_OK)                       */
} vgtb_request_stats;

typedef struct {
  double makespan_s;             /* from the call to the last completion           */
  double k_steps;                /* sum of n_k * n_steps of the finished requests  */
  double k_steps_per_s;          /* k_steps / makespan_s                           */
  size_t peak_bytes;             /* most arena bytes in use at once                */
  int32_t peak_active;           /* most requests admitted at once                 */
} vgtb_server_stats;

vgtb_status vgtb_server_create(void *dev_arena, size_t arena_bytes, int32_t max_active,
                               vgtb_server **out);
vgtb_status vgtb_server_run(vgtb_server *srv, int32_t n, const vgtb_request *requests,
                            vgtb_request_stats *stats_host, vgtb_server_stats *summary_host);
void vgtb_server_destroy(vgtb_server *srv);

/* Kernel classes of one step, for vgtb_profile_read. */
typedef enum {
  VGTB_K_OBSERVE = 0,   /* Mulliken / energy / current sweep of D_n            */
  VGTB_K_REDUCE = 1,    /* k-sum, SCC shift, history row                       */
  VGTB_K_SPMM = 2,      /* block-sparse W = H D (deviation forms: H D - H0 D0) */
  VGTB_K_GEMM = 3,      /* dense Y = S^-1 W on the matrix cores (all k)        */
  VGTB_K_UPDATE = 4,    /* leapfrog D_{n+1} = D_{n-1} - 2 i dt (Y - Y^dag)     */
  VGTB_K_RESCALE = 5,   /* deviation forms: re-Hermitise + trace rescale       */
  VGTB_K_ASSEMBLE = 6,  /* Peierls assembly of the pair blocks of H_k(t)       */
  VGTB_K_SMALL = 7,     /* small N (<= 40), Peierls, leapfrog, any precision
                           form, with or without SCC: up to 64 whole steps in
                           one launch (the other classes then stay at zero
                           except REDUCE, which is the per-block history
                           reduction)                                          */
  VGTB_K_CN_PATTERN = 8, /* Crank-Nicolson: D = sum f C C^dag on the pair pattern */
  VGTB_K_CN_SOLVE = 9,  /* Crank-Nicolson: [S + i dt/2 H | S C] build and the
                           recursive block elimination (leaf-block inverses +
                           GEMMs)                                               */
  VGTB_K_CN_UPDATE = 10, /* Crank-Nicolson: C(t + dt) = 2 X - C(t)             */
  VGTB_K_COUNT = 11
} vgtb_kernel;

/*
 * Autotuning of the kernel variants of the per-step path.
 *
 * Times, on this context's own buffers and stream, every candidate of
 *   - the block-sparse product W = H D: FP64 matrix cores with 1, 2 or 4
 *     16-column slices per wavefront, four real products per complex one
 *     (variant -1, -2, -4) or three (variant -11, -12, -14; four orbitals per
 *     atom), or vector FMAs with 1 or 2 columns per thread (variant 1, 2;
 *     row groups of at most 8 atoms);
 *   - the dense product S^-1 W: workgroup tiles 1 = 32x32, 2 = 64x64,
 *     3 = 128x64 (FP64 and FP32 forms); 1 = 64x64, and 128x128 as 2 = 16
 *     wavefronts of 32x32, 3 = 8 of 64x32, 4 = 8 of 32x64, 5 = 4 of 64x64
 *     (3xBF16 and FP16X3; the 128x128 shapes when the padded size is a
 *     multiple of 128),
 * after one warm-up launch of each, in `reps` interleaved rounds (every
 * candidate once per round, each launch between its own events), and keeps
 * the fastest of each kernel by the mean over rounds for the following steps;
 * the current choice is kept unless another is at least 1% faster.  Only
 * scratch buffers are written: the densities, history and step index are
 * unchanged; in the deviation forms the constant H0 D0 is formed again with a
 * newly chosen sparse product.  The variants agree to rounding.  Needs a density (VGTB_E_STATE otherwise), reps >= 1
 * (VGTB_E_INVAL).  out_host may be NULL.  Synchronises the stream.  For a
 * context on the small-system path (whole steps per launch) or with the
 * Crank-Nicolson propagator nothing is timed (n_spmm = n_gemm = 0).
 */
typedef struct {
  int32_t spmm_variant;          /* chosen sparse-product variant               */
  int32_t gemm_tile;             /* chosen dense-product tile (0: size rule)    */
  int32_t n_spmm, n_gemm;        /* number of candidates timed                  */
  int32_t spmm_candidates[8];
  double spmm_ms[8];             /* average launch time of each candidate (ms)  */
  int32_t gemm_candidates[8];
  double gemm_ms[8];
} vgtb_tuning;

vgtb_status vgtb_autotune(vgtb_ctx *ctx, int32_t reps, vgtb_tuning *out_host);

/*
 * Per-kernel timing with HIP events recorded on the context stream around
 * every launch of vgtb_step while enabled (enable != 0).  Enabling clears
 * the totals.  vgtb_profile_read synchronises the stream and returns the
 * summed device time (ms) and the number of launches of one kernel class.
 */
vgtb_status vgtb_profile_enable(vgtb_ctx *ctx, int enable);
vgtb_status vgtb_profile_read(vgtb_ctx *ctx, int32_t kernel, double *total_ms_host,
                              int64_t *launches_host);

/*
 * Spectrum of a delta-kick run (paper Eqs. 15-16), on the device:
 *   sigma(w) = (1/E0) int_0^T exp(i w t) (J(t) - <J>) exp(-t / tau0) dt
 *   epsilon(w) = 1 + 4 pi i sigma(w) / w
 * with the trapezoid rule on t_n = n dt.  j_host: n_t samples of one current
 * component; omega_host: n_w frequencies (nonzero); e0 the kick field
 * (E0 = -A0 / c for A(t) = A0 from t = 0); subtract_mean != 0 removes the mean
 * current first.  sigma_host / eps_host (either may be NULL) receive n_w
 * complex128 values.  Synchronous; uses the context's stream and scratch.
 */
vgtb_status vgtb_spectrum(vgtb_ctx *ctx, int64_t n_t, const double *j_host, double dt,
                          int64_t n_w, const double *omega_host, double e0, double tau0,
                          int subtract_mean, void *sigma_host, void *eps_host);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid hipMalloc): vgtb_spectrum without a
 * context and without any allocation.  The same arithmetic and arguments as
 * vgtb_spectrum; work is queued on hip_stream (a hipStream_t; NULL = the null
 * stream) of the current device, and the call returns when sigma_host and
 * eps_host (either may be NULL) hold the n_w results.
 * Scratch: a fixed 1 MiB array in the library's device image, one per GPU,
 * kept until the process ends; the trace and the grid stream through it, so
 * the limits are those of vgtb_spectrum: 2 <= n_t <= 2^30, 1 <= n_w <= 2^24
 * (VGTB_E_INVAL beyond them, message in vgtb_last_error(NULL)).  Calls on one
 * GPU share the array: calls that overlap in time on one GPU (from several
 * threads) race and must be serialised by the caller.
 */
vgtb_status vgtb_spectrum_noalloc(int64_t n_t, const double *j_host, double dt, int64_t n_w,
                                  const double *omega_host, double e0, double tau0,
                                  int subtract_mean, void *sigma_host, void *eps_host,
                                  void *hip_stream);

/*
 * Stand-alone kernel entry: C = A * B for `batch` row-major N x N complex128
 * matrices (strides N*N), on the FP64 matrix cores - the dense product
 * S_k^-1 (H_k D_k) of Eq. 6.  Device pointers, queued on hip_stream.
 */
vgtb_status vgtb_zgemm(const void *a_dev, const void *b_dev, void *c_dev, int32_t n, int32_t batch,
                       void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* VGTB_H */
