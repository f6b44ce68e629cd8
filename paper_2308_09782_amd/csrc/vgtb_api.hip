// C ABI of the propagator: validation, device arena layout, initialisation
// (S_k, S_k^-1, ground state) and the per-step launch sequence.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "vgtb_internal.h"

using vgtb::PairGraph;

namespace {

// Message of the last error raised before a context existed (per thread; a
// fixed buffer, so that setting it never allocates).
thread_local char g_global_err[512];
void set_global_err(const char *m) {
  size_t i = 0;
  for (; m && m[i] && i + 1 < sizeof(g_global_err); ++i) g_global_err[i] = m[i];
  g_global_err[i] = '\0';
}

vgtb_status fail(vgtb_ctx *ctx, vgtb_status st, const std::string &msg) {
  if (ctx) {
    ctx->err = msg;
    if (st == VGTB_E_DEVICE || st == VGTB_E_NONFINITE) ctx->poisoned = true;
  } else {
    set_global_err(msg.c_str());
  }
  return st;
}

#define HIP_TRY(ctx, expr)                                                                 \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess)                                                                  \
      return fail(ctx, VGTB_E_DEVICE, std::string(#expr " failed: ") + hipGetErrorString(_e)); \
  } while (0)

#define BLAS_TRY(ctx, expr)                                                                \
  do {                                                                                     \
    rocblas_status _s = (expr);                                                            \
    if (_s != rocblas_status_success)                                                      \
      return fail(ctx, VGTB_E_DEVICE,                                                      \
                  std::string(#expr " failed: ") + rocblas_status_to_string(_s));          \
  } while (0)

// ---------------------------------------------------------------------------
// Host-side pair graph: group the real-space blocks by (I, J).
// ---------------------------------------------------------------------------
struct HostGraph {
  int na = 0, norb = 0;
  std::vector<int> row_ptr, pair_col, pair_row, img_ptr;
  std::vector<double> img_d, img_h0, img_s, img_ds;
  std::vector<int> grp_ptr, ent_j, ent_mask, ent_pp, gp_pair, gp_il;
};

// Kernel choices of a context, from its options (no process-wide state).
// Sparse product W = H D: spmm_variant -1, -2, -4 = FP64 matrix cores with
// that many 16-column slices per wavefront (four orbitals per atom), -11,
// -12, -14 = the same with three real products per complex one, 1 or 2 =
// vector FMAs with that many columns per thread; 0 = -1 (the vector form is
// always used for one orbital per atom).  spmm_group: atoms per row group,
// 4 or 8 (0 = 8), or 16 with the matrix-core variants.
int spmm_variant_of(const vgtb_options *o) { return o->spmm_variant == 0 ? -1 : o->spmm_variant; }
int spmm_group_of(const vgtb_options *o) { return o->spmm_group == 0 ? 8 : o->spmm_group; }

// Row groups of G consecutive atoms and the union of their neighbours.
void build_groups(HostGraph &hg, int G) {
  const int ng = (hg.na + G - 1) / G;
  hg.grp_ptr.assign(1, 0);
  hg.ent_pp.assign(1, 0);
  for (int g = 0; g < ng; ++g) {
    std::map<int, std::vector<std::pair<int, int>>> by_j;   // J -> (il, pair)
    for (int il = 0; il < G && g * G + il < hg.na; ++il) {
      const int I = g * G + il;
      for (int p = hg.row_ptr[I]; p < hg.row_ptr[I + 1]; ++p) by_j[hg.pair_col[p]].push_back({il, p});
    }
    for (auto &kv : by_j) {
      int mask = 0;
      for (auto &ip : kv.second) {
        mask |= 1 << ip.first;
        hg.gp_pair.push_back(ip.second);
        hg.gp_il.push_back(ip.first);
      }
      hg.ent_j.push_back(kv.first);
      hg.ent_mask.push_back(mask);
      hg.ent_pp.push_back((int)hg.gp_pair.size());
    }
    hg.grp_ptr.push_back((int)hg.ent_j.size());
  }
}

vgtb_status build_graph(const vgtb_system *s, const vgtb_options *o, HostGraph &hg,
                        std::string &msg) {
  const int na = s->n_atoms, no = s->orbs_per_atom, nb = s->n_blocks;
  const int e2 = no * no;
  std::vector<int> order(nb);
  std::iota(order.begin(), order.end(), 0);
  for (int b = 0; b < nb; ++b) {
    if (s->blk_i[b] < 0 || s->blk_i[b] >= na || s->blk_j[b] < 0 || s->blk_j[b] >= na) {
      msg = "block " + std::to_string(b) + " refers to an atom outside [0, n_atoms)";
      return VGTB_E_INVAL;
    }
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(s->blk_d[3 * b + c])) {
        msg = "non-finite bond vector in block " + std::to_string(b);
        return VGTB_E_INVAL;
      }
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (s->blk_i[a] != s->blk_i[b]) return s->blk_i[a] < s->blk_i[b];
    return s->blk_j[a] < s->blk_j[b];
  });
  // Hermitian partner check: (I, J, d) needs (J, I, -d) with transposed values.
  auto key = [&](int i, int j, const double *d) {
    return std::make_tuple(i, j, std::llround(d[0] * 1e6), std::llround(d[1] * 1e6),
                           std::llround(d[2] * 1e6));
  };
  std::map<std::tuple<int, int, long long, long long, long long>, int> index;
  for (int b = 0; b < nb; ++b) {
    auto k = key(s->blk_i[b], s->blk_j[b], s->blk_d + 3 * b);
    if (!index.emplace(k, b).second) {
      msg = "duplicate block (same atoms and bond vector) at index " + std::to_string(b);
      return VGTB_E_INVAL;
    }
  }
  for (int b = 0; b < nb; ++b) {
    const double nd[3] = {-s->blk_d[3 * b], -s->blk_d[3 * b + 1], -s->blk_d[3 * b + 2]};
    auto it = index.find(key(s->blk_j[b], s->blk_i[b], nd));
    if (it == index.end()) {
      msg = "block " + std::to_string(b) + " has no Hermitian partner (J, I, -d)";
      return VGTB_E_INVAL;
    }
    const int c = it->second;
    for (int mu = 0; mu < no; ++mu)
      for (int nu = 0; nu < no; ++nu) {
        const double h1 = s->blk_h0[(size_t)b * e2 + mu * no + nu];
        const double h2 = s->blk_h0[(size_t)c * e2 + nu * no + mu];
        const double s1 = s->blk_s[(size_t)b * e2 + mu * no + nu];
        const double s2 = s->blk_s[(size_t)c * e2 + nu * no + mu];
        if (!(std::fabs(h1 - h2) <= 1e-12 * (1.0 + std::fabs(h1))) ||
            !(std::fabs(s1 - s2) <= 1e-12 * (1.0 + std::fabs(s1)))) {
          msg = "block " + std::to_string(b) + " is not the transpose of its partner";
          return VGTB_E_INVAL;
        }
        if (s->blk_ds)
          for (int a = 0; a < 3; ++a) {
            const double g1 = s->blk_ds[((size_t)b * 3 + a) * e2 + mu * no + nu];
            const double g2 = s->blk_ds[((size_t)c * 3 + a) * e2 + nu * no + mu];
            if (!std::isfinite(g1) || !(std::fabs(g1 + g2) <= 1e-12 * (1.0 + std::fabs(g1)))) {
              msg = "overlap gradient of block " + std::to_string(b) + " is not minus the transpose of its partner's";
              return VGTB_E_INVAL;
            }
          }
      }
  }
  hg.na = na;
  hg.norb = no;
  hg.row_ptr.assign(na + 1, 0);
  int prev_i = -1, prev_j = -1;
  for (int t = 0; t < nb; ++t) {
    const int b = order[t];
    const int i = s->blk_i[b], j = s->blk_j[b];
    if (i != prev_i || j != prev_j) {
      hg.pair_col.push_back(j);
      hg.pair_row.push_back(i);
      hg.img_ptr.push_back((int)(hg.img_d.size() / 3));
      hg.row_ptr[i + 1] += 1;
      prev_i = i;
      prev_j = j;
    }
    for (int c = 0; c < 3; ++c) hg.img_d.push_back(s->blk_d[3 * b + c]);
    for (int e = 0; e < e2; ++e) {
      hg.img_h0.push_back(s->blk_h0[(size_t)b * e2 + e]);
      hg.img_s.push_back(s->blk_s[(size_t)b * e2 + e]);
    }
    if (s->blk_ds)
      for (int e = 0; e < 3 * e2; ++e) hg.img_ds.push_back(s->blk_ds[(size_t)b * 3 * e2 + e]);
  }
  hg.img_ptr.push_back((int)(hg.img_d.size() / 3));
  for (int i = 0; i < na; ++i) hg.row_ptr[i + 1] += hg.row_ptr[i];
  for (int i = 0; i < na; ++i)
    if (hg.row_ptr[i + 1] == hg.row_ptr[i]) {
      msg = "atom " + std::to_string(i) + " has no blocks (an on-site block is required)";
      return VGTB_E_INVAL;
    }
  build_groups(hg, spmm_group_of(o));
  return VGTB_OK;
}

vgtb_status validate(const vgtb_system *s, const vgtb_options *o, std::string &msg) {
  if (!s || !o) { msg = "null system or options"; return VGTB_E_INVAL; }
  if (s->n_atoms <= 0) { msg = "n_atoms must be positive"; return VGTB_E_INVAL; }
  if (s->orbs_per_atom != 1 && s->orbs_per_atom != 4) {
    msg = "orbs_per_atom must be 1 or 4";
    return VGTB_E_INVAL;
  }
  const long long n = (long long)s->n_atoms * s->orbs_per_atom;
  if (n > 16384) { msg = "N = n_atoms * orbs_per_atom must be <= 16384"; return VGTB_E_INVAL; }
  if (s->n_blocks <= 0 || !s->blk_i || !s->blk_j || !s->blk_d || !s->blk_h0 || !s->blk_s) {
    msg = "missing block arrays";
    return VGTB_E_INVAL;
  }
  if (s->n_k <= 0 || !s->kpts || !s->kw) { msg = "missing k-points"; return VGTB_E_INVAL; }
  double wsum = 0.0;
  for (int k = 0; k < s->n_k; ++k) wsum += s->kw[k];
  if (std::fabs(wsum - 1.0) > 1e-10) { msg = "k-point weights must sum to 1"; return VGTB_E_INVAL; }
  double vol = 0.0;
  {
    const double *c = s->cell;
    vol = c[0] * (c[4] * c[8] - c[5] * c[7]) - c[1] * (c[3] * c[8] - c[5] * c[6]) +
          c[2] * (c[3] * c[7] - c[4] * c[6]);
  }
  if (!(std::fabs(vol) > 0.0) || !std::isfinite(vol)) { msg = "degenerate cell"; return VGTB_E_INVAL; }
  if (!std::isfinite(o->dt) || o->dt == 0.0) { msg = "dt must be finite and nonzero"; return VGTB_E_INVAL; }
  if (o->precision < VGTB_FP64 || o->precision > VGTB_FP16X3) {
    msg = "unknown precision";
    return VGTB_E_INVAL;
  }
  if (o->history_capacity < 1) { msg = "history_capacity must be >= 1"; return VGTB_E_INVAL; }
  if (o->rescale_every < 0) { msg = "bad options"; return VGTB_E_INVAL; }
  if (o->coupling != VGTB_COUPLING_PEIERLS && o->coupling != VGTB_COUPLING_MOMENTUM) {
    msg = "unknown coupling";
    return VGTB_E_INVAL;
  }
  if (o->propagator != VGTB_PROP_LEAPFROG && o->propagator != VGTB_PROP_CRANK_NICOLSON) {
    msg = "unknown propagator";
    return VGTB_E_INVAL;
  }
  if (o->tile_override < 0 || o->tile_override > (o->precision >= VGTB_BF16X3 ? 5 : 3)) {
    msg = "tile_override must be 0 (default), 1-3 (FP64, FP32, Crank-Nicolson) or 1-5 (3xBF16, FP16X3)";
    return VGTB_E_INVAL;
  }
  {
    const int v = o->spmm_variant, g = o->spmm_group;
    if (v != 0 && v != -1 && v != -2 && v != -4 && v != -11 && v != -12 && v != -14 && v != 1 && v != 2) {
      msg = "spmm_variant must be 0, -1, -2, -4, -11, -12, -14 (matrix cores) or 1, 2 (vector FMAs)";
      return VGTB_E_INVAL;
    }
    if (v < 0 && s->orbs_per_atom != 4) {
      msg = "the matrix-core sparse product needs four orbitals per atom";
      return VGTB_E_INVAL;
    }
    if (g != 0 && g != 4 && g != 8 && g != 16) { msg = "spmm_group must be 0, 4, 8 or 16"; return VGTB_E_INVAL; }
    if (g == 16 && (v > 0 || s->orbs_per_atom != 4)) {
      msg = "row groups of 16 atoms need the matrix-core sparse product";
      return VGTB_E_INVAL;
    }
  }
  if ((o->flags & ~(VGTB_OPT_NO_GRAPHS | VGTB_OPT_NO_SMALL_PATH | VGTB_OPT_FUSE_UPDATE)) != 0) {
    msg = "unknown option flags";
    return VGTB_E_INVAL;
  }
  if (o->propagator == VGTB_PROP_CRANK_NICOLSON && o->precision != VGTB_FP64) {
    msg = "the Crank-Nicolson propagator is FP64 only";
    return VGTB_E_INVAL;
  }
  if (o->coupling == VGTB_COUPLING_MOMENTUM && !s->blk_ds) {
    msg = "the momentum coupling needs the overlap gradients blk_ds";
    return VGTB_E_INVAL;
  }
  if (!(s->n_electrons >= 0.0) || s->n_electrons > 2.0 * n) {
    msg = "n_electrons out of range";
    return VGTB_E_INVAL;
  }
  if (s->gamma) {
    const int na = s->n_atoms;
    for (int i = 0; i < na; ++i)
      for (int j = 0; j < na; ++j)
        if (std::fabs(s->gamma[(size_t)i * na + j] - s->gamma[(size_t)j * na + i]) > 1e-12) {
          msg = "gamma must be symmetric";
          return VGTB_E_INVAL;
        }
  }
  return VGTB_OK;
}

// Arena carving: the same walk sizes the arena (base = 0) and assigns pointers.
struct Carver {
  char *base;
  size_t off = 0;
  explicit Carver(void *b) : base(static_cast<char *>(b)) {}
  template <typename T>
  T *take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T *p = reinterpret_cast<T *>(base + off);
    off += count * sizeof(T);
    return p;
  }
};

struct Sizes {
  int na, no, n, nk, np, ni, cap, precision, npad, ng, ne;
  bool scc, deviation, small, mom, cn;
};

template <typename Ctx>
void carve(Carver &cv, const Sizes &z, Ctx *c) {
  const size_t n2 = (size_t)z.n * z.n * z.nk;
  const size_t e2 = (size_t)z.no * z.no;
  c->kpts_dev = cv.template take<double>(3 * (size_t)z.nk);
  c->kw_dev = cv.template take<double>(z.nk);
  c->g.row_ptr = cv.template take<int>(z.na + 1);
  c->g.pair_col = cv.template take<int>(z.np);
  c->g.pair_row = cv.template take<int>(z.np);
  c->g.img_ptr = cv.template take<int>(z.np + 1);
  c->g.img_d = cv.template take<double>(3 * (size_t)z.ni);
  c->g.img_h0 = cv.template take<double>(e2 * z.ni);
  c->g.img_s = cv.template take<double>(e2 * z.ni);
  c->g.img_ds = z.mom ? cv.template take<double>(3 * e2 * z.ni) : nullptr;
  c->g.grp_ptr = cv.template take<int>(z.ng + 1);
  c->g.ent_j = cv.template take<int>(z.ne);
  c->g.ent_mask = cv.template take<int>(z.ne);
  c->g.ent_pp = cv.template take<int>(z.ne + 1);
  c->g.gp_pair = cv.template take<int>(z.np);
  c->g.gp_il = cv.template take<int>(z.np);
  c->spk = cv.template take<double2>(e2 * z.np * z.nk);
  c->hq = cv.template take<double2>(e2 * z.np * z.nk);
  c->h0k = z.mom ? cv.template take<double2>(e2 * z.np * z.nk) : nullptr;
  c->ppk = z.mom ? cv.template take<double2>(3 * e2 * z.np * z.nk) : nullptr;
  c->c0 = z.deviation ? cv.template take<double2>(n2) : nullptr;
  c->sinv = cv.template take<double2>(n2);
  c->dlev[0] = cv.template take<double2>(n2);
  c->dlev[1] = cv.template take<double2>(n2);
  c->d0 = z.deviation ? cv.template take<double2>(n2) : nullptr;
  c->w = cv.template take<double2>(n2);
  // y doubles as the spectrum's scratch between steps: at least 4096 doubles.
  c->y = cv.template take<double2>(std::max<size_t>(n2, 2048));
  c->part = cv.template take<double>((size_t)z.nk * z.na * 5);
  c->v = cv.template take<double>(z.na);
  c->z = cv.template take<double>(z.na);
  c->qbuf = cv.template take<double>(z.na);
  c->rowpart = cv.template take<double>((size_t)z.na * 5);
  c->gamma = z.scc ? cv.template take<double>((size_t)z.na * z.na) : nullptr;
  c->hist = cv.template take<double>((size_t)z.cap * (5 + z.na));
  c->eig = cv.template take<double>((size_t)z.nk * z.n);
  c->eig_e = cv.template take<double>((size_t)z.nk * z.n);
  c->occ = cv.template take<double>((size_t)z.nk * z.n);
  c->info = cv.template take<int>(z.nk);
  c->flag = cv.template take<int>(1);
  if (z.deviation) {
    const size_t lo = (z.precision == VGTB_FP32) ? n2 * sizeof(float2)
                                                  : (size_t)4 * z.npad * z.npad * z.nk * sizeof(uint16_t);
    // S^-1 - I: the bf16 form keeps kADither copies with dithered lo planes.
    c->sinv_lo = cv.template take<char>(z.precision == VGTB_BF16X3 ? lo * vgtb::kADither : lo);
    c->w_lo = cv.template take<char>(lo);
    c->y_lo = cv.template take<float2>(n2);
    c->w32 = (z.precision == VGTB_BF16X3 || z.precision == VGTB_FP16X3) ? cv.template take<float2>(n2)
                                                                         : nullptr;
    if (z.precision == VGTB_FP16X3) {
      c->scale_a = cv.template take<float>(z.nk);
      c->scale_w = cv.template take<float>(z.nk);
      c->scale_part = cv.template take<float>((size_t)z.nk * vgtb::f16_scale_parts());
      c->wmax = cv.template take<unsigned>((size_t)z.nk * vgtb::kMaxSlots * vgtb::kMaxStride);
      c->wflag = cv.template take<int>(z.nk);
    } else {
      c->scale_a = c->scale_w = c->scale_part = nullptr;
      c->wmax = nullptr;
      c->wflag = nullptr;
    }
    c->tpart = cv.template take<double>((size_t)2 * z.nk * z.na);
    c->tfac = cv.template take<double>((size_t)2 * z.nk);
    c->trace0 = cv.template take<double>(z.nk);
    c->m0 = cv.template take<double2>(n2);
  } else {
    c->m0 = nullptr;
    c->sinv_lo = c->w_lo = nullptr;
    c->y_lo = c->w32 = nullptr;
    c->scale_a = c->scale_w = c->scale_part = nullptr;
    c->wmax = nullptr;
    c->wflag = nullptr;
    c->tpart = c->tfac = c->trace0 = nullptr;
  }
  c->sm_part = z.small ? cv.template take<double>((size_t)vgtb::kSmallChunk * z.nk * z.na * 5) : nullptr;
  const bool small_scc = z.small && z.scc;
  c->sm_bar = small_scc ? cv.template take<unsigned>(4) : nullptr;
  c->sm_err = small_scc ? cv.template take<int>(4) : nullptr;
  c->sm_escc = small_scc ? cv.template take<double>(vgtb::kSmallChunk) : nullptr;
  c->ring = cv.template take<double>(3 * (size_t)vgtb::kStepRing);
  c->ctr = cv.template take<int64_t>(1);
  if (z.cn) {
    c->aug = cv.template take<double2>(2 * n2);
    c->cinv = cv.template take<double2>((size_t)vgtb::kCnBlock * vgtb::kCnBlock * z.nk);
    c->sq = cv.template take<double2>(e2 * z.np * z.nk);
    c->cocc = cv.template take<double>((size_t)z.nk * z.n);
    c->vprev = cv.template take<double>(z.na);
    c->vmid = cv.template take<double>(z.na);
    c->ring_mid = cv.template take<double>(3 * (size_t)vgtb::kStepRing);
  } else {
    c->aug = c->cinv = c->sq = nullptr;
    c->cocc = c->vprev = c->vmid = c->ring_mid = nullptr;
  }
}

// Mutable stand-in used for the size query (PairGraph members are const).
struct SizeProbe {
  struct {
    int *row_ptr, *pair_col, *pair_row, *img_ptr;
    double *img_d, *img_h0, *img_s, *img_ds;
    int *grp_ptr, *ent_j, *ent_mask, *ent_pp, *gp_pair, *gp_il;
  } g;
  double *kpts_dev, *kw_dev, *part, *v, *z, *qbuf, *rowpart, *gamma, *hist, *eig, *eig_e, *occ;
  double2 *spk, *hq, *h0k, *ppk, *c0, *sinv, *dlev[2], *d0, *w, *y;
  int *info, *flag;
  void *sinv_lo, *w_lo;
  float2 *y_lo, *w32;
  float *scale_a, *scale_w, *scale_part;
  unsigned *wmax;
  int *wflag;
  double *tpart, *tfac, *trace0;
  double2 *m0;
  double *sm_part, *ring;
  unsigned *sm_bar;
  int *sm_err;
  double *sm_escc;
  int64_t *ctr;
  double2 *aug, *cinv, *sq;
  double *cocc, *vprev, *vmid, *ring_mid;
};

struct DevPtrs : SizeProbe {};

Sizes sizes_of(const vgtb_system *s, const vgtb_options *o, const HostGraph &hg) {
  Sizes z;
  z.na = s->n_atoms;
  z.no = s->orbs_per_atom;
  z.n = z.na * z.no;
  z.nk = s->n_k;
  z.np = (int)hg.pair_col.size();
  z.ni = (int)(hg.img_d.size() / 3);
  z.ng = (int)hg.grp_ptr.size() - 1;
  z.ne = (int)hg.ent_j.size();
  z.cap = o->history_capacity;
  z.scc = s->gamma != nullptr;
  z.deviation = o->precision != VGTB_FP64;
  z.precision = o->precision;
  z.npad = (z.n + 63) / 64 * 64;
  z.mom = o->coupling == VGTB_COUPLING_MOMENTUM;
  z.cn = o->propagator == VGTB_PROP_CRANK_NICOLSON;
  z.small = !(o->flags & VGTB_OPT_NO_SMALL_PATH) && !z.mom && !z.cn && z.n <= vgtb::kSmallN &&
            (!z.scc || z.nk <= vgtb::kSmallSccMaxK) &&
            z.ni <= vgtb::kSmallImages;
  return z;
}

// Aufbau with f = 2; a degenerate group (spread < tol) straddling the Fermi
// level shares the remaining electrons equally.  eps ascending.
void fill_states(const double *eps, int n, double n_el, double tol, double *f) {
  double left = n_el;
  int i = 0;
  for (int t = 0; t < n; ++t) f[t] = 0.0;
  while (i < n && left > 1e-12) {
    int j = i + 1;
    while (j < n && std::fabs(eps[j] - eps[i]) < tol) ++j;
    const int g = j - i;
    const double take = std::min(2.0 * g, left);
    for (int t = i; t < j; ++t) f[t] = take / g;
    left -= take;
    i = j;
  }
}

// Run one launch, bracketed by timing events when profiling is on.
template <typename F>
void timed(vgtb_ctx *c, int id, F &&launch) {
  if (!c->profiling) {
    launch();
    return;
  }
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  if (!c->ev_free.empty()) {
    ev = c->ev_free.back();
    c->ev_free.pop_back();
  } else if (hipEventCreate(&ev.first) != hipSuccess || hipEventCreate(&ev.second) != hipSuccess) {
    launch();
    return;
  }
  (void)hipEventRecord(ev.first, c->stream);
  launch();
  (void)hipEventRecord(ev.second, c->stream);
  c->ev_pending.push_back({id, ev.first, ev.second});
}

void drop_graphs(vgtb_ctx *c);

// Deviation forms: C0 = H0_k(A=0) D0 (constant part of the sparse product)
// and, for a reference that is not stationary, m0 = -i (S^-1 C0 - C0^dag S^-1).
int product_format(const vgtb_ctx *c);

// Arguments of the next block of small-path steps of c beyond the state:
// the deviation form's constants and, with the SCC shift, the charges' inputs
// and the grid-wide barrier (whose count restarts from zero, on stream s,
// before it could wrap).
vgtb::SmallDeviation small_block_args(vgtb_ctx *c, hipStream_t s) {
  vgtb::SmallDeviation sd;
  if (c->precision != VGTB_FP64) {
    sd.form = product_format(c);
    sd.c0 = c->c0;
    sd.m0 = c->m0_active ? c->m0 : nullptr;
    sd.scale_a = c->scale_a;
    sd.trace0 = c->trace0;
    sd.rescale_every = c->rescale_every;
    sd.step0 = c->step;
  }
  if (c->scc) {
    if (c->bar_count > (1u << 30)) {
      vgtb::launch_fill_zero(reinterpret_cast<double2 *>(c->sm_bar), 1, s);
      c->bar_count = 0;
    }
    sd.gamma = c->gamma;
    sd.z = c->z;
    sd.kw = c->kw_dev;
    sd.bar = c->sm_bar;
    sd.bar_base = c->bar_count;
    sd.err = c->sm_err;
    sd.escc = c->sm_escc;
  }
  return sd;
}

void prepare_reference(vgtb_ctx *c, bool with_m0) {
  drop_graphs(c);   // captured updates name m0 (or not)
  if (c->small_path) {
    // The small path forms H D itself; C0 comes from the same arithmetic.
    vgtb::launch_small_c0(c->g, c->kpts_dev, c->nk, c->d0, c->c0, c->n, c->stream);
  } else {
    const vgtb::StepSource zero{nullptr, nullptr};
    vgtb::launch_assemble(c->g, c->kpts_dev, c->nk, zero, c->spk, nullptr, c->hq, c->h0k, c->ppk,
                          c->stream);
    vgtb::launch_spmm(c->g, c->d0, nullptr, c->n, c->nk, c->hq, nullptr, c->c0, 0, 0, nullptr,
                      c->spmm_variant, c->stream);
  }
  c->m0_active = with_m0;
  if (!with_m0) return;
  vgtb::launch_zgemm_f64(c->sinv, c->c0, c->y, c->n, c->nk, c->stream);
  vgtb::launch_fill_zero(c->w, (size_t)c->n * c->n * c->nk, c->stream);
  vgtb::launch_update_const(c->y, c->w, c->m0, c->n, c->nk, c->stream);
}

void drop_graphs(vgtb_ctx *c) {
  for (auto &g : c->graph)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

// Field ring: A(t)/c of steps [lo, lo + kStepRing) at slot step mod kStepRing.
// Refilled (one small launch) when steps [stp, stp + need) are not all in it.
void fill_ring(vgtb_ctx *c, int64_t stp, int need) {
  if (c->ring_lo >= 0 && stp >= c->ring_lo && stp + need <= c->ring_lo + vgtb::kStepRing) return;
  const int64_t nf = (int64_t)(c->field.size() / 3);
  vgtb::FieldChunk fc;
  for (int i = 0; i < vgtb::kStepRing; ++i) {
    const double *a = c->field.data() + 3 * std::min<int64_t>(stp + i, nf - 1);
    for (int x = 0; x < 3; ++x) fc.a[3 * i + x] = a[x] / vgtb::kLightSpeed;
  }
  vgtb::launch_store_ring(fc, stp, vgtb::kStepRing, c->ring, c->stream);
  if (c->cn) {
    // Crank-Nicolson: the field of the step's midpoint, (A(t_n) + A(t_{n+1})) / 2.
    for (int i = 0; i < vgtb::kStepRing; ++i) {
      const double *a = c->field.data() + 3 * std::min<int64_t>(stp + i, nf - 1);
      const double *b = c->field.data() + 3 * std::min<int64_t>(stp + i + 1, nf - 1);
      for (int x = 0; x < 3; ++x) fc.a[3 * i + x] = 0.5 * (a[x] + b[x]) / vgtb::kLightSpeed;
    }
    vgtb::launch_store_ring(fc, stp, vgtb::kStepRing, c->ring_mid, c->stream);
  }
  c->ring_lo = stp;
}

// One Crank-Nicolson step of the coefficients (Eq. 5): observables of C_n,
// SCC shift, H at the midpoint, W = S C_n, the solve of
// (S + i dt/2 H) X = W, and C_{n+1} = 2 X - C_n.
void enqueue_step_cn(vgtb_ctx *c, hipStream_t s) {
  const int n = c->n, nk = c->nk, ns = c->ns;
  const double jscale = -1.0 / c->volume;   // the k weights enter the sum
  const vgtb::StepSource src{c->ring, c->ctr}, mid{c->ring_mid, c->ctr};
  double2 *cc = c->dlev[0];
  double2 *dp = c->dlev[1];
  timed(c, VGTB_K_CN_PATTERN, [&] { vgtb::launch_cn_pattern(c->g, cc, c->cocc, n, ns, nk, dp, s); });
  timed(c, VGTB_K_OBSERVE, [&] {
    vgtb::launch_observe(c->g, dp, n, c->kpts_dev, nk, src, c->spk, c->h0k, c->ppk, c->part, s);
  });
  timed(c, VGTB_K_REDUCE, [&] {
    vgtb::launch_reduce(c->part, nk, c->na, c->kw_dev, jscale, c->scc ? c->gamma : nullptr, c->z,
                        c->v, c->qbuf, c->rowpart, c->hist, c->hist_cap, c->ctr, c->flag, s);
    if (c->scc) vgtb::launch_cn_vmid(c->v, c->vprev, c->vmid, c->na, !c->have_vprev, s);
  });
  c->have_vprev = true;
  timed(c, VGTB_K_ASSEMBLE, [&] {
    vgtb::launch_assemble(c->g, c->kpts_dev, nk, mid, c->spk, c->scc ? c->vmid : nullptr, c->hq,
                          c->h0k, c->ppk, s);
  });
  timed(c, VGTB_K_SPMM, [&] {
    vgtb::launch_spmm(c->g, cc, nullptr, n, nk, c->sq, nullptr, c->w, 0, 0, nullptr, c->spmm_variant, s, ns);
  });
  timed(c, VGTB_K_CN_SOLVE, [&] {
    vgtb::launch_cn_build(c->g, c->w, c->hq, c->spk, 0.5 * c->dt, n, ns, nk, c->aug, s);
    vgtb::launch_cn_solve(c->aug, c->cinv, n, ns, nk, c->gemm_tile, s);
  });
  timed(c, VGTB_K_CN_UPDATE, [&] { vgtb::launch_cn_update(c->aug, cc, n, ns, nk, c->ctr, s); });
}

// Operand format of the reduced product: 1 complex64, 2 bf16 planes, 3 scaled
// fp16 planes (0: FP64, no reduced product).
int product_format(const vgtb_ctx *c) {
  switch (c->precision) {
    case VGTB_FP32: return 1;
    case VGTB_BF16X3: return 2;
    case VGTB_FP16X3: return 3;
    default: return 0;
  }
}

// Deviation form W = H D - H0 D0 in FP64, written in the product's operand
// format (fp16: as complex64 into w32, then scaled and split into planes).
void launch_deviation_spmm(vgtb_ctx *c, const double2 *dcur, int fmt, int variant, hipStream_t s) {
  const int n = c->n, nk = c->nk;
  if (fmt == 3) {
    // The planes are written with the previous step's scales; a k-point whose
    // maximum calls for another scale is split again from the complex64 W.
    vgtb::launch_spmm(c->g, dcur, c->d0, n, nk, c->hq, c->c0, c->w_lo, 3, c->np, c->w32, variant, s, 0,
                      c->scale_w, c->wmax);
    vgtb::launch_f16_scale_check(c->wmax, c->scale_w, c->wflag, nk, s);
    vgtb::launch_split_w_f16(c->w32, c->scale_w, static_cast<uint16_t *>(c->w_lo), n, c->np, nk,
                             c->wflag, s);
  } else {
    vgtb::launch_spmm(c->g, dcur, c->d0, n, nk, c->hq, c->c0, c->w_lo, fmt, c->np, c->w32, variant, s);
  }
}

// G = (S^-1 - I) W in the reduced format, into y_lo.
void launch_reduced_product(vgtb_ctx *c, int fmt, int tile, hipStream_t s) {
  const int n = c->n, nk = c->nk;
  if (fmt == 1)
    vgtb::launch_cgemm_f32(static_cast<const float2 *>(c->sinv_lo), static_cast<const float2 *>(c->w_lo),
                           c->y_lo, n, nk, s, tile);
  else if (fmt == 2)
    vgtb::launch_cgemm_bf16x3(static_cast<const uint16_t *>(c->sinv_lo),
                              static_cast<const uint16_t *>(c->w_lo), c->y_lo, n, c->np, nk, s, tile,
                              c->ctr);
  else
    vgtb::launch_cgemm_f16x3(static_cast<const uint16_t *>(c->sinv_lo),
                             static_cast<const uint16_t *>(c->w_lo), c->y_lo, n, c->np, nk, c->scale_a,
                             c->scale_w, s, tile);
}

// The launches of one step at the current parity, on stream s.  With
// may_time, each launch is bracketed by profiling events when enabled
// (never while capturing).
void enqueue_step(vgtb_ctx *c, hipStream_t s, bool may_time) {
  const int n = c->n, nk = c->nk;
  const bool dev = c->precision != VGTB_FP64;
  const double jscale = -1.0 / c->volume;   // the k weights enter the sum
  const vgtb::StepSource src{c->ring, c->ctr};
  double2 *dcur = c->dlev[c->cur];
  double2 *doth = c->dlev[c->cur ^ 1];
  const bool first = !c->have_prev;
  auto run = [&](int id, auto &&launch) {
    if (may_time) timed(c, id, launch);
    else launch();
  };
  run(VGTB_K_OBSERVE, [&] {
    vgtb::launch_observe(c->g, dcur, n, c->kpts_dev, nk, src, c->spk, c->h0k, c->ppk, c->part, s);
  });
  run(VGTB_K_REDUCE, [&] {
    vgtb::launch_reduce(c->part, nk, c->na, c->kw_dev, jscale, c->scc ? c->gamma : nullptr, c->z,
                        c->v, c->qbuf, c->rowpart, c->hist, c->hist_cap, c->ctr, c->flag, s);
  });
  run(VGTB_K_ASSEMBLE, [&] {
    vgtb::launch_assemble(c->g, c->kpts_dev, nk, src, c->spk, c->scc ? c->v : nullptr, c->hq, c->h0k,
                          c->ppk, s);
  });
  if (!dev) {
    run(VGTB_K_SPMM, [&] {
      vgtb::launch_spmm(c->g, dcur, nullptr, n, nk, c->hq, nullptr, c->w, 0, 0, nullptr,
                        c->spmm_variant, s);
    });
    run(VGTB_K_GEMM, [&] { vgtb::launch_zgemm_f64(c->sinv, c->w, c->y, n, nk, s, c->gemm_tile); });
    run(VGTB_K_UPDATE, [&] {
      vgtb::launch_update(c->y, first ? dcur : doth, doth, n, nk, first ? c->dt : 2.0 * c->dt,
                          c->ctr, s);
    });
    return;
  }
  // Deviation form: W = H D - H0 D0 in FP64 (C0 = H0 D0 kept from the
  // reference), rounded to the product's format; S^-1 W = W + (S^-1 - I) W
  // with only the second term in reduced precision.  The state D stays FP64.
  const int fmt = product_format(c);
  run(VGTB_K_SPMM, [&] { launch_deviation_spmm(c, dcur, fmt, c->spmm_variant, s); });
  const float2 *wid = fmt == 1 ? static_cast<const float2 *>(c->w_lo) : c->w32;
  const double2 *m0 = c->m0_active ? c->m0 : nullptr;
  if (fmt >= 2 && c->fuse_update) {
    // The 16-bit split product and the update in one launch over mirrored tile pairs.
    bool done = false;
    run(VGTB_K_GEMM, [&] {
      done = vgtb::launch_cgemm_update_split16(
          fmt, static_cast<const uint16_t *>(c->sinv_lo), static_cast<const uint16_t *>(c->w_lo), c->y_lo,
          wid, m0, first ? dcur : doth, doth, n, c->np, nk, first ? c->dt : 2.0 * c->dt, c->ctr,
          fmt == 3 ? c->scale_a : nullptr, fmt == 3 ? c->scale_w : nullptr, s, c->gemm_tile);
    });
    if (done) return;
  }
  run(VGTB_K_GEMM, [&] { launch_reduced_product(c, fmt, c->gemm_tile, s); });
  run(VGTB_K_UPDATE, [&] {
    vgtb::launch_update_split(c->y_lo, wid, m0, first ? dcur : doth, doth, n, nk,
                              first ? c->dt : 2.0 * c->dt, c->ctr, s);
  });
}

// Capture two consecutive steps starting at leapfrog parity `parity` (both with
// a previous level) on the private capture stream and instantiate the graph.
vgtb_status capture_pair(vgtb_ctx *c, int parity) {
  if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  const int saved_cur = c->cur;
  const bool saved_prev = c->have_prev;
  HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  c->cur = parity;
  c->have_prev = true;
  enqueue_step(c, c->cap_stream, false);
  c->cur ^= 1;
  enqueue_step(c, c->cap_stream, false);
  c->cur = saved_cur;
  c->have_prev = saved_prev;
  hipGraph_t graph = nullptr;
  const hipError_t e1 = hipStreamEndCapture(c->cap_stream, &graph);
  if (e1 != hipSuccess) return fail(c, VGTB_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e1));
  const hipError_t e2 = hipGraphInstantiate(&c->graph[parity], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) {
    c->graph[parity] = nullptr;
    return fail(c, VGTB_E_DEVICE, std::string("graph instantiation: ") + hipGetErrorString(e2));
  }
  return VGTB_OK;
}

vgtb_status check_ready(vgtb_ctx *ctx) {
  if (!ctx) return fail(nullptr, VGTB_E_INVAL, "null context");
  if (ctx->poisoned) return VGTB_E_STATE;
  return VGTB_OK;
}

}  // namespace

namespace vgtb {
void set_last_error(const char *m) { set_global_err(m); }
}  // namespace vgtb

extern "C" {

vgtb_status vgtb_workspace_size(const vgtb_system *s, const vgtb_options *o, size_t *bytes) {
  std::string msg;
  vgtb_status st = validate(s, o, msg);
  if (st != VGTB_OK) return fail(nullptr, st, msg);
  if (!bytes) return fail(nullptr, VGTB_E_INVAL, "null bytes pointer");
  HostGraph hg;
  st = build_graph(s, o, hg, msg);
  if (st != VGTB_OK) return fail(nullptr, st, msg);
  Carver cv(nullptr);
  SizeProbe probe;
  carve(cv, sizes_of(s, o, hg), &probe);
  *bytes = cv.off + 256;
  return VGTB_OK;
}

vgtb_status vgtb_create(const vgtb_system *s, const vgtb_options *o, void *arena,
                        size_t arena_bytes, void *hip_stream, vgtb_ctx **out) {
  std::string msg;
  vgtb_status st = validate(s, o, msg);
  if (st != VGTB_OK) return fail(nullptr, st, msg);
  if (!out || !arena) return fail(nullptr, VGTB_E_INVAL, "null arena or output pointer");
  if ((reinterpret_cast<uintptr_t>(arena) & 255) != 0)
    return fail(nullptr, VGTB_E_INVAL, "arena must be 256-byte aligned");
  HostGraph hg;
  st = build_graph(s, o, hg, msg);
  if (st != VGTB_OK) return fail(nullptr, st, msg);
  const Sizes z = sizes_of(s, o, hg);
  {
    Carver probe_cv(nullptr);
    SizeProbe probe;
    carve(probe_cv, z, &probe);
    if (probe_cv.off + 256 > arena_bytes)
      return fail(nullptr, VGTB_E_NOMEM, "arena too small: need " + std::to_string(probe_cv.off + 256));
  }

  vgtb_ctx *c = new vgtb_ctx();
  c->na = z.na;
  c->no = z.no;
  c->n = z.n;
  c->nk = z.nk;
  c->hist_cap = z.cap;
  c->scc = z.scc;
  c->precision = o->precision;
  c->rescale_every = o->rescale_every;
  c->dt = o->dt;
  c->n_electrons = s->n_electrons;
  {
    const double *cl = s->cell;
    c->volume = std::fabs(cl[0] * (cl[4] * cl[8] - cl[5] * cl[7]) - cl[1] * (cl[3] * cl[8] - cl[5] * cl[6]) +
                          cl[2] * (cl[3] * cl[7] - cl[4] * cl[6]));
  }
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->kpts.assign(s->kpts, s->kpts + 3 * (size_t)z.nk);
  c->kw.assign(s->kw, s->kw + z.nk);
  c->field.assign(3, 0.0);
  c->z_host.assign(z.na, 0.0);
  c->z_from_ground_state = (s->z_ref == nullptr);
  if (s->z_ref) c->z_host.assign(s->z_ref, s->z_ref + z.na);

  auto bail = [&](vgtb_status code, const std::string &m) {
    set_global_err(m.c_str());
    if (c->blas) rocblas_destroy_handle(c->blas);
    delete c;
    return code;
  };
  if (hipGetDevice(&c->device) != hipSuccess) return bail(VGTB_E_DEVICE, "hipGetDevice failed");

  Carver cv(arena);
  DevPtrs dp;
  carve(cv, z, &dp);
  c->kpts_dev = dp.kpts_dev;
  c->kw_dev = dp.kw_dev;
  c->g.n_atoms = z.na;
  c->g.norb = z.no;
  c->g.n_pairs = z.np;
  c->g.n_images = z.ni;
  c->g.row_ptr = dp.g.row_ptr;
  c->g.pair_col = dp.g.pair_col;
  c->g.pair_row = dp.g.pair_row;
  c->g.img_ptr = dp.g.img_ptr;
  c->g.img_d = dp.g.img_d;
  c->g.img_h0 = dp.g.img_h0;
  c->g.img_s = dp.g.img_s;
  c->g.img_ds = dp.g.img_ds;
  c->g.group_size = spmm_group_of(o);
  c->spmm_variant = spmm_variant_of(o);
  c->gemm_tile = o->tile_override;
  c->g.n_groups = z.ng;
  c->g.n_entries = z.ne;
  c->g.grp_ptr = dp.g.grp_ptr;
  c->g.ent_j = dp.g.ent_j;
  c->g.ent_mask = dp.g.ent_mask;
  c->g.ent_pp = dp.g.ent_pp;
  c->g.gp_pair = dp.g.gp_pair;
  c->g.gp_il = dp.g.gp_il;
  c->spk = dp.spk;
  c->hq = dp.hq;
  c->h0k = dp.h0k;
  c->ppk = dp.ppk;
  c->c0 = dp.c0;
  c->sinv = dp.sinv;
  c->dlev[0] = dp.dlev[0];
  c->dlev[1] = dp.dlev[1];
  c->d0 = dp.d0;
  c->w = dp.w;
  c->y = dp.y;
  c->part = dp.part;
  c->v = dp.v;
  c->z = dp.z;
  c->qbuf = dp.qbuf;
  c->rowpart = dp.rowpart;
  c->gamma = dp.gamma;
  c->hist = dp.hist;
  c->eig = dp.eig;
  c->eig_e = dp.eig_e;
  c->occ = dp.occ;
  c->info = dp.info;
  c->flag = dp.flag;
  c->np = z.npad;
  c->sinv_lo = dp.sinv_lo;
  c->w_lo = dp.w_lo;
  c->y_lo = dp.y_lo;
  c->w32 = dp.w32;
  c->scale_a = dp.scale_a;
  c->scale_w = dp.scale_w;
  c->scale_part = dp.scale_part;
  c->wmax = dp.wmax;
  c->wflag = dp.wflag;
  c->tpart = dp.tpart;
  c->tfac = dp.tfac;
  c->trace0 = dp.trace0;
  c->m0 = dp.m0;
  c->sm_part = dp.sm_part;
  c->sm_bar = dp.sm_bar;
  c->sm_err = dp.sm_err;
  c->sm_escc = dp.sm_escc;
  c->ring = dp.ring;
  c->ctr = dp.ctr;
  c->small_path = z.small;
  // The SCC small path needs every k-point's workgroup resident at once.
  if (z.small && z.scc && vgtb::small_scc_max_kpoints(z.no) < z.nk) c->small_path = false;
  c->use_graphs = !(o->flags & VGTB_OPT_NO_GRAPHS) && !z.cn;
  c->fuse_update = (o->flags & VGTB_OPT_FUSE_UPDATE) != 0;
  c->cn = z.cn;
  c->aug = dp.aug;
  c->cinv = dp.cinv;
  c->sq = dp.sq;
  c->cocc = dp.cocc;
  c->vprev = dp.vprev;
  c->vmid = dp.vmid;
  c->ring_mid = dp.ring_mid;

  hipStream_t st_ = c->stream;
#define CREATE_HIP(expr)                                                              \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess) return bail(VGTB_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(_e)); \
  } while (0)
  CREATE_HIP(hipMemcpyAsync(dp.kpts_dev, s->kpts, 3 * sizeof(double) * z.nk, hipMemcpyHostToDevice, st_));
  CREATE_HIP(hipMemcpyAsync(dp.kw_dev, s->kw, sizeof(double) * z.nk, hipMemcpyHostToDevice, st_));
  CREATE_HIP(hipMemcpyAsync(dp.g.row_ptr, hg.row_ptr.data(), sizeof(int) * hg.row_ptr.size(), hipMemcpyHostToDevice, st_));
  CREATE_HIP(hipMemcpyAsync(dp.g.pair_col, hg.pair_col.data(), sizeof(int) * hg.pair_col.size(), hipMemcpyHostToDevice, st_));
  CREATE_HIP(hipMemcpyAsync(dp.g.pair_row, hg.pair_row.data(), sizeof(int) * hg.pair_row.size(), hipMemcpyHostToDevice, st_));
  CREATE_HIP(hipMemcpyAsync(dp.g.img_ptr, hg.img_ptr.data(), sizeof(int) * hg.img_ptr.size(), hipMemcpyHostToDevice, st_));
  CREATE_HIP(hipMemcpyAsync(dp.g.img_d, hg.img_d.data(), sizeof(double) * hg.img_d.size(), hipMemcpyHostToDevice, st_));
  CREATE_HIP(hipMemcpyAsync(dp.g.img_h0, hg.img_h0.data(), sizeof(double) * hg.img_h0.size(), hipMemcpyHostToDevice, st_));
  CREATE_HIP(hipMemcpyAsync(dp.g.img_s, hg.img_s.data(), sizeof(double) * hg.img_s.size(), hipMemcpyHostToDevice, st_));
  if (z.mom)
    CREATE_HIP(hipMemcpyAsync(dp.g.img_ds, hg.img_ds.data(), sizeof(double) * hg.img_ds.size(), hipMemcpyHostToDevice, st_));
  CREATE_HIP(hipMemcpyAsync(dp.g.grp_ptr, hg.grp_ptr.data(), sizeof(int) * hg.grp_ptr.size(), hipMemcpyHostToDevice, st_));
  CREATE_HIP(hipMemcpyAsync(dp.g.ent_j, hg.ent_j.data(), sizeof(int) * hg.ent_j.size(), hipMemcpyHostToDevice, st_));
  CREATE_HIP(hipMemcpyAsync(dp.g.ent_mask, hg.ent_mask.data(), sizeof(int) * hg.ent_mask.size(), hipMemcpyHostToDevice, st_));
  CREATE_HIP(hipMemcpyAsync(dp.g.ent_pp, hg.ent_pp.data(), sizeof(int) * hg.ent_pp.size(), hipMemcpyHostToDevice, st_));
  CREATE_HIP(hipMemcpyAsync(dp.g.gp_pair, hg.gp_pair.data(), sizeof(int) * hg.gp_pair.size(), hipMemcpyHostToDevice, st_));
  CREATE_HIP(hipMemcpyAsync(dp.g.gp_il, hg.gp_il.data(), sizeof(int) * hg.gp_il.size(), hipMemcpyHostToDevice, st_));
  CREATE_HIP(hipMemcpyAsync(dp.z, c->z_host.data(), sizeof(double) * z.na, hipMemcpyHostToDevice, st_));
  if (z.scc)
    CREATE_HIP(hipMemcpyAsync(dp.gamma, s->gamma, sizeof(double) * z.na * z.na, hipMemcpyHostToDevice, st_));
  CREATE_HIP(hipMemsetAsync(dp.v, 0, sizeof(double) * z.na, st_));
  CREATE_HIP(hipMemsetAsync(dp.flag, 0, sizeof(int), st_));
  if (dp.sm_bar) {
    CREATE_HIP(hipMemsetAsync(dp.sm_bar, 0, sizeof(unsigned), st_));
    CREATE_HIP(hipMemsetAsync(dp.sm_err, 0, sizeof(int), st_));
  }
  vgtb::launch_set_counter(dp.ctr, 0, st_);

  // S_k on the pair graph (Eq. 7), dense S_k, then S_k^-1 by Cholesky.
  vgtb::launch_pair_bloch_s(c->g, dp.kpts_dev, z.nk, dp.spk, st_);
  if (z.mom) vgtb::launch_pair_bloch_momentum(c->g, dp.kpts_dev, z.nk, dp.h0k, dp.ppk, st_);
  if (z.cn) vgtb::launch_cn_permute_pairs(c->g, dp.spk, dp.sq, z.nk, st_);
  const size_t n2 = (size_t)z.n * z.n * z.nk;
  vgtb::launch_fill_zero(dp.sinv, n2, st_);
  vgtb::launch_scatter_pairs(c->g, dp.kpts_dev, z.nk, dp.spk, 0, dp.sinv, z.n, st_);
  CREATE_HIP(hipGetLastError());
  if (rocblas_create_handle(&c->blas) != rocblas_status_success) {
    c->blas = nullptr;
    return bail(VGTB_E_DEVICE, "rocblas_create_handle failed");
  }
  if (rocblas_set_stream(c->blas, st_) != rocblas_status_success)
    return bail(VGTB_E_DEVICE, "rocblas_set_stream failed");
  // Row-major Hermitian storage read column-major is conj(S); the factor /
  // inverse of its column-major upper triangle is S^-1's row-major lower one.
  if (rocsolver_zpotrf_strided_batched(c->blas, rocblas_fill_upper, z.n,
                                       reinterpret_cast<rocblas_double_complex *>(dp.sinv), z.n,
                                       (rocblas_stride)z.n * z.n, dp.info, z.nk) != rocblas_status_success)
    return bail(VGTB_E_DEVICE, "rocsolver_zpotrf_strided_batched failed");
  std::vector<int> info(z.nk);
  CREATE_HIP(hipMemcpyAsync(info.data(), dp.info, sizeof(int) * z.nk, hipMemcpyDeviceToHost, st_));
  CREATE_HIP(hipStreamSynchronize(st_));
  for (int k = 0; k < z.nk; ++k)
    if (info[k] != 0)
      return bail(VGTB_E_NOT_PD, "S_k is not positive definite at k-point " + std::to_string(k) +
                                     " (leading minor " + std::to_string(info[k]) + ")");
  if (rocsolver_zpotri_strided_batched(c->blas, rocblas_fill_upper, z.n,
                                       reinterpret_cast<rocblas_double_complex *>(dp.sinv), z.n,
                                       (rocblas_stride)z.n * z.n, dp.info, z.nk) != rocblas_status_success)
    return bail(VGTB_E_DEVICE, "rocsolver_zpotri_strided_batched failed");
  vgtb::launch_hermitian_from_lower(dp.sinv, z.n, z.nk, st_);
  CREATE_HIP(hipGetLastError());
  CREATE_HIP(hipMemcpyAsync(info.data(), dp.info, sizeof(int) * z.nk, hipMemcpyDeviceToHost, st_));
  CREATE_HIP(hipStreamSynchronize(st_));
  for (int k = 0; k < z.nk; ++k)
    if (info[k] != 0) return bail(VGTB_E_NOT_PD, "S_k is singular at k-point " + std::to_string(k));
  if (z.deviation) {
    // S^-1 in the reduced-precision operand format; W's padding stays zero.
    const int fmt = z.precision == VGTB_FP32 ? 1 : (z.precision == VGTB_BF16X3 ? 2 : 3);
    if (fmt == 3) {
      vgtb::launch_f16_scale(dp.sinv, z.n, z.nk, true, dp.scale_part, dp.scale_a, st_);
      vgtb::launch_f16_scale_init(dp.wmax, dp.scale_w, z.nk, st_);
      vgtb::launch_split_a_f16(dp.sinv, dp.scale_a, static_cast<uint16_t *>(dp.sinv_lo), z.n, z.npad,
                               z.nk, st_);
    } else {
      vgtb::launch_convert_operand(dp.sinv, dp.sinv_lo, z.n, z.npad, z.nk, fmt, st_);
    }
    if (fmt >= 2) {
      const size_t bytes = (size_t)4 * z.npad * z.npad * z.nk * sizeof(uint16_t);
      vgtb::launch_fill_zero(static_cast<double2 *>(dp.w_lo), bytes / sizeof(double2), st_);
    }
    CREATE_HIP(hipGetLastError());
    CREATE_HIP(hipStreamSynchronize(st_));
  }
#undef CREATE_HIP
  *out = c;
  return VGTB_OK;
}

vgtb_status vgtb_ground_state(vgtb_ctx *c, double *min_gap) {
  vgtb_status st = check_ready(c);
  if (st != VGTB_OK) return st;
  const int n = c->n, nk = c->nk;
  const size_t n2 = (size_t)n * n * nk;
  hipStream_t s = c->stream;
  vgtb::launch_fill_zero(c->w, n2, s);
  vgtb::launch_scatter_pairs(c->g, c->kpts_dev, nk, c->spk, 0, c->w, n, s);
  vgtb::launch_fill_zero(c->y, n2, s);
  vgtb::launch_scatter_pairs(c->g, c->kpts_dev, nk, c->spk, 1, c->y, n, s);
  HIP_TRY(c, hipGetLastError());
  BLAS_TRY(c, rocsolver_zhegvd_strided_batched(
                  c->blas, rocblas_eform_ax, rocblas_evect_original, rocblas_fill_upper, n,
                  reinterpret_cast<rocblas_double_complex *>(c->y), n, (rocblas_stride)n * n,
                  reinterpret_cast<rocblas_double_complex *>(c->w), n, (rocblas_stride)n * n, c->eig,
                  n, c->eig_e, n, c->info, nk));
  std::vector<int> info(nk);
  std::vector<double> eps((size_t)nk * n), occ((size_t)nk * n);
  HIP_TRY(c, hipMemcpyAsync(info.data(), c->info, sizeof(int) * nk, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(eps.data(), c->eig, sizeof(double) * eps.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  for (int k = 0; k < nk; ++k) {
    if (info[k] > n) return fail(c, VGTB_E_NOT_PD, "S_k not positive definite at k-point " + std::to_string(k));
    if (info[k] != 0) return fail(c, VGTB_E_DEVICE, "eigensolver did not converge at k-point " + std::to_string(k));
  }
  double gap = INFINITY, width = 0.0;
  const int n_occ = (int)std::lround(c->n_electrons / 2.0);
  for (int k = 0; k < nk; ++k) {
    const double *e = eps.data() + (size_t)k * n;
    fill_states(e, n, c->n_electrons, 1e-8, occ.data() + (size_t)k * n);
    if (n_occ > 0 && n_occ < n) gap = std::min(gap, e[n_occ] - e[n_occ - 1]);
    width = std::max(width, e[n - 1] - e[0]);
  }
  HIP_TRY(c, hipMemcpyAsync(c->occ, occ.data(), sizeof(double) * occ.size(), hipMemcpyHostToDevice, s));
  double2 *dtarget = c->dlev[c->cn ? 1 : 0];
  vgtb::launch_density_from_vectors(c->y, c->occ, dtarget, n, nk, s);
  if (c->cn) {
    // Coefficients: the occupied vectors (the largest occupied count over k).
    int ns = 1;
    for (int k = 0; k < nk; ++k) {
      int cnt = 0;
      for (int t = 0; t < n; ++t) cnt += occ[(size_t)k * n + t] > 0.0 ? 1 : 0;
      ns = std::max(ns, cnt);
    }
    vgtb::launch_cn_from_vectors(c->y, c->dlev[0], n, ns, nk, s);
    HIP_TRY(c, hipMemcpyAsync(c->cocc, c->occ, sizeof(double) * occ.size(), hipMemcpyDeviceToDevice, s));
    c->ns = ns;
    c->have_vprev = false;
  }
  HIP_TRY(c, hipGetLastError());
  c->cur = 0;
  if (c->precision != VGTB_FP64) {
    // The ground state is also the reference D0 of the reduced-precision product.
    HIP_TRY(c, hipMemcpyAsync(c->d0, c->dlev[0], sizeof(double2) * n2, hipMemcpyDeviceToDevice, s));
    vgtb::launch_trace_target(c->g, c->dlev[0], n, nk, c->spk, c->tpart, c->trace0, s);
    prepare_reference(c, false);   // the ground state commutes with S^-1 H0: no m0 term
  }
  c->have_density = true;
  c->have_prev = false;
  c->step = 0;
  if (c->z_from_ground_state) {
    // Reference charges = Mulliken charges of the ground state (dq = 0 at t = 0).
    const vgtb::StepSource zero{nullptr, nullptr};
    vgtb::launch_observe(c->g, dtarget, n, c->kpts_dev, nk, zero, c->spk, c->h0k, c->ppk, c->part, s);
    vgtb::launch_reduce(c->part, nk, c->na, c->kw_dev, 0.0, nullptr, c->z, c->v, c->qbuf,
                        c->rowpart, c->hist, c->hist_cap, nullptr, c->flag, s);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipMemcpyAsync(c->z, c->qbuf, sizeof(double) * c->na, hipMemcpyDeviceToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(c->z_host.data(), c->qbuf, sizeof(double) * c->na, hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(c, hipMemsetAsync(c->v, 0, sizeof(double) * c->na, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (min_gap) *min_gap = (n_occ > 0 && n_occ < n) ? gap : 0.0;
  // The leapfrog needs |dt| times the spectral width below 1; Crank-Nicolson
  // is stable for any step.
  if (!c->cn && std::fabs(c->dt) * width >= 1.0)
    return fail(c, VGTB_E_UNSTABLE, "|dt| * spectral width = " + std::to_string(std::fabs(c->dt) * width) + " >= 1");
  return VGTB_OK;
}

vgtb_status vgtb_set_density(vgtb_ctx *c, const void *d, int on_device) {
  vgtb_status st = check_ready(c);
  if (st != VGTB_OK) return st;
  if (c->cn) return fail(c, VGTB_E_STATE, "a Crank-Nicolson context holds coefficients: use vgtb_set_coefficients");
  if (!d) return fail(c, VGTB_E_INVAL, "null density");
  const size_t bytes = sizeof(double2) * (size_t)c->n * c->n * c->nk;
  HIP_TRY(c, hipMemcpyAsync(c->dlev[0], d, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
  c->cur = 0;
  if (c->precision != VGTB_FP64) {
    HIP_TRY(c, hipMemcpyAsync(c->d0, c->dlev[0], bytes, hipMemcpyDeviceToDevice, c->stream));
    vgtb::launch_trace_target(c->g, c->dlev[0], c->n, c->nk, c->spk, c->tpart, c->trace0, c->stream);
    // A density given by the caller need not be stationary: keep the constant
    // part of dD/dt, m0 = -i (S^-1 H0 D0 - D0 H0 S^-1), in FP64.
    prepare_reference(c, true);
  }
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->cur = 0;
  c->have_density = true;
  c->have_prev = false;
  c->step = 0;
  return VGTB_OK;
}

vgtb_status vgtb_set_coefficients(vgtb_ctx *c, const void *cf, const double *occ, int32_t ns,
                                  int on_device) {
  vgtb_status st = check_ready(c);
  if (st != VGTB_OK) return st;
  if (!c->cn) return fail(c, VGTB_E_STATE, "coefficients need a Crank-Nicolson context");
  if (!cf || !occ) return fail(c, VGTB_E_INVAL, "null coefficients or occupations");
  if (ns < 1 || ns > c->n) return fail(c, VGTB_E_INVAL, "n_states must be in 1 .. N");
  const int n = c->n, nk = c->nk;
  std::vector<double> f((size_t)nk * n, 0.0);
  for (int k = 0; k < nk; ++k)
    for (int t = 0; t < ns; ++t) {
      const double v = occ[(size_t)k * ns + t];
      if (!std::isfinite(v) || v < 0.0) return fail(c, VGTB_E_INVAL, "occupations must be finite and >= 0");
      f[(size_t)k * n + t] = v;
    }
  hipStream_t s = c->stream;
  // Columns past n_states stay zero: the sparse product reads every column.
  vgtb::launch_fill_zero(c->dlev[0], (size_t)n * n * nk, s);
  HIP_TRY(c, hipMemcpy2DAsync(c->dlev[0], sizeof(double2) * n, cf, sizeof(double2) * ns,
                              sizeof(double2) * ns, (size_t)n * nk,
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(c->cocc, f.data(), sizeof(double) * f.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(s));
  c->ns = ns;
  c->cur = 0;
  c->have_density = true;
  c->have_prev = false;
  c->have_vprev = false;
  c->step = 0;
  return VGTB_OK;
}

int32_t vgtb_num_states(const vgtb_ctx *c) { return (c && c->cn) ? c->ns : -1; }

vgtb_status vgtb_get_coefficients(vgtb_ctx *c, void *out, double *occ, int on_device) {
  vgtb_status st = check_ready(c);
  if (st != VGTB_OK) return st;
  if (!c->cn) return fail(c, VGTB_E_STATE, "coefficients need a Crank-Nicolson context");
  if (!c->have_density) return fail(c, VGTB_E_STATE, "no coefficients set");
  if (!out) return fail(c, VGTB_E_INVAL, "null output");
  const int n = c->n, nk = c->nk, ns = c->ns;
  hipStream_t s = c->stream;
  HIP_TRY(c, hipMemcpy2DAsync(out, sizeof(double2) * ns, c->dlev[0], sizeof(double2) * n,
                              sizeof(double2) * ns, (size_t)n * nk,
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  std::vector<double> f((size_t)nk * n);
  HIP_TRY(c, hipMemcpyAsync(f.data(), c->cocc, sizeof(double) * f.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (occ)
    for (int k = 0; k < nk; ++k)
      for (int t = 0; t < ns; ++t) occ[(size_t)k * ns + t] = f[(size_t)k * n + t];
  return VGTB_OK;
}

vgtb_status vgtb_set_field_table(vgtb_ctx *c, int64_t n, const double *a) {
  vgtb_status st = check_ready(c);
  if (st != VGTB_OK) return st;
  if (n < 1 || !a) return fail(c, VGTB_E_INVAL, "field table needs n >= 1 entries");
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!std::isfinite(a[i])) return fail(c, VGTB_E_INVAL, "non-finite vector potential");
  c->field.assign(a, a + 3 * n);
  c->ring_lo = -1;   // the device ring holds the old table
  return VGTB_OK;
}

vgtb_status vgtb_set_field(vgtb_ctx *c, const double a[3]) { return vgtb_set_field_table(c, 1, a); }

vgtb_status vgtb_step(vgtb_ctx *c, int64_t n_steps) {
  vgtb_status st = check_ready(c);
  if (st != VGTB_OK) return st;
  if (!c->have_density) return fail(c, VGTB_E_STATE, "vgtb_step before a density was set");
  if (n_steps < 0) return fail(c, VGTB_E_INVAL, "negative step count");
  HIP_TRY(c, hipSetDevice(c->device));
  const int n = c->n, nk = c->nk;
  const bool dev = c->precision != VGTB_FP64;
  const int64_t nf = (int64_t)(c->field.size() / 3);
  const double jscale = -1.0 / c->volume;   // the k weights enter the sum
  hipStream_t s = c->stream;
  if (c->small_path) {
    hipError_t launch_err = hipSuccess;
    for (int64_t done = 0; done < n_steps;) {
      const int ns = (int)std::min<int64_t>(vgtb::kSmallChunk, n_steps - done);
      vgtb::FieldChunk fc;
      for (int i = 0; i < ns; ++i) {
        const double *a = c->field.data() + 3 * std::min<int64_t>(c->step + i, nf - 1);
        for (int x = 0; x < 3; ++x) fc.a[3 * i + x] = a[x] / vgtb::kLightSpeed;
      }
      vgtb::SmallDeviation sd;
      timed(c, VGTB_K_SMALL, [&] {
        sd = small_block_args(c, s);
        launch_err = vgtb::launch_small_steps(c->g, c->kpts_dev, nk, c->spk, c->sinv, c->dlev[0],
                                              c->dlev[1], c->cur, c->have_prev, n, fc, ns, c->dt,
                                              c->sm_part, sd, s);
        if (c->scc) c->bar_count += (unsigned)ns * (unsigned)nk;
      });
      if (launch_err != hipSuccess)
        return fail(c, VGTB_E_DEVICE, std::string("small-system launch: ") + hipGetErrorString(launch_err));
      timed(c, VGTB_K_REDUCE, [&] {
        vgtb::launch_reduce_steps(c->sm_part, nk, c->na, c->kw_dev, jscale, c->hist, c->step,
                                  c->hist_cap, ns, c->flag, c->scc ? c->sm_escc : nullptr, s);
      });
      c->cur ^= (ns & 1);
      c->have_prev = true;
      c->step += ns;
      done += ns;
    }
    HIP_TRY(c, hipGetLastError());
    return VGTB_OK;
  }
  if (c->cn) {
    if (c->ctr_step != c->step) {
      vgtb::launch_set_counter(c->ctr, c->step, s);
      c->ctr_step = c->step;
    }
    for (int64_t it = 0; it < n_steps; ++it) {
      fill_ring(c, c->step, 1);
      enqueue_step_cn(c, s);
      c->step += 1;
      c->ctr_step += 1;
    }
    HIP_TRY(c, hipGetLastError());
    return VGTB_OK;
  }
  // Per-step path.  Every step's launches are the same (the kernels read the
  // step index and A(t)/c from the device), so pairs of steps are replayed from
  // graphs captured once per leapfrog parity; the forward-Euler first step and
  // the steps that end in a rescale are launched directly.
  if (c->ctr_step != c->step) {
    vgtb::launch_set_counter(c->ctr, c->step, s);
    c->ctr_step = c->step;
  }
  const bool rescale_on = dev && c->rescale_every > 0;
  for (int64_t it = 0; it < n_steps;) {
    const int64_t stp = c->step;
    fill_ring(c, stp, 2);
    const bool pair = c->use_graphs && !c->profiling && c->have_prev && it + 2 <= n_steps &&
                      !(rescale_on && ((stp + 1) % c->rescale_every == 0 ||
                                       (stp + 2) % c->rescale_every == 0));
    if (pair) {
      if (!c->graph[c->cur]) {
        st = capture_pair(c, c->cur);
        if (st != VGTB_OK) return st;
      }
      HIP_TRY(c, hipGraphLaunch(c->graph[c->cur], s));
      c->step += 2;
      c->ctr_step += 2;
      it += 2;
      continue;
    }
    enqueue_step(c, s, true);
    c->cur ^= 1;
    c->have_prev = true;
    c->step += 1;
    c->ctr_step += 1;
    it += 1;
    if (rescale_on && c->step % c->rescale_every == 0) {
      timed(c, VGTB_K_RESCALE, [&] {
        vgtb::launch_rescale(c->g, c->dlev[c->cur], c->dlev[c->cur ^ 1], n, nk, c->spk, c->tpart,
                             c->trace0, c->tfac, s);
      });
    }
  }
  HIP_TRY(c, hipGetLastError());
  return VGTB_OK;
}

vgtb_status vgtb_synchronize(vgtb_ctx *c) {
  vgtb_status st = check_ready(c);
  if (st != VGTB_OK) return st;
  int flag = 0, barrier_err = 0;
  HIP_TRY(c, hipMemcpyAsync(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  if (c->sm_err)
    HIP_TRY(c, hipMemcpyAsync(&barrier_err, c->sm_err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (barrier_err)
    return fail(c, VGTB_E_DEVICE, "the grid-wide barrier of the small-system SCC path timed out");
  if (flag) return fail(c, VGTB_E_NONFINITE, "non-finite trace or energy observed");
  return VGTB_OK;
}

vgtb_status vgtb_read_observables(vgtb_ctx *c, int64_t first, int64_t count, double *j,
                                  double *e, double *tr, double *q) {
  vgtb_status st = vgtb_synchronize(c);
  if (st != VGTB_OK) return st;
  if (first < 0 || count < 0 || first + count > c->step || first < c->step - c->hist_cap)
    return fail(c, VGTB_E_INVAL, "requested steps are not in the history ring");
  const int row = 5 + c->na;
  std::vector<double> ring((size_t)c->hist_cap * row);
  HIP_TRY(c, hipMemcpy(ring.data(), c->hist, sizeof(double) * ring.size(), hipMemcpyDeviceToHost));
  for (int64_t t = 0; t < count; ++t) {
    const double *r = ring.data() + (size_t)((first + t) % c->hist_cap) * row;
    if (j) for (int a = 0; a < 3; ++a) j[3 * t + a] = r[a];
    if (e) e[t] = r[3];
    if (tr) tr[t] = r[4];
    if (q) std::memcpy(q + (size_t)t * c->na, r + 5, sizeof(double) * c->na);
  }
  return VGTB_OK;
}

vgtb_status vgtb_get_density(vgtb_ctx *c, int32_t level, void *out, int on_device) {
  vgtb_status st = check_ready(c);
  if (st != VGTB_OK) return st;
  if (!c->have_density) return fail(c, VGTB_E_STATE, "no density set");
  if (level != 0 && level != 1) return fail(c, VGTB_E_INVAL, "level must be 0 or 1");
  if (level == 1 && (c->cn || !c->have_prev)) return fail(c, VGTB_E_STATE, "no previous level");
  if (!out) return fail(c, VGTB_E_INVAL, "null output");
  const size_t bytes = sizeof(double2) * (size_t)c->n * c->n * c->nk;
  if (c->cn) {
    // D = sum_s f_s C_s C_s^dag through the eigenvector-layout density kernel.
    vgtb::launch_cn_to_vectors(c->dlev[0], c->y, c->n, c->ns, c->nk, c->stream);
    double2 *dst = on_device ? static_cast<double2 *>(out) : c->w;
    vgtb::launch_density_from_vectors(c->y, c->cocc, dst, c->n, c->nk, c->stream);
    HIP_TRY(c, hipGetLastError());
    if (!on_device) HIP_TRY(c, hipMemcpyAsync(out, c->w, bytes, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return VGTB_OK;
  }
  const double2 *src = c->dlev[level == 0 ? c->cur : (c->cur ^ 1)];
  HIP_TRY(c, hipMemcpyAsync(out, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return VGTB_OK;
}

vgtb_status vgtb_get_reference_charges(vgtb_ctx *c, double *zh) {
  vgtb_status st = check_ready(c);
  if (st != VGTB_OK) return st;
  if (!zh) return fail(c, VGTB_E_INVAL, "null output");
  std::memcpy(zh, c->z_host.data(), sizeof(double) * c->na);
  return VGTB_OK;
}

namespace {
struct StateHeader {
  uint64_t magic;
  int64_t step;
  int32_t n, nk, na, precision, have_prev, pad;   // pad: reference carries a constant term
};
constexpr uint64_t kStateMagic = 0x7667746273743031ull;
}  // namespace

// Crank-Nicolson layout: header (have_prev = V_{n-1} set, pad = n_states),
// coefficients (the full nk * N * N buffer), occupations (nk * N), V_{n-1},
// Z.  Leapfrog: header, both levels, reference density, Z.
vgtb_status vgtb_state_size(const vgtb_ctx *c, size_t *bytes) {
  if (!c || !bytes) return fail(nullptr, VGTB_E_INVAL, "null argument");
  const size_t n2 = sizeof(double2) * (size_t)c->n * c->n * c->nk;
  if (c->cn)
    *bytes = sizeof(StateHeader) + n2 + sizeof(double) * ((size_t)c->nk * c->n + 2 * (size_t)c->na);
  else
    *bytes = sizeof(StateHeader) + 3 * n2 + sizeof(double) * c->na;
  return VGTB_OK;
}

vgtb_status vgtb_save_state(vgtb_ctx *c, void *buf, size_t bytes) {
  vgtb_status st = check_ready(c);
  if (st != VGTB_OK) return st;
  size_t need = 0;
  vgtb_state_size(c, &need);
  if (!buf || bytes < need) return fail(c, VGTB_E_INVAL, "state buffer too small");
  if (!c->have_density) return fail(c, VGTB_E_STATE, "no density set");
  const size_t n2 = sizeof(double2) * (size_t)c->n * c->n * c->nk;
  char *p = static_cast<char *>(buf);
  if (c->cn) {
    StateHeader h{kStateMagic + 1, c->step, c->n, c->nk, c->na, c->precision, c->have_vprev ? 1 : 0, c->ns};
    std::memcpy(p, &h, sizeof(h));
    p += sizeof(h);
    const size_t fo = sizeof(double) * (size_t)c->nk * c->n;
    HIP_TRY(c, hipMemcpyAsync(p, c->dlev[0], n2, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(p + n2, c->cocc, fo, hipMemcpyDeviceToHost, c->stream));
    if (c->scc) HIP_TRY(c, hipMemcpyAsync(p + n2 + fo, c->vprev, sizeof(double) * c->na, hipMemcpyDeviceToHost, c->stream));
    else std::memset(p + n2 + fo, 0, sizeof(double) * c->na);
    std::memcpy(p + n2 + fo + sizeof(double) * c->na, c->z_host.data(), sizeof(double) * c->na);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return VGTB_OK;
  }
  StateHeader h{kStateMagic, c->step, c->n, c->nk, c->na, c->precision, c->have_prev ? 1 : 0,
                c->m0_active ? 1 : 0};
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  HIP_TRY(c, hipMemcpyAsync(p, c->dlev[c->cur], n2, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(p + n2, c->dlev[c->cur ^ 1], n2, hipMemcpyDeviceToHost, c->stream));
  if (c->d0) HIP_TRY(c, hipMemcpyAsync(p + 2 * n2, c->d0, n2, hipMemcpyDeviceToHost, c->stream));
  else std::memset(p + 2 * n2, 0, n2);
  std::memcpy(p + 3 * n2, c->z_host.data(), sizeof(double) * c->na);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return VGTB_OK;
}

vgtb_status vgtb_load_state(vgtb_ctx *c, const void *buf, size_t bytes) {
  vgtb_status st = check_ready(c);
  if (st != VGTB_OK) return st;
  size_t need = 0;
  vgtb_state_size(c, &need);
  if (!buf || bytes < need) return fail(c, VGTB_E_INVAL, "state buffer too small");
  StateHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (h.magic != kStateMagic + (c->cn ? 1 : 0) || h.n != c->n || h.nk != c->nk || h.na != c->na ||
      h.precision != c->precision)
    return fail(c, VGTB_E_INVAL, "state does not match this context");
  const size_t n2 = sizeof(double2) * (size_t)c->n * c->n * c->nk;
  const char *p = static_cast<const char *>(buf) + sizeof(h);
  if (c->cn) {
    if (h.pad < 1 || h.pad > c->n) return fail(c, VGTB_E_INVAL, "state does not match this context");
    const size_t fo = sizeof(double) * (size_t)c->nk * c->n;
    HIP_TRY(c, hipMemcpyAsync(c->dlev[0], p, n2, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->cocc, p + n2, fo, hipMemcpyHostToDevice, c->stream));
    if (c->scc) HIP_TRY(c, hipMemcpyAsync(c->vprev, p + n2 + fo, sizeof(double) * c->na, hipMemcpyHostToDevice, c->stream));
    std::memcpy(c->z_host.data(), p + n2 + fo + sizeof(double) * c->na, sizeof(double) * c->na);
    HIP_TRY(c, hipMemcpyAsync(c->z, c->z_host.data(), sizeof(double) * c->na, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->step = h.step;
    c->ns = h.pad;
    c->have_vprev = h.have_prev != 0;
    c->have_density = true;
    c->have_prev = false;
    return VGTB_OK;
  }
  c->cur = 0;
  HIP_TRY(c, hipMemcpyAsync(c->dlev[0], p, n2, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->dlev[1], p + n2, n2, hipMemcpyHostToDevice, c->stream));
  if (c->d0) HIP_TRY(c, hipMemcpyAsync(c->d0, p + 2 * n2, n2, hipMemcpyHostToDevice, c->stream));
  std::memcpy(c->z_host.data(), p + 3 * n2, sizeof(double) * c->na);
  HIP_TRY(c, hipMemcpyAsync(c->z, c->z_host.data(), sizeof(double) * c->na, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->step = h.step;
  c->have_prev = h.have_prev != 0;
  c->have_density = true;
  c->m0_active = false;
  if (c->d0) {
    // Rebuild C0 (and m0 for a non-stationary reference): same kernels, same bits.
    prepare_reference(c, h.pad != 0);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  return VGTB_OK;
}

vgtb_status vgtb_profile_enable(vgtb_ctx *c, int enable) {
  vgtb_status st = check_ready(c);
  if (st != VGTB_OK) return st;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (auto &e : c->ev_pending) c->ev_free.push_back({e.a, e.b});
  c->ev_pending.clear();
  for (int i = 0; i < VGTB_K_COUNT; ++i) {
    c->prof_ms[i] = 0.0;
    c->prof_n[i] = 0;
  }
  c->profiling = enable != 0;
  return VGTB_OK;
}

vgtb_status vgtb_profile_read(vgtb_ctx *c, int32_t kernel, double *ms, int64_t *launches) {
  vgtb_status st = check_ready(c);
  if (st != VGTB_OK) return st;
  if (kernel < 0 || kernel >= VGTB_K_COUNT) return fail(c, VGTB_E_INVAL, "unknown kernel class");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (auto &e : c->ev_pending) {
    float t = 0.0f;
    HIP_TRY(c, hipEventElapsedTime(&t, e.a, e.b));
    c->prof_ms[e.id] += t;
    c->prof_n[e.id] += 1;
    c->ev_free.push_back({e.a, e.b});
  }
  c->ev_pending.clear();
  if (ms) *ms = c->prof_ms[kernel];
  if (launches) *launches = c->prof_n[kernel];
  return VGTB_OK;
}

vgtb_status vgtb_spectrum(vgtb_ctx *c, int64_t n_t, const double *j, double dt, int64_t n_w,
                          const double *omega, double e0, double tau0, int subtract_mean,
                          void *sigma_out, void *eps_out) {
  vgtb_status st = check_ready(c);
  if (st != VGTB_OK) return st;
  if (n_t < 2 || n_w < 1 || !j || !omega || !(std::fabs(e0) > 0.0) || !(tau0 > 0.0) ||
      !std::isfinite(dt) || n_t > (int64_t)1 << 30 || n_w > (int64_t)1 << 24)
    return fail(c, VGTB_E_INVAL, "bad spectrum arguments");
  for (int64_t i = 0; i < n_w; ++i)
    if (!(std::fabs(omega[i]) > 0.0)) return fail(c, VGTB_E_INVAL, "frequencies must be nonzero");
  // Device scratch: the FP64 product buffer (n_k * N * N complex) is unused
  // between steps; the trace and the grid stream through it in chunks.
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const size_t cap = 2 * std::max<size_t>((size_t)c->n * c->n * c->nk, 2048);
  const hipError_t e = vgtb::spectrum_chunked(reinterpret_cast<double *>(c->y), cap,
                                              c->stream, n_t, j, dt, n_w, omega, e0, tau0,
                                              subtract_mean != 0, sigma_out, eps_out);
  if (e != hipSuccess) return fail(c, VGTB_E_DEVICE, std::string("spectrum: ") + hipGetErrorString(e));
  return VGTB_OK;
}

int64_t vgtb_step_index(const vgtb_ctx *c) { return c ? c->step : -1; }

const char *vgtb_last_error(const vgtb_ctx *c) { return c ? c->err.c_str() : g_global_err; }

void vgtb_destroy(vgtb_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto &e : c->ev_pending) c->ev_free.push_back({e.a, e.b});
  for (auto &e : c->ev_free) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  if (c->blas) rocblas_destroy_handle(c->blas);
  drop_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

vgtb_status vgtb_autotune(vgtb_ctx *c, int32_t reps, vgtb_tuning *out) {
  vgtb_status st = check_ready(c);
  if (st != VGTB_OK) return st;
  if (reps < 1) return fail(c, VGTB_E_INVAL, "reps must be >= 1");
  if (!c->have_density) return fail(c, VGTB_E_STATE, "vgtb_autotune before a density was set");
  HIP_TRY(c, hipSetDevice(c->device));
  vgtb_tuning t{};
  t.spmm_variant = c->spmm_variant;
  t.gemm_tile = c->gemm_tile;
  if (c->small_path || c->cn) {   // no tuned variant on these paths
    if (out) *out = t;
    return VGTB_OK;
  }
  const int n = c->n, nk = c->nk;
  const bool dev = c->precision != VGTB_FP64;
  const int fmt = product_format(c);
  hipStream_t s = c->stream;
  // The candidates of one kernel are timed in interleaved rounds (each launch
  // between its own events), so that a drift of the clock during the
  // measurement does not favour the ones timed first; the mean over rounds is
  // kept.  A candidate replaces the first one (the current choice) only when it
  // is at least 1% faster: closer than that, the timings are noise.
  std::vector<hipEvent_t> ev;
  auto time_all = [&](int count, auto &&launch, double *ms) -> vgtb_status {
    ev.assign((size_t)2 * count * reps, nullptr);
    vgtb_status rs = VGTB_OK;
    for (auto &e : ev) {
      const hipError_t he = hipEventCreate(&e);
      if (he != hipSuccess) {
        rs = fail(c, VGTB_E_DEVICE, std::string("hipEventCreate: ") + hipGetErrorString(he));
        break;
      }
    }
    for (int i = 0; rs == VGTB_OK && i < count; ++i) launch(i);   // warm-up (code load, caches)
    for (int r = 0; rs == VGTB_OK && r < reps; ++r)
      for (int i = 0; i < count; ++i) {
        hipEvent_t *e = &ev[(size_t)2 * (r * count + i)];
        if (hipEventRecord(e[0], s) != hipSuccess) rs = VGTB_E_DEVICE;
        launch(i);
        if (hipEventRecord(e[1], s) != hipSuccess) rs = VGTB_E_DEVICE;
      }
    if (rs == VGTB_OK && hipStreamSynchronize(s) != hipSuccess) rs = VGTB_E_DEVICE;
    for (int i = 0; rs == VGTB_OK && i < count; ++i) {
      double sum = 0.0;
      for (int r = 0; r < reps; ++r) {
        float el = 0.f;
        hipEvent_t *e = &ev[(size_t)2 * (r * count + i)];
        if (hipEventElapsedTime(&el, e[0], e[1]) != hipSuccess) rs = VGTB_E_DEVICE;
        sum += el;
      }
      ms[i] = sum / reps;
    }
    for (auto &e : ev)
      if (e) (void)hipEventDestroy(e);
    if (rs == VGTB_E_DEVICE && c->err.empty()) fail(c, rs, "vgtb_autotune: event timing failed");
    return rs;
  };
  auto pick = [](const std::vector<int> &cand, const double *ms, int &choice) {
    int best = 0;
    for (size_t i = 1; i < cand.size(); ++i)
      if (ms[i] < ms[best]) best = (int)i;
    choice = (ms[best] < 0.99 * ms[0]) ? cand[(size_t)best] : cand[0];
  };
  // Operands: H_k at A = 0 and the current level (only scratch buffers are written).
  vgtb::launch_assemble(c->g, c->kpts_dev, nk, vgtb::StepSource{nullptr, nullptr}, c->spk,
                        c->scc ? c->v : nullptr, c->hq, c->h0k, c->ppk, s);
  const double2 *dcur = c->dlev[c->cur];
  // Candidates, the current choice first.
  std::vector<int> sv;
  if (c->g.norb == 4) sv = {-1, -2, -4, -11, -12, -14};
  if (c->g.group_size <= 8) {
    sv.push_back(1);
    sv.push_back(2);
  }
  auto cur_sv = std::find(sv.begin(), sv.end(), c->spmm_variant);
  if (cur_sv != sv.end()) std::rotate(sv.begin(), cur_sv, cur_sv + 1);
  std::vector<double> sms(sv.size(), 0.0);
  st = time_all((int)sv.size(), [&](int i) {
    if (dev) launch_deviation_spmm(c, dcur, fmt, sv[(size_t)i], s);
    else vgtb::launch_spmm(c->g, dcur, nullptr, n, nk, c->hq, nullptr, c->w, 0, c->np, nullptr,
                           sv[(size_t)i], s);
  }, sms.data());
  if (st != VGTB_OK) return st;
  for (size_t i = 0; i < sv.size() && t.n_spmm < 8; ++i) {
    t.spmm_candidates[t.n_spmm] = sv[i];
    t.spmm_ms[t.n_spmm++] = sms[i];
  }
  pick(sv, sms.data(), t.spmm_variant);
  std::vector<int> gv;
  if (fmt >= 2) {
    gv.push_back(1);
    if (c->np % 128 == 0) gv.insert(gv.end(), {2, 3, 4, 5});
  } else {
    gv = {1, 2, 3};
  }
  // The current tile first (0, the size rule, counts as the tile it picks).
  const int cur_tile = c->gemm_tile != 0 ? c->gemm_tile
                                         : (fmt >= 2 ? vgtb::split16_default_tile(c->np)
                                                     : vgtb::zgemm_default_tile(n));
  auto cur_gv = std::find(gv.begin(), gv.end(), cur_tile);
  if (cur_gv != gv.end()) std::rotate(gv.begin(), cur_gv, cur_gv + 1);
  std::vector<double> gms(gv.size(), 0.0);
  st = time_all((int)gv.size(), [&](int i) {
    if (fmt == 0) vgtb::launch_zgemm_f64(c->sinv, c->w, c->y, n, nk, s, gv[(size_t)i]);
    else launch_reduced_product(c, fmt, gv[(size_t)i], s);
  }, gms.data());
  if (st != VGTB_OK) return st;
  for (size_t i = 0; i < gv.size() && t.n_gemm < 8; ++i) {
    t.gemm_candidates[t.n_gemm] = gv[i];
    t.gemm_ms[t.n_gemm++] = gms[i];
  }
  pick(gv, gms.data(), t.gemm_tile);
  HIP_TRY(c, hipGetLastError());
  const bool new_spmm = c->spmm_variant != t.spmm_variant;
  c->spmm_variant = t.spmm_variant;
  c->gemm_tile = t.gemm_tile;
  drop_graphs(c);   // captured steps name the previous kernels
  // C0 = H0 D0 again with the chosen sparse product, whose rounding may differ:
  // a stationary density then still gives W = H D - C0 = 0 exactly.
  if (new_spmm && c->d0) {
    prepare_reference(c, c->m0_active);
    HIP_TRY(c, hipGetLastError());
  }
  if (out) *out = t;
  return VGTB_OK;
}

vgtb_status vgtb_zgemm(const void *a, const void *b, void *cc, int32_t n, int32_t batch,
                       void *stream) {
  if (!a || !b || !cc || n <= 0 || batch <= 0) return fail(nullptr, VGTB_E_INVAL, "bad zgemm arguments");
  vgtb::launch_zgemm_f64(static_cast<const double2 *>(a), static_cast<const double2 *>(b),
                         static_cast<double2 *>(cc), n, batch, static_cast<hipStream_t>(stream));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(nullptr, VGTB_E_DEVICE, hipGetErrorString(e));
  return VGTB_OK;
}


// ---------------------------------------------------------------------------
// Several small systems stepped in one launch per block of steps.
// ---------------------------------------------------------------------------
struct vgtb_group {
  std::vector<vgtb_ctx *> ctx;
  int device = 0, no = 0, form = 0, n_wg = 0;
  bool scc = false;
  hipStream_t stream = nullptr;            // the first context's stream
  static constexpr int kSlots = 4;         // blocks in flight before the host waits
  size_t jobs_off = 0, map_off = 0, field_off = 0, slot_bytes = 0;
  char *host = nullptr;                    // pinned staging, kSlots * slot_bytes
  char *dev = nullptr;                     // device copy of the slots
  hipEvent_t slot_ev[kSlots] = {};
  bool slot_used[kSlots] = {};
  int next = 0;
  hipEvent_t join = nullptr;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static vgtb_status group_fail(vgtb_group *g, vgtb_status st, const std::string &msg) {
  if (g && (st == VGTB_E_DEVICE || st == VGTB_E_NONFINITE))
    for (vgtb_ctx *c : g->ctx) fail(c, st, msg);
  set_global_err(msg.c_str());
  return st;
}

#define GROUP_HIP(g, expr)                                                                 \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess)                                                                  \
      return group_fail(g, VGTB_E_DEVICE, std::string(#expr " failed: ") + hipGetErrorString(_e)); \
  } while (0)

vgtb_status vgtb_group_create(vgtb_ctx *const *ctxs, int32_t n_ctx, vgtb_group **out) {
  if (!ctxs || !out || n_ctx < 1 || n_ctx > 4096)
    return fail(nullptr, VGTB_E_INVAL, "vgtb_group_create: needs 1 to 4096 contexts and an output handle");
  *out = nullptr;
  std::vector<vgtb_ctx *> v(ctxs, ctxs + n_ctx);
  for (vgtb_ctx *c : v) {
    if (!c) return fail(nullptr, VGTB_E_INVAL, "vgtb_group_create: null context");
    if (c->poisoned) return fail(nullptr, VGTB_E_STATE, "vgtb_group_create: a context is poisoned");
  }
  std::vector<vgtb_ctx *> sorted = v;
  std::sort(sorted.begin(), sorted.end());
  if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
    return fail(nullptr, VGTB_E_INVAL, "vgtb_group_create: a context appears twice");
  const vgtb_ctx *c0 = v[0];
  int n_wg = 0;
  for (const vgtb_ctx *c : v) {
    if (!c->small_path)
      return fail(nullptr, VGTB_E_INVAL,
                  "vgtb_group_create: every context must be on the small-system path "
                  "(N <= 40, Peierls, leapfrog, small path not switched off)");
    if (c->device != c0->device || c->no != c0->no || c->precision != c0->precision || c->scc != c0->scc)
      return fail(nullptr, VGTB_E_INVAL,
                  "vgtb_group_create: contexts differ in device, orbitals per atom, precision form "
                  "or the SCC term");
    n_wg += c->nk;
  }
  if (hipSetDevice(c0->device) != hipSuccess)
    return fail(nullptr, VGTB_E_DEVICE, "vgtb_group_create: hipSetDevice failed");
  const int form = product_format(c0);
  if (c0->scc) {
    const int cap = vgtb::small_group_max_workgroups(c0->no, form);
    if (n_wg > cap)
      return fail(nullptr, VGTB_E_INVAL,
                  "vgtb_group_create: with the SCC term the systems' k-points together (" +
                      std::to_string(n_wg) + ") must fit the GPU at once (" + std::to_string(cap) + ")");
  } else if (n_wg > 65535) {
    return fail(nullptr, VGTB_E_INVAL, "vgtb_group_create: more than 65535 k-points in all");
  }
  auto *g = new vgtb_group;
  g->ctx = v;
  g->device = c0->device;
  g->no = c0->no;
  g->form = form;
  g->scc = c0->scc;
  g->n_wg = n_wg;
  g->stream = c0->stream;
  g->jobs_off = 0;
  g->map_off = align256(sizeof(vgtb::SmallJob) * v.size());
  g->field_off = g->map_off + align256(sizeof(int) * (size_t)n_wg);
  g->slot_bytes = g->field_off + align256(sizeof(double) * 3 * vgtb::kSmallChunk * v.size());
  const size_t total = g->slot_bytes * vgtb_group::kSlots;
  hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&g->host), total, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&g->dev), total);
  for (int i = 0; e == hipSuccess && i < vgtb_group::kSlots; ++i)
    e = hipEventCreateWithFlags(&g->slot_ev[i], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&g->join, hipEventDisableTiming);
  if (e != hipSuccess) {
    const std::string m = std::string("vgtb_group_create: ") + hipGetErrorString(e);
    vgtb_group_destroy(g);
    return fail(nullptr, e == hipErrorOutOfMemory ? VGTB_E_NOMEM : VGTB_E_DEVICE, m);
  }
  // Workgroup -> system map: the same in every slot.
  for (int slot = 0; slot < vgtb_group::kSlots; ++slot) {
    int *map = reinterpret_cast<int *>(g->host + slot * g->slot_bytes + g->map_off);
    int w = 0;
    for (size_t j = 0; j < v.size(); ++j)
      for (int k = 0; k < v[j]->nk; ++k) map[w++] = (int)j;
  }
  *out = g;
  return VGTB_OK;
}

vgtb_status vgtb_group_step(vgtb_group *g, int64_t n_steps) {
  if (!g) return fail(nullptr, VGTB_E_INVAL, "null group");
  if (n_steps < 0) return fail(nullptr, VGTB_E_INVAL, "vgtb_group_step: negative step count");
  for (vgtb_ctx *c : g->ctx) {
    if (c->poisoned) return fail(nullptr, VGTB_E_STATE, "vgtb_group_step: a context is poisoned");
    if (!c->have_density) return fail(nullptr, VGTB_E_STATE, "vgtb_group_step: a context has no density");
  }
  if (n_steps == 0) return VGTB_OK;
  GROUP_HIP(g, hipSetDevice(g->device));
  hipStream_t s = g->stream;
  // Each context's earlier work comes first.
  for (vgtb_ctx *c : g->ctx) {
    if (c->stream == s) continue;
    GROUP_HIP(g, hipEventRecord(g->join, c->stream));
    GROUP_HIP(g, hipStreamWaitEvent(s, g->join, 0));
  }
  const size_t nj = g->ctx.size();
  for (int64_t done = 0; done < n_steps;) {
    const int ns = (int)std::min<int64_t>(vgtb::kSmallChunk, n_steps - done);
    const int slot = g->next;
    g->next = (g->next + 1) % vgtb_group::kSlots;
    if (g->slot_used[slot]) GROUP_HIP(g, hipEventSynchronize(g->slot_ev[slot]));
    char *hs = g->host + slot * g->slot_bytes;
    char *ds = g->dev + slot * g->slot_bytes;
    auto *jobs = reinterpret_cast<vgtb::SmallJob *>(hs + g->jobs_off);
    auto *fields = reinterpret_cast<double *>(hs + g->field_off);
    int wg0 = 0;
    for (size_t j = 0; j < nj; ++j) {
      vgtb_ctx *c = g->ctx[j];
      vgtb::SmallJob J;
      J.g = c->g;
      J.kpts = c->kpts_dev;
      J.spk = c->spk;
      J.sinv = c->sinv;
      J.dlev0 = c->dlev[0];
      J.dlev1 = c->dlev[1];
      J.field = reinterpret_cast<const double *>(ds + g->field_off) + j * 3 * vgtb::kSmallChunk;
      J.part = c->sm_part;
      J.dev = small_block_args(c, s);
      J.kw = c->kw_dev;
      J.jscale = -1.0 / c->volume;
      J.dt = c->dt;
      J.hist = c->hist;
      J.step0 = c->step;
      J.flag = c->flag;
      J.cap = c->hist_cap;
      J.cur = c->cur;
      J.have_prev = c->have_prev ? 1 : 0;
      J.n = c->n;
      J.nk = c->nk;
      J.na = c->na;
      J.wg0 = wg0;
      wg0 += c->nk;
      std::memcpy(&jobs[j], &J, sizeof(J));
      const int64_t nf = (int64_t)(c->field.size() / 3);
      double *fj = fields + j * 3 * vgtb::kSmallChunk;
      for (int i = 0; i < ns; ++i) {
        const double *a = c->field.data() + 3 * std::min<int64_t>(c->step + i, nf - 1);
        for (int x = 0; x < 3; ++x) fj[3 * i + x] = a[x] / vgtb::kLightSpeed;
      }
    }
    GROUP_HIP(g, hipMemcpyAsync(ds, hs, g->slot_bytes, hipMemcpyHostToDevice, s));
    const hipError_t e = vgtb::launch_small_group(
        reinterpret_cast<const vgtb::SmallJob *>(ds + g->jobs_off),
        reinterpret_cast<const int *>(ds + g->map_off), (int)nj, g->n_wg, g->no, g->form, g->scc, ns, s);
    if (e != hipSuccess)
      return group_fail(g, VGTB_E_DEVICE, std::string("small-system group launch: ") + hipGetErrorString(e));
    GROUP_HIP(g, hipEventRecord(g->slot_ev[slot], s));
    g->slot_used[slot] = true;
    for (vgtb_ctx *c : g->ctx) {
      c->cur ^= (ns & 1);
      c->have_prev = true;
      c->step += ns;
      if (c->scc) c->bar_count += (unsigned)ns * (unsigned)c->nk;
    }
    done += ns;
  }
  // Each context's later work waits for the group's.
  GROUP_HIP(g, hipEventRecord(g->join, s));
  for (vgtb_ctx *c : g->ctx)
    if (c->stream != s) GROUP_HIP(g, hipStreamWaitEvent(c->stream, g->join, 0));
  return VGTB_OK;
}

void vgtb_group_destroy(vgtb_group *g) {
  if (!g) return;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  for (hipEvent_t &e : g->slot_ev)
    if (e) (void)hipEventDestroy(e);
  if (g->join) (void)hipEventDestroy(g->join);
  if (g->dev) (void)hipFree(g->dev);
  if (g->host) (void)hipHostFree(g->host);
  delete g;
}

}  // extern "C"
