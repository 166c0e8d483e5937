// Host side of libmlc: argument checking, geometry tables, workspace layout and the
// launch sequence of one correction step.  No arithmetic of the method runs here:
// every step of Algorithms 4.1/4.2 is a kernel on the caller's stream.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mlc.h"
#include "mlc_launch.h"

int64_t item_bytes_fp64(int cw, int ch, int m);
int64_t item_bytes_mixed(int cw, int ch, int m);

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct SubBox {
  int id;          // sy * sub_x + sx
  int D[4];        // x0, x1, y0, y1 (coarse cells)
  int Om[4];
};

// Geometry derived from a problem description (host tables only).
struct Geometry {
  int L = 0, q = 0, nc = 0, nH = 0, kind = 0, domain = 0;
  double side = 1.0;
  std::vector<int> bx, by;
  std::vector<SubBox> subs;              // kept subdomains
  std::vector<int> coarse_nodes, coarse_index;
  std::vector<TileItem> items;           // order shared by every level
  std::vector<int> sub_item;             // (sub_x*sub_y)*q -> item, -1 dropped
  std::vector<int64_t> inv_off;          // per kept subdomain (doubles)
  int64_t inv_total = 0;

  int64_t N(int l) const { return (int64_t)nc << l; }
  int64_t nodes(int l) const { return (N(l) + 1) * (N(l) + 1); }
};

bool is_dof_host(int domain, int N, int gx, int gy) {
  if (gx <= 0 || gy <= 0 || gx >= N || gy >= N) return false;
  if (domain == 1 && gx >= N / 2 && gy <= N / 2) return false;
  return true;
}

mlc_status build_geometry(const mlc_problem_desc* d, const mlc_solver_opts* o, Geometry& g,
                          std::string& msg) {
  if (!d || !o) {
    msg = "null descriptor or options";
    return MLC_EINVAL;
  }
  if (d->domain != 0 && d->domain != 1) { msg = "domain must be 0 or 1"; return MLC_EINVAL; }
  if (d->coef_kind < 0 || d->coef_kind > 2) { msg = "coef_kind must be 0, 1 or 2"; return MLC_EINVAL; }
  if (d->n_coarse < 2 || d->n_coarse > 4096) { msg = "n_coarse must be in 2..4096"; return MLC_EINVAL; }
  if (d->domain == 1 && (d->n_coarse & 1)) { msg = "the L-shape needs an even n_coarse"; return MLC_EINVAL; }
  if (d->n_refine < 1 || d->n_refine > MLC_MAX_LEVELS) { msg = "n_refine must be in 1..10"; return MLC_EINVAL; }
  if ((int64_t)d->n_coarse << d->n_refine > 32768) { msg = "finest grid above 32768 cells per side"; return MLC_EINVAL; }
  if (d->sub_x < 1 || d->sub_x > d->n_coarse || d->sub_y < 1 || d->sub_y > d->n_coarse) {
    msg = "sub_x and sub_y must be in 1..n_coarse";
    return MLC_EINVAL;
  }
  if (d->overlap < 1 || d->overlap > d->n_coarse) { msg = "overlap must be in 1..n_coarse"; return MLC_EINVAL; }
  if (d->n_eig < 1 || d->n_eig > MLC_MAX_Q) { msg = "n_eig must be in 1..8"; return MLC_EINVAL; }
  if (o->precision != 0 && o->precision != 1) { msg = "precision must be 0 or 1"; return MLC_EINVAL; }
  if (!(o->rtol > 0.0 && o->rtol < 1.0)) { msg = "rtol must be in (0,1)"; return MLC_EINVAL; }
  if (o->max_it < 1 || o->nu < 1 || o->nu > 8 || !(o->omega > 0.0 && o->omega < 1.0)) {
    msg = "max_it >= 1, nu in 1..8, omega in (0,1) required";
    return MLC_EINVAL;
  }
  if (o->precision == 1 && (o->max_refine < 1 || !(o->inner_rtol > 0.0 && o->inner_rtol < 1.0))) {
    msg = "mixed precision needs max_refine >= 1 and inner_rtol in (0,1)";
    return MLC_EINVAL;
  }
  if (o->block != 0 && o->block != 256 && o->block != 512 && o->block != 1024) {
    msg = "block must be 0, 256, 512 or 1024";
    return MLC_EINVAL;
  }
  g.L = d->n_refine;
  g.q = d->n_eig;
  g.nc = d->n_coarse;
  g.kind = d->coef_kind;
  g.domain = d->domain;
  g.side = d->domain == 0 ? 1.0 : 2.0;
  const int nc = g.nc;
  if (g.kind != 0) {
    if (!d->kappa) { msg = "kappa is NULL"; return MLC_EINVAL; }
    const int64_t n = g.kind == 1 ? (int64_t)nc * nc : g.N(g.L) * g.N(g.L);
    for (int64_t i = 0; i < n; ++i) {
      const double k = d->kappa[i];
      if (!(k > 0.0) || !std::isfinite(k)) { msg = "kappa must be positive and finite"; return MLC_EINVAL; }
    }
  }
  // coarse dofs
  g.coarse_index.assign((size_t)(nc + 1) * (nc + 1), -1);
  for (int j = 0; j <= nc; ++j)
    for (int i = 0; i <= nc; ++i)
      if (is_dof_host(g.domain, nc, i, j)) {
        g.coarse_index[(size_t)j * (nc + 1) + i] = (int)g.coarse_nodes.size();
        g.coarse_nodes.push_back(j * (nc + 1) + i);
      }
  g.nH = (int)g.coarse_nodes.size();
  if (g.q > g.nH) { msg = "n_eig exceeds the number of coarse interior nodes"; return MLC_EINVAL; }
  if ((int64_t)g.nH * (1 + 3 * g.q) > 8192) { msg = "coarse space too large for the device Rayleigh-Ritz solve"; return MLC_EINVAL; }
  // subdomains (Section 4): D_j blocks, Omega_j = D_j grown by `overlap` coarse cells
  for (int b = 0; b <= d->sub_x; ++b) g.bx.push_back((b * nc) / d->sub_x);
  for (int b = 0; b <= d->sub_y; ++b) g.by.push_back((b * nc) / d->sub_y);
  const int ov = d->overlap;
  for (int sy = 0; sy < d->sub_y; ++sy)
    for (int sx = 0; sx < d->sub_x; ++sx) {
      SubBox s;
      s.id = sy * d->sub_x + sx;
      s.D[0] = g.bx[sx]; s.D[1] = g.bx[sx + 1];
      s.D[2] = g.by[sy]; s.D[3] = g.by[sy + 1];
      if (g.domain == 1 && s.D[0] >= nc / 2 && s.D[3] <= nc / 2) continue;  // in the removed quadrant
      s.Om[0] = std::max(0, s.D[0] - ov); s.Om[1] = std::min(nc, s.D[1] + ov);
      s.Om[2] = std::max(0, s.D[2] - ov); s.Om[3] = std::min(nc, s.D[3] + ov);
      const int cw = s.Om[1] - s.Om[0], ch = s.Om[3] - s.Om[2];
      if ((cw - 1) * (ch - 1) > MLC_MAX_TILE_COARSE) {
        msg = "a subdomain has more than 64 coarse interior nodes (use more subdomains)";
        return MLC_EINVAL;
      }
      g.subs.push_back(s);
    }
  if (d->sub_x * d->sub_y * 3 > MLC_MAX_CAND * MLC_MAX_CAND * 1000) { msg = "too many subdomains"; return MLC_EINVAL; }
  // candidate bound of the gluing kernel: blocks reaching a node along one axis
  {
    auto max_cand = [&](const std::vector<int>& b) {
      int best = 0;
      for (int t = 0; t <= 2 * nc; ++t) {  // half-cell resolution is enough to find maxima
        int c = 0;
        for (size_t k = 0; k + 1 < b.size(); ++k)
          if (2 * b[k] - 2 * ov < t && t < 2 * b[k + 1] + 2 * ov) ++c;
        best = std::max(best, c);
      }
      return best;
    };
    if (max_cand(g.bx) > MLC_MAX_CAND || max_cand(g.by) > MLC_MAX_CAND) {
      msg = "overlap too wide for the subdomain width (more than 8 overlapping blocks)";
      return MLC_EINVAL;
    }
  }
  // items: every kept subdomain x every eigenpair, largest tiles first
  std::vector<SubBox> order = g.subs;
  std::stable_sort(order.begin(), order.end(), [](const SubBox& a, const SubBox& b) {
    return (a.Om[1] - a.Om[0]) * (a.Om[3] - a.Om[2]) > (b.Om[1] - b.Om[0]) * (b.Om[3] - b.Om[2]);
  });
  g.sub_item.assign((size_t)d->sub_x * d->sub_y * g.q, -1);
  std::vector<int64_t> inv_of_id((size_t)d->sub_x * d->sub_y, -1);
  for (const SubBox& s : g.subs) {
    const int n = (s.Om[1] - s.Om[0] - 1) * (s.Om[3] - s.Om[2] - 1);
    inv_of_id[s.id] = g.inv_total;
    g.inv_total += (int64_t)n * n;
  }
  for (const SubBox& s : order)
    for (int i = 0; i < g.q; ++i) {
      TileItem it;
      std::memset(&it, 0, sizeof(it));
      it.prob = 0;
      it.sub = s.id;
      it.rhs = i;
      it.cx0 = s.Om[0];
      it.cy0 = s.Om[2];
      it.cw = s.Om[1] - s.Om[0];
      it.ch = s.Om[3] - s.Om[2];
      it.inv_off = inv_of_id[s.id];
      g.sub_item[(size_t)s.id * g.q + i] = (int)g.items.size();
      g.items.push_back(it);
    }
  return MLC_OK;
}

// Workspace layout: byte offsets from the workspace base.
struct Layout {
  size_t prob, bx, by, sub_item, coarse_nodes, coarse_index, kH;
  size_t kLR[MLC_MAX_LEVELS + 1], kUL[MLC_MAX_LEVELS + 1];
  size_t u[2], lam, ubar, res, ut, rchain, Kc, Mc, Lam, E, info, fg, partials, rr_x, rr_y, rr_t,
      cH, out_parts, stats, inv, store;
  size_t items[MLC_MAX_LEVELS + 1];
  int64_t rchain_off[MLC_MAX_LEVELS + 1];
  std::vector<std::vector<int64_t>> item_off;  // [m][item] byte offsets within store
  size_t store_bytes = 0;
  size_t total = 0;
};

void plan_layout(const Geometry& g, int precision, Layout& Lo) {
  size_t p = 0;
  auto take = [&](size_t bytes) {
    const size_t at = p;
    p = align_up(p + std::max<size_t>(bytes, 1));
    return at;
  };
  const size_t q = (size_t)g.q;
  const size_t nnL = (size_t)g.nodes(g.L);
  const size_t ncs = (size_t)(g.nc + 1) * (g.nc + 1);
  const size_t nsub = g.sub_item.size() / q;
  Lo.prob = take(sizeof(ProbDev));
  Lo.bx = take(g.bx.size() * 4);
  Lo.by = take(g.by.size() * 4);
  Lo.sub_item = take(nsub * q * 4);
  Lo.coarse_nodes = take((size_t)g.nH * 4);
  Lo.coarse_index = take(ncs * 4);
  Lo.kH = take((size_t)g.nc * g.nc * 8);
  for (int l = 0; l <= g.L; ++l) {
    Lo.kLR[l] = Lo.kUL[l] = 0;
    if (g.kind == 2) {
      const size_t c = (size_t)(g.N(l) * g.N(l)) * 8;
      Lo.kLR[l] = take(c);
      Lo.kUL[l] = (l == g.L) ? Lo.kLR[l] : take(c);
    }
  }
  Lo.u[0] = take(q * nnL * 8);
  Lo.u[1] = take(q * nnL * 8);
  Lo.lam = take(2 * MLC_MAX_Q * 8);
  Lo.ubar = take(q * nnL * 8);
  Lo.res = take(q * nnL * 8);
  Lo.ut = take(q * nnL * 8);
  int64_t rc = 0;
  for (int l = 0; l < g.L; ++l) {
    Lo.rchain_off[l] = rc;
    rc += (int64_t)(2 * q * g.nodes(l));
  }
  Lo.rchain_off[g.L] = rc;
  Lo.rchain = take((size_t)rc * 8);
  const size_t nH = (size_t)g.nH;
  Lo.Kc = take(nH * nH * 8);
  Lo.Mc = take(nH * nH * 8);
  Lo.Lam = take(nH * 8);
  Lo.E = take(nH * 8);
  Lo.info = take(4);
  Lo.fg = take(2 * q * nH * 8);
  const size_t nblk = (nnL + 255) / 256;
  Lo.partials = take(nblk * (2 * q * q + q) * 8);
  Lo.rr_x = take(q * (nH + q) * 8);
  Lo.rr_y = take(q * nH * 8);
  Lo.rr_t = take(q * q * 8);
  Lo.cH = take(q * ncs * 8);
  Lo.out_parts = take(64 * q * 8);
  Lo.stats = take(g.items.size() * sizeof(ItemStat));
  Lo.inv = take((size_t)g.inv_total * 8);
  for (int m = 0; m <= g.L; ++m) Lo.items[m] = take(g.items.size() * sizeof(TileItem));
  Lo.item_off.assign(g.L + 1, std::vector<int64_t>(g.items.size(), 0));
  size_t sb = 0;
  for (int m = 1; m <= g.L; ++m) {
    size_t o = 0;
    for (size_t k = 0; k < g.items.size(); ++k) {
      Lo.item_off[m][k] = (int64_t)o;
      const TileItem& it = g.items[k];
      const int64_t b = precision == 0 ? item_bytes_fp64(it.cw, it.ch, m)
                                       : item_bytes_mixed(it.cw, it.ch, m);
      o = align_up(o + (size_t)b);
    }
    sb = std::max(sb, o);
  }
  Lo.store_bytes = sb;
  Lo.store = take(sb);
  Lo.total = p;
}

}  // namespace

struct mlc_ctx {
  mlc_problem_desc d{};
  mlc_solver_opts o{};
  std::vector<double> kappa;
  Geometry g;
  Layout lo;
  hipStream_t st = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  ProbDev hp{};
  ProbDev* dprob = nullptr;
  std::vector<std::vector<TileItem>> items_lv;  // host copies uploaded per level
  int level = -1, cur = 0;
  bool setup = false, can_rewind = false;
  std::string err;
  rocblas_handle rb = nullptr;
  std::vector<hipEvent_t> ev_free;
  std::vector<std::array<hipEvent_t, 4>> ev_pending;
  int nt = 1024;
};

namespace {

#define MLC_HIP(ctx, expr)                                                        \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);             \
      return MLC_EHIP;                                                            \
    }                                                                             \
  } while (0)

hipEvent_t get_event(mlc_ctx* c) {
  if (!c->ev_free.empty()) {
    hipEvent_t e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

extern "C" {

mlc_status mlc_default_opts(mlc_solver_opts* o) {
  if (!o) return MLC_EINVAL;
  o->precision = 0;
  o->rtol = 1e-12;
  o->max_it = 200;
  o->max_refine = 10;
  o->inner_rtol = 1e-5;
  o->nu = 2;
  o->omega = 0.8;
  o->block = 0;
  o->timing = 0;
  return MLC_OK;
}

mlc_status mlc_workspace_size(const mlc_problem_desc* d, const mlc_solver_opts* o, size_t* bytes) {
  if (!bytes) return MLC_EINVAL;
  Geometry g;
  std::string msg;
  mlc_status s = build_geometry(d, o, g, msg);
  if (s != MLC_OK) return s;
  Layout lo;
  plan_layout(g, o->precision, lo);
  *bytes = lo.total;
  return MLC_OK;
}

mlc_status mlc_create(const mlc_problem_desc* d, const mlc_solver_opts* o, void* ws, size_t bytes,
                      void* stream, mlc_ctx** out) {
  if (!out) return MLC_EINVAL;
  *out = nullptr;
  mlc_ctx* c = new (std::nothrow) mlc_ctx();
  if (!c) return MLC_ENOMEM;
  mlc_status s = build_geometry(d, o, c->g, c->err);
  if (s != MLC_OK) {
    std::fprintf(stderr, "mlc_create: %s\n", c->err.c_str());
    delete c;
    return s;
  }
  plan_layout(c->g, o->precision, c->lo);
  if (!ws || bytes < c->lo.total || ((uintptr_t)ws % kAlign) != 0) {
    std::fprintf(stderr, "mlc_create: workspace missing, misaligned or smaller than %zu bytes\n",
                 c->lo.total);
    delete c;
    return ws && bytes < c->lo.total ? MLC_ENOMEM : MLC_EINVAL;
  }
  c->d = *d;
  c->o = *o;
  c->st = (hipStream_t)stream;
  c->ws = (char*)ws;
  c->ws_bytes = bytes;
  c->nt = o->block ? o->block : 1024;
  const Geometry& g = c->g;
  const Layout& L = c->lo;
  char* b = c->ws;
  if (g.kind == 1) c->kappa.assign(d->kappa, d->kappa + (size_t)g.nc * g.nc);
  if (g.kind == 0) c->kappa.assign((size_t)g.nc * g.nc, 1.0);
  if (g.kind == 2) c->kappa.assign(d->kappa, d->kappa + (size_t)(g.N(g.L) * g.N(g.L)));
  ProbDev& P = c->hp;
  std::memset(&P, 0, sizeof(P));
  P.domain = g.domain;
  P.n_c = g.nc;
  P.L = g.L;
  P.q = g.q;
  P.coef_kind = g.kind;
  P.sub_x = d->sub_x;
  P.sub_y = d->sub_y;
  P.overlap = d->overlap;
  P.nH = g.nH;
  P.side = g.side;
  P.kH = (const double*)(b + L.kH);
  for (int l = 0; l <= g.L; ++l) {
    P.kLR[l] = g.kind == 2 ? (const double*)(b + L.kLR[l]) : nullptr;
    P.kUL[l] = g.kind == 2 ? (const double*)(b + L.kUL[l]) : nullptr;
  }
  P.bx = (const int32_t*)(b + L.bx);
  P.by = (const int32_t*)(b + L.by);
  P.sub_item = (const int32_t*)(b + L.sub_item);
  P.coarse_nodes = (const int32_t*)(b + L.coarse_nodes);
  P.coarse_index = (const int32_t*)(b + L.coarse_index);
  P.u[0] = (double*)(b + L.u[0]);
  P.u[1] = (double*)(b + L.u[1]);
  P.lam = (double*)(b + L.lam);
  P.ubar = (double*)(b + L.ubar);
  P.res = (double*)(b + L.res);
  P.ut = (double*)(b + L.ut);
  P.rchain = (double*)(b + L.rchain);
  for (int l = 0; l <= g.L; ++l) P.rchain_off[l] = L.rchain_off[l];
  P.Kc = (double*)(b + L.Kc);
  P.V = P.Kc;
  P.Mc = (double*)(b + L.Mc);
  P.VT = P.Mc;
  P.Lam = (double*)(b + L.Lam);
  P.fg = (double*)(b + L.fg);
  P.partials = (double*)(b + L.partials);
  P.nparts = (int)((g.nodes(g.L) + 255) / 256);
  P.rr_x = (double*)(b + L.rr_x);
  P.rr_y = (double*)(b + L.rr_y);
  P.rr_t = (double*)(b + L.rr_t);
  P.cH_grid = (double*)(b + L.cH);
  P.sum_parts = (double*)(b + L.out_parts);
  c->dprob = (ProbDev*)(b + L.prob);
  // per-level item tables (storage offsets differ per level)
  c->items_lv.assign(g.L + 1, g.items);
  for (int m = 1; m <= g.L; ++m)
    for (size_t k = 0; k < g.items.size(); ++k) c->items_lv[m][k].off = L.item_off[m][k];
  hipStream_t st = c->st;
  auto fail = [&](mlc_status e) {
    std::fprintf(stderr, "mlc_create: %s\n", c->err.c_str());
    delete c;
    return e;
  };
#define MLC_UP(dst, vec)                                                                    \
  do {                                                                                      \
    hipError_t e_ = hipMemcpyAsync(b + (dst), (vec).data(), (vec).size() * sizeof((vec)[0]), \
                                   hipMemcpyHostToDevice, st);                              \
    if (e_ != hipSuccess) {                                                                 \
      c->err = std::string("upload: ") + hipGetErrorString(e_);                             \
      return fail(MLC_EHIP);                                                                \
    }                                                                                       \
  } while (0)
  MLC_UP(L.bx, g.bx);
  MLC_UP(L.by, g.by);
  MLC_UP(L.sub_item, g.sub_item);
  MLC_UP(L.coarse_nodes, g.coarse_nodes);
  MLC_UP(L.coarse_index, g.coarse_index);
  if (g.kind == 2) {
    MLC_UP(L.kLR[g.L], c->kappa);
    const std::vector<double> ones((size_t)g.nc * g.nc, 1.0);
    MLC_UP(L.kH, ones);
    if (hipStreamSynchronize(st) != hipSuccess) return fail(MLC_EHIP);
  } else {
    MLC_UP(L.kH, c->kappa);
  }
  for (int m = 1; m <= g.L; ++m) MLC_UP(L.items[m], c->items_lv[m]);
  {
    std::vector<ProbDev> one(1, P);
    MLC_UP(L.prob, one);
    if (hipStreamSynchronize(st) != hipSuccess) {
      c->err = "stream synchronize after upload failed";
      return fail(MLC_EHIP);
    }
  }
#undef MLC_UP
  *out = c;
  return MLC_OK;
}

mlc_status mlc_coarse_setup(mlc_ctx* c) {
  if (!c) return MLC_EINVAL;
  const Geometry& g = c->g;
  const Layout& L = c->lo;
  char* b = c->ws;
  hipStream_t st = c->st;
  // coefficients on every level: children means (kind 2 only; kinds 0/1 are per coarse cell)
  if (g.kind == 2) {
    for (int l = g.L - 1; l >= 0; --l)
      MLC_HIP(c, launch_coarsen_kappa(c->hp.kLR[l + 1], c->hp.kUL[l + 1], (double*)(b + L.kLR[l]),
                                      (double*)(b + L.kUL[l]), (int)g.N(l), st));
  }
  const size_t nH = (size_t)g.nH;
  MLC_HIP(c, hipMemsetAsync(b + L.Kc, 0, nH * nH * 8, st));
  MLC_HIP(c, hipMemsetAsync(b + L.Mc, 0, nH * nH * 8, st));
  MLC_HIP(c, launch_coarse_matrices(g.kind, c->dprob, 1, g.nH, st));
  if (!c->rb) {
    if (rocblas_create_handle(&c->rb) != rocblas_status_success) {
      c->err = "rocblas_create_handle failed";
      return MLC_EHIP;
    }
  }
  if (rocblas_set_stream(c->rb, st) != rocblas_status_success) {
    c->err = "rocblas_set_stream failed";
    return MLC_EHIP;
  }
  // Algorithm 4.2 step 1 on V_0H: K_H V = M_H V Lambda, V^T M_H V = I (full spectrum)
  rocblas_status rs = rocsolver_dsygvd(c->rb, rocblas_eform_ax, rocblas_evect_original,
                                       rocblas_fill_upper, g.nH, (double*)(b + L.Kc), g.nH,
                                       (double*)(b + L.Mc), g.nH, (double*)(b + L.Lam),
                                       (double*)(b + L.E), (rocblas_int*)(b + L.info));
  if (rs != rocblas_status_success) {
    c->err = std::string("rocsolver_dsygvd: ") + rocblas_status_to_string(rs);
    return MLC_EHIP;
  }
  MLC_HIP(c, launch_transpose_v(c->dprob, 1, g.nH, st));
  MLC_HIP(c, launch_init_u0(c->dprob, 1, 0, (g.nc + 1) * (g.nc + 1), st));
  MLC_HIP(c, launch_tile_inverse(g.kind, c->dprob, (const TileItem*)(b + L.items[1]),
                                 (int)g.items.size(), (double*)(b + L.inv), st));
  MLC_HIP(c, hipStreamSynchronize(st));
  int info = 0;
  MLC_HIP(c, hipMemcpy(&info, b + L.info, 4, hipMemcpyDeviceToHost));
  if (info != 0) {
    c->err = "coarse generalized eigensolve failed (info " + std::to_string(info) + ")";
    return MLC_EHIP;
  }
  c->level = 0;
  c->cur = 0;
  c->setup = true;
  c->can_rewind = false;
  return MLC_OK;
}

static mlc_status level_correct_impl(mlc_ctx* c) {
  const Geometry& g = c->g;
  const Layout& L = c->lo;
  char* b = c->ws;
  hipStream_t st = c->st;
  const int m = c->level + 1;
  const int src = c->cur, dst = 1 - c->cur;
  const int64_t nn = g.nodes(m);
  const TileItem* items = (const TileItem*)(b + L.items[m]);
  const int nitems = (int)g.items.size();
  std::array<hipEvent_t, 4> ev{};
  const bool timing = c->o.timing != 0;
  if (timing) {
    for (auto& e : ev) {
      e = get_event(c);
      if (!e) {
        c->err = "hipEventCreate failed";
        return MLC_EHIP;
      }
    }
    MLC_HIP(c, hipEventRecord(ev[0], st));
  }
  MLC_HIP(c, launch_prolong_residual(g.kind, c->dprob, 1, m, src, nn, st));
  if (timing) MLC_HIP(c, hipEventRecord(ev[1], st));
  if (c->o.precision == 0) {
    const int64_t lds = pcg_lds_bytes(c->items_lv[m].data(), nitems, m, (int)sizeof(double));
    MLC_HIP(c, launch_local_pcg(g.kind, c->nt, c->dprob, items, nitems, b + L.store,
                                (const double*)(b + L.inv), m, (ItemStat*)(b + L.stats),
                                c->o.rtol, c->o.max_it, c->o.nu, c->o.omega, lds, st));
  } else {
    MLC_HIP(c, launch_local_mixed(g.kind, c->nt, c->dprob, items, nitems, b + L.store,
                                  (const double*)(b + L.inv), m, (ItemStat*)(b + L.stats),
                                  c->o.rtol, c->o.max_it, c->o.max_refine, c->o.inner_rtol,
                                  c->o.nu, c->o.omega, st));
  }
  if (timing) MLC_HIP(c, hipEventRecord(ev[2], st));
  MLC_HIP(c, launch_pou_glue(c->dprob, 1, items, b + L.store, m, nn, st));
  MLC_HIP(c, launch_rr_apply(g.kind, c->dprob, 1, m, nn, st));
  for (int l = m - 1; l >= 0; --l) MLC_HIP(c, launch_restrict(c->dprob, 1, l, m, g.nodes(l), st));
  MLC_HIP(c, launch_rr_project(c->dprob, 1, g.nH, st));
  MLC_HIP(c, launch_rr_solve(g.q, c->dprob, 1, m, g.nH, dst, st));
  MLC_HIP(c, launch_rr_combine(c->dprob, 1, (g.nc + 1) * (g.nc + 1), st));
  MLC_HIP(c, launch_assemble(c->dprob, 1, m, dst, nn, st));
  if (timing) {
    MLC_HIP(c, hipEventRecord(ev[3], st));
    c->ev_pending.push_back(ev);
  }
  c->cur = dst;
  c->level = m;
  c->can_rewind = true;
  return MLC_OK;
}

mlc_status mlc_level_correct(mlc_ctx* c, mlc_level_stats* stt) {
  if (!c) return MLC_EINVAL;
  if (!c->setup || c->level < 0 || c->level >= c->g.L) {
    c->err = "level_correct needs coarse_setup and a level below the finest";
    return MLC_ESTATE;
  }
  mlc_status s = level_correct_impl(c);
  if (s != MLC_OK || !stt) return s;
  const Geometry& g = c->g;
  MLC_HIP(c, hipStreamSynchronize(c->st));
  std::vector<ItemStat> is(g.items.size());
  MLC_HIP(c, hipMemcpy(is.data(), c->ws + c->lo.stats, is.size() * sizeof(ItemStat),
                       hipMemcpyDeviceToHost));
  double lam[2 * MLC_MAX_Q];
  MLC_HIP(c, hipMemcpy(lam, c->ws + c->lo.lam, sizeof(lam), hipMemcpyDeviceToHost));
  std::memset(stt, 0, sizeof(*stt));
  const int m = c->level;
  stt->level = m;
  stt->n_items = (int)g.items.size();
  stt->h = g.side / (double)g.N(m);
  int64_t ndof = 0;
  const int N = (int)g.N(m);
  for (int j = 1; j < N; ++j)
    for (int i = 1; i < N; ++i) ndof += is_dof_host(g.domain, N, i, j) ? 1 : 0;
  stt->n_dofs = ndof;
  for (size_t k = 0; k < g.items.size(); ++k) {
    const TileItem& it = g.items[k];
    const int64_t S = (int64_t)(it.cw * (1 << m) - 1) * (it.ch * (1 << m) - 1);
    stt->n_tile_dofs += S;
    stt->it_max = std::max(stt->it_max, is[k].iters);
    stt->refine_max = std::max(stt->refine_max, is[k].refine);
    stt->it_sum += is[k].iters;
    stt->it_dofs += (int64_t)is[k].iters * S;
    stt->refine_dofs += (int64_t)is[k].refine * S;
    stt->relres_max = std::max(stt->relres_max, is[k].relres);
  }
  for (int i = 0; i < g.q; ++i) stt->lambda[i] = lam[c->cur * MLC_MAX_Q + i];
  if (stt->relres_max > c->o.rtol * 1.0000001) {
    c->err = "a local solve did not converge within max_it";
    return MLC_ENOCONV;
  }
  return MLC_OK;
}

mlc_status mlc_run(mlc_ctx* c) {
  if (!c) return MLC_EINVAL;
  if (!c->setup) return MLC_ESTATE;
  while (c->level < c->g.L) {
    mlc_status s = level_correct_impl(c);
    if (s != MLC_OK) return s;
  }
  return MLC_OK;
}

mlc_status mlc_rewind(mlc_ctx* c) {
  if (!c) return MLC_EINVAL;
  if (!c->setup || !c->can_rewind || c->level < 1) {
    c->err = "nothing to rewind";
    return MLC_ESTATE;
  }
  c->cur = 1 - c->cur;
  c->level -= 1;
  c->can_rewind = false;
  return MLC_OK;
}

mlc_status mlc_current_level(const mlc_ctx* c, int32_t* level) {
  if (!c || !level) return MLC_EINVAL;
  *level = c->level;
  return MLC_OK;
}

mlc_status mlc_get_eigenpairs(mlc_ctx* c, double* lam_host, double* u_dev) {
  if (!c) return MLC_EINVAL;
  if (!c->setup) {
    c->err = "no eigenpairs before coarse_setup";
    return MLC_ESTATE;
  }
  const Geometry& g = c->g;
  if (u_dev) {
    MLC_HIP(c, launch_output_signed(c->hp.u[c->cur], g.nodes(c->level), g.q,
                                    (double*)(c->ws + c->lo.out_parts), u_dev, c->st));
  }
  if (lam_host) {
    MLC_HIP(c, hipStreamSynchronize(c->st));
    MLC_HIP(c, hipMemcpy(lam_host, c->ws + c->lo.lam + (size_t)c->cur * MLC_MAX_Q * 8,
                         (size_t)g.q * 8, hipMemcpyDeviceToHost));
  }
  return MLC_OK;
}

mlc_status mlc_set_state(mlc_ctx* c, int32_t level, const double* lam_host, const double* u_dev) {
  if (!c || !lam_host || !u_dev) return MLC_EINVAL;
  if (!c->setup) {
    c->err = "set_state needs coarse_setup";
    return MLC_ESTATE;
  }
  if (level < 0 || level > c->g.L) {
    c->err = "level out of range";
    return MLC_EINVAL;
  }
  MLC_HIP(c, launch_set_state(c->dprob, level, 0, u_dev, c->g.nodes(level), c->st));
  MLC_HIP(c, hipStreamSynchronize(c->st));
  MLC_HIP(c, hipMemcpy(c->ws + c->lo.lam, lam_host, (size_t)c->g.q * 8, hipMemcpyHostToDevice));
  c->level = level;
  c->cur = 0;
  c->can_rewind = false;
  return MLC_OK;
}

mlc_status mlc_phase_times(mlc_ctx* c, double* ms, int32_t n) {
  if (!c || !ms || n < 1) return MLC_EINVAL;
  MLC_HIP(c, hipStreamSynchronize(c->st));
  double acc[2] = {0.0, 0.0};
  for (auto& ev : c->ev_pending) {
    float a = 0.f, t = 0.f;
    MLC_HIP(c, hipEventElapsedTime(&a, ev[1], ev[2]));
    MLC_HIP(c, hipEventElapsedTime(&t, ev[0], ev[3]));
    acc[0] += a;
    acc[1] += t;
    for (auto e : ev) c->ev_free.push_back(e);
  }
  c->ev_pending.clear();
  for (int i = 0; i < n; ++i) ms[i] = i < 2 ? acc[i] : 0.0;
  return MLC_OK;
}

mlc_status mlc_destroy(mlc_ctx* c) {
  if (!c) return MLC_EINVAL;
  if (c->st) (void)hipStreamSynchronize(c->st);
  for (auto& ev : c->ev_pending)
    for (auto e : ev) c->ev_free.push_back(e);
  for (auto e : c->ev_free) (void)hipEventDestroy(e);
  if (c->rb) rocblas_destroy_handle(c->rb);
  delete c;
  return MLC_OK;
}

const char* mlc_status_str(mlc_status s) {
  switch (s) {
    case MLC_OK: return "MLC_OK";
    case MLC_EINVAL: return "MLC_EINVAL";
    case MLC_ENOMEM: return "MLC_ENOMEM";
    case MLC_EHIP: return "MLC_EHIP";
    case MLC_ENOCONV: return "MLC_ENOCONV";
    case MLC_ESTATE: return "MLC_ESTATE";
  }
  return "MLC_UNKNOWN";
}

const char* mlc_last_error(const mlc_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
