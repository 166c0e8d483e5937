// Host side of libmlc: argument checking, geometry tables, workspace layout and the
// launch sequence of a correction step.  No arithmetic of the method runs here: every
// step of Algorithms 4.1/4.2 is a kernel on the caller's stream.
//
// Every context is a batch of independent problems (a single-problem context is a batch
// of one).  Per problem the workspace holds its grids and coarse data; the local-solve
// item tables, the subdomain -> item maps and the local-solve storage are per level step
// and shared by all problems, so one launch per kernel serves the whole batch.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <array>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <sys/stat.h>
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
hipError_t launch_p2_prolong_residual(int kind, const ProbDev* probs, int nprob, int m, int src,
                                      int64_t max_nodes, int max_q, hipStream_t s);
hipError_t launch_p2_rr_apply(int kind, const ProbDev* probs, int nprob, int m, int64_t max_nodes,
                              int max_q, hipStream_t s);
hipError_t launch_p2_restrict(const ProbDev* probs, int nprob, int l, int m, int64_t max_nodes_l,
                              int max_q, hipStream_t s);
hipError_t launch_p2_assemble(const ProbDev* probs, int nprob, int m, int dst, int64_t max_nodes,
                              int max_q, hipStream_t s);
hipError_t launch_p2_coarse_matrices(int kind, const ProbDev* probs, int nprob, int max_nH,
                                     hipStream_t s);
hipError_t launch_local_p2(int kind, int nt, const ProbDev* probs, const TileItem* items,
                           int nitems, char* store, const double* inv, int m, ItemStat* stats,
                           double rtol, int max_it, int nu, double omega, double omega2,
                           int max_tile_nx, hipStream_t s);

namespace {

constexpr size_t kAlign = 256;
constexpr int kGlueMaxIt = 1000;  // eager G_{m+1} CG: iteration cap (MLC_ENOCONV beyond)

// Damping of the first and second sweep of each smoothing pair of the local solves'
// V-cycle.  smoother 1 with nu = 2: the reciprocals of the roots of the degree-2
// Chebyshev polynomial of [1/2, 2], the part of the spectrum of D^-1 K that the coarse
// grid does not reduce (D^-1 K lies in (0, 2] for these stencils, rows summing to zero off
// the boundary), so the pair damps it by at most 1/T_2(5/3) = 0.22 instead of the 0.36 of
// two sweeps at 0.8; otherwise (smoother 0, or nu != 2) omega for every sweep.
void sweep_weights(const mlc_solver_opts& o, int nu, double* w1, double* w2) {
  if (o.smoother == 1 && nu == 2) {
    const double c = 1.25, d = 0.75 / std::sqrt(2.0);
    *w1 = 1.0 / (c - d);
    *w2 = 1.0 / (c + d);
  } else {
    *w1 = *w2 = o.omega;
  }
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct SubBox {
  int id;    // sy * sub_x + sx
  int D[4];  // x0, x1, y0, y1 (coarse cells)
  int Om[4];
};

// Geometry derived from one problem description (host tables only).
struct Geometry {
  int L = 0, q = 0, nc = 0, nH = 0, kind = 0, domain = 0, sub_x = 1, sub_y = 1, overlap = 1, pou = 0;
  int order = 1;  // element degree: level-l vectors live on the grid of nc 2^(l+order-1) intervals
  double side = 1.0;
  std::vector<int> bx, by;
  std::vector<SubBox> subs;     // kept subdomains, largest first
  std::vector<int> coarse_nodes, coarse_index;
  std::vector<int64_t> inv_off; // per kept subdomain (doubles, relative to the problem)
  int64_t inv_total = 0;
  int64_t cells(int l) const { return (int64_t)nc << l; }  // mesh cells per side
  int64_t N(int l) const { return (int64_t)nc << (l + order - 1); }  // node-grid intervals
  int64_t nodes(int l) const { return (N(l) + 1) * (N(l) + 1); }
  int per_coarse(int l) const { return order << l; }  // node-grid intervals per coarse cell
};

bool is_dof_host(int domain, int N, int gx, int gy) {
  if (gx <= 0 || gy <= 0 || gx >= N || gy >= N) return false;
  if (domain == 1 && gx >= N / 2 && gy <= N / 2) return false;
  return true;
}

mlc_status check_opts(const mlc_solver_opts* o, std::string& msg) {
  if (!o) { msg = "null options"; return MLC_EINVAL; }
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
  if (o->smoother != 0 && o->smoother != 1) {
    msg = "smoother must be 0 (damped Jacobi) or 1 (Chebyshev weights)";
    return MLC_EINVAL;
  }
  if (o->glue_graph_it < 1 || o->glue_graph_it > 1000) {
    msg = "glue_graph_it must be in 1..1000";
    return MLC_EINVAL;
  }
  return MLC_OK;
}

mlc_status build_geometry(const mlc_problem_desc* d, Geometry& g, std::string& msg) {
  if (!d) { msg = "null descriptor"; return MLC_EINVAL; }
  if (d->domain < 0 || d->domain > 2) { msg = "domain must be 0, 1 or 2"; return MLC_EINVAL; }
  if (d->coef_kind < 0 || d->coef_kind > 3) { msg = "coef_kind must be 0, 1, 2 or 3"; return MLC_EINVAL; }
  if (d->n_coarse < 2 || d->n_coarse > 4096) { msg = "n_coarse must be in 2..4096"; return MLC_EINVAL; }
  if (d->domain == 1 && (d->n_coarse & 1)) { msg = "the L-shape needs an even n_coarse"; return MLC_EINVAL; }
  if (d->n_refine < 1 || d->n_refine > MLC_MAX_LEVELS) { msg = "n_refine must be in 1..10"; return MLC_EINVAL; }
  if ((int64_t)d->n_coarse << d->n_refine > 32768) { msg = "finest grid above 32768 cells per side"; return MLC_EINVAL; }
  if (d->sub_x < 1 || d->sub_x > d->n_coarse || d->sub_y < 1 || d->sub_y > d->n_coarse) {
    msg = "sub_x and sub_y must be in 1..n_coarse";
    return MLC_EINVAL;
  }
  if (d->pou < MLC_POU_RAMP || d->pou > MLC_POU_INTERFACE) { msg = "pou must be 0, 1 or 2"; return MLC_EINVAL; }
  if (d->overlap < (d->pou == MLC_POU_RAMP ? 1 : 0) || d->overlap > d->n_coarse) {
    msg = "overlap must be in 1..n_coarse (0..n_coarse unless the gluing is the ramp)";
    return MLC_EINVAL;
  }
  if (d->n_eig < 1 || d->n_eig > MLC_MAX_Q) { msg = "n_eig must be in 1..8"; return MLC_EINVAL; }
  const int order = d->order == 0 ? 1 : d->order;
  if (order != 1 && order != 2) { msg = "order must be 0, 1 or 2"; return MLC_EINVAL; }
  if (order == 2 && (d->coef_kind > 1 || d->pou == MLC_POU_INTERFACE)) {
    msg = "P2 elements need coef_kind 0 or 1 and a partition-of-unity gluing";
    return MLC_EINVAL;
  }
  if ((int64_t)d->n_coarse << (d->n_refine + order - 1) > 32768) {
    msg = "finest node grid above 32768 intervals per side";
    return MLC_EINVAL;
  }
  g.order = order;
  g.L = d->n_refine;
  g.q = d->n_eig;
  g.nc = d->n_coarse;
  g.kind = d->coef_kind;
  g.domain = d->domain;
  g.sub_x = d->sub_x;
  g.sub_y = d->sub_y;
  g.overlap = d->overlap;
  g.pou = d->pou;
  g.side = d->domain == 0 ? 1.0 : 2.0;
  const int nc = g.nc;
  if (g.kind == 1 || g.kind == 2) {
    if (!d->kappa) { msg = "kappa is NULL"; return MLC_EINVAL; }
    const int64_t n = g.kind == 1 ? (int64_t)nc * nc : g.cells(g.L) * g.cells(g.L);
    for (int64_t i = 0; i < n; ++i) {
      const double k = d->kappa[i];
      if (!(k > 0.0) || !std::isfinite(k)) { msg = "kappa must be positive and finite"; return MLC_EINVAL; }
    }
  }
  if (g.kind == 3) {  // per finest triangle: A symmetric positive definite, phi > 0
    if (!d->kappa) { msg = "kappa is NULL"; return MLC_EINVAL; }
    const int64_t n = 2 * g.cells(g.L) * g.cells(g.L);
    const double* a11 = d->kappa;
    const double* a12 = d->kappa + n;
    const double* a22 = d->kappa + 2 * n;
    const double* phi = d->kappa + 3 * n;
    for (int64_t i = 0; i < n; ++i) {
      const bool ok = std::isfinite(a11[i]) && std::isfinite(a12[i]) && std::isfinite(a22[i]) &&
                      std::isfinite(phi[i]) && a11[i] > 0.0 && a22[i] > 0.0 &&
                      a11[i] * a22[i] - a12[i] * a12[i] > 0.0 && phi[i] > 0.0;
      if (!ok) { msg = "coef_kind 3 needs finite values, A positive definite and phi > 0 on every triangle"; return MLC_EINVAL; }
    }
  }
  // coarse dofs: the interior nodes of the level-0 node grid (the mesh nodes for P1, the
  // vertices and edge midpoints for P2)
  const int n0 = (int)g.N(0);
  g.coarse_index.assign((size_t)(n0 + 1) * (n0 + 1), -1);
  for (int j = 0; j <= n0; ++j)
    for (int i = 0; i <= n0; ++i)
      if (is_dof_host(g.domain, n0, i, j)) {
        g.coarse_index[(size_t)j * (n0 + 1) + i] = (int)g.coarse_nodes.size();
        g.coarse_nodes.push_back(j * (n0 + 1) + i);
      }
  g.nH = (int)g.coarse_nodes.size();
  if (g.q > g.nH) { msg = "n_eig exceeds the number of coarse interior nodes"; return MLC_EINVAL; }
  // the device Rayleigh-Ritz solve keeps Lambda, Z, f, g and the q eigenvectors of the
  // reduced problem in LDS: n_H (1 + 4 q) + q^2 doubles, at most 144 KiB of the 160 KiB
  if ((int64_t)g.nH * (1 + 4 * g.q) + g.q * g.q > 18432) {
    msg = "coarse space too large for the device Rayleigh-Ritz solve";
    return MLC_EINVAL;
  }
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
      if (cw < 2 || ch < 2) {
        msg = "every Omega_j must span at least 2 coarse cells each way (more overlap or fewer subdomains)";
        return MLC_EINVAL;
      }
      if ((cw - 1) * (ch - 1) > MLC_MAX_TILE_COARSE_ALL) {
        msg = "a subdomain has more than 1024 coarse interior nodes (use more subdomains)";
        return MLC_EINVAL;
      }
      g.subs.push_back(s);
    }
  // candidate bound of the gluing kernel: blocks reaching a node along one axis
  auto max_cand = [&](const std::vector<int>& b) {
    int best = 0;
    for (int t = 0; t <= 2 * nc; ++t) {  // half-cell resolution finds the maxima
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
  std::stable_sort(g.subs.begin(), g.subs.end(), [](const SubBox& a, const SubBox& b) {
    return (a.Om[1] - a.Om[0]) * (a.Om[3] - a.Om[2]) > (b.Om[1] - b.Om[0]) * (b.Om[3] - b.Om[2]);
  });
  for (const SubBox& s : g.subs) {
    const int n = (s.Om[1] - s.Om[0] - 1) * (s.Om[3] - s.Om[2] - 1);
    g.inv_off.push_back(g.inv_total);
    g.inv_total += (int64_t)n * n;
  }
  return MLC_OK;
}

// Byte offsets (from the workspace base) of one problem's buffers.
struct ProbLayout {
  size_t bx, by, coarse_nodes, coarse_index, kH, u[2], lam, ubar, res, ut, rchain, Kc, Mc, Lam,
      E, info, fg, partials, rr_y, rr_t, rr_ab, cH, out_parts, skel, skel_parts, skel_scal,
      skel_rec;
  size_t kLR[MLC_MAX_LEVELS + 1], kUL[MLC_MAX_LEVELS + 1];
  size_t st7[MLC_MAX_LEVELS + 1], st7f[MLC_MAX_LEVELS + 1], coef3;  // coef kind 3: stencil
                                                                     // planes, input
  int64_t rchain_off[MLC_MAX_LEVELS + 1];
  int64_t eig_off = -1;  // bytes into the local-solve store: device eigensolver scratch (setup)
  int64_t inv_base;      // doubles, into the batch inverse region
  int32_t sub_item_off;  // into every step's subdomain -> item table
};

// One level step of the batch: its local solves and where their storage lives.
struct StepTables {
  std::vector<TileItem> items;
  std::vector<int32_t> sub_item;
  size_t items_off = 0, sub_item_off = 0;
  int64_t max_nodes = 0;         // largest (N_s+1)^2 among the active problems
  int32_t max_tile_nx = 0;       // widest tile row (interior nodes) among the items
  std::vector<int64_t> nodes_l;  // per coarser level l < s: largest (N_l+1)^2
};

// Forward tape and reverse-sweep buffers (single problem, q = 1): per level m the
// eigenvector, u~, the local corrections e_j (item order) and the Rayleigh-Ritz data
// (c_H, c_u, f, g, alpha, beta, mu); per level the triangle adjoints; grid scratch.
struct TapeLayout {
  bool on = false;
  size_t tu[MLC_MAX_LEVELS + 1], tut[MLC_MAX_LEVELS + 1], te[MLC_MAX_LEVELS + 1],
      te_off[MLC_MAX_LEVELS + 1], trr[MLC_MAX_LEVELS + 1];
  size_t klo[MLC_MAX_LEVELS + 1], kup[MLC_MAX_LEVELS + 1];
  size_t adj_u, adj_next, utbar, shat, rbar, ubar, cbar_H, scal, ycoef, coef, parts, a0, e0, ygrid,
      v0grid;
  std::vector<std::vector<int64_t>> te_offsets;  // per level, per item (doubles)
};

struct Plan {
  TapeLayout tape;
  std::vector<Geometry> geo;
  std::vector<ProbLayout> pl;
  std::vector<StepTables> steps;  // index s (1..Lmax); steps[0] unused
  int n = 0, q = 0, kind = 0, order = 1, Lmax = 0, max_nH = 0, max_nc1sq = 0, precision = 0;
  size_t probdev = 0, stats = 0, conv = 0, inv = 0, store = 0, store_bytes = 0, total = 0;
  int64_t max_items = 0, inv_total = 0;
};

mlc_status make_plan(int32_t n, const mlc_problem_desc* descs, const mlc_solver_opts* o, Plan& P,
                     std::string& msg) {
  if (n < 1 || !descs) { msg = "need at least one problem"; return MLC_EINVAL; }
  mlc_status st = check_opts(o, msg);
  if (st != MLC_OK) return st;
  P.n = n;
  P.precision = o->precision;
  P.geo.resize(n);
  for (int i = 0; i < n; ++i) {
    st = build_geometry(&descs[i], P.geo[i], msg);
    if (st != MLC_OK) {
      if (n > 1) msg = "problem " + std::to_string(i) + ": " + msg;
      return st;
    }
  }
  P.q = P.geo[0].q;
  P.kind = P.geo[0].kind;
  P.order = P.geo[0].order;
  for (const Geometry& g : P.geo) {
    if (g.q != P.q || g.kind != P.kind || g.order != P.order) {
      msg = "all problems of a batch need the same n_eig, coef_kind and order";
      return MLC_EINVAL;
    }
    if (g.order == 2 && (o->precision != 0 || o->record_tape)) {
      msg = "P2 elements run in FP64 without a tape";
      return MLC_EINVAL;
    }
    if (g.pou == MLC_POU_INTERFACE && (n != 1 || o->record_tape)) {
      msg = "the interface gluing runs on single-problem contexts without a tape";
      return MLC_EINVAL;
    }
    P.Lmax = std::max(P.Lmax, g.L);
    P.max_nH = std::max(P.max_nH, g.nH);
    P.max_nc1sq = std::max(P.max_nc1sq, (int)g.nodes(0));
  }
  size_t p = 0;
  auto take = [&](size_t bytes) {
    const size_t at = p;
    p = align_up(p + std::max<size_t>(bytes, 1));
    return at;
  };
  const size_t q = (size_t)P.q;
  P.probdev = take((size_t)n * sizeof(ProbDev));
  P.pl.resize(n);
  int32_t sub_off = 0;
  for (int i = 0; i < n; ++i) {
    const Geometry& g = P.geo[i];
    ProbLayout& L = P.pl[i];
    const size_t nnL = (size_t)g.nodes(g.L);
    const size_t ncs = (size_t)g.nodes(0);
    L.bx = take(g.bx.size() * 4);
    L.by = take(g.by.size() * 4);
    L.coarse_nodes = take((size_t)g.nH * 4);
    L.coarse_index = take(ncs * 4);
    L.kH = take((size_t)g.nc * g.nc * 8);
    for (int l = 0; l <= MLC_MAX_LEVELS; ++l) L.kLR[l] = L.kUL[l] = L.st7[l] = L.st7f[l] = 0;
    L.coef3 = 0;
    if (g.kind == 2)
      for (int l = 0; l <= g.L; ++l) {
        const size_t c = (size_t)(g.cells(l) * g.cells(l)) * 8;
        L.kLR[l] = take(c);
        L.kUL[l] = (l == g.L) ? L.kLR[l] : take(c);
      }
    if (g.kind == 3) {
      L.coef3 = take((size_t)(8 * g.cells(g.L) * g.cells(g.L)) * 8);
      for (int l = 0; l <= g.L; ++l) {
        L.st7[l] = take((size_t)(7 * g.nodes(l)) * 8);
        L.st7f[l] = take((size_t)(3 * g.nodes(l)) * 4);
      }
    }
    L.u[0] = take(q * nnL * 8);
    L.u[1] = take(q * nnL * 8);
    L.lam = take(2 * MLC_MAX_Q * 8);
    L.ubar = take(q * nnL * 8);
    L.res = take(q * nnL * 8);
    L.ut = take(q * nnL * 8);
    int64_t rc = 0;
    for (int l = 0; l <= g.L; ++l) {
      L.rchain_off[l] = rc;
      if (l < g.L) rc += (int64_t)(2 * q * g.nodes(l));
    }
    L.rchain = take((size_t)rc * 8);
    const size_t nH = (size_t)g.nH;
    L.Kc = take(nH * nH * 8);
    L.Mc = take(nH * nH * 8);
    L.Lam = take(nH * 8);
    L.E = take(nH * 8);
    L.info = take(4);
    L.fg = take(2 * q * nH * 8);
    L.partials = take(((nnL + 255) / 256) * (2 * q * q + q) * 8);
    L.rr_y = take(q * nH * 8);
    L.rr_t = take(q * q * 8);
    L.rr_ab = take(2 * 8);
    L.cH = take(q * ncs * 8);
    L.out_parts = take(4 * 64 * q * 8);  // output sign partials (4 per block)
    L.skel = L.skel_parts = L.skel_scal = L.skel_rec = 0;
    if (g.pou == MLC_POU_INTERFACE) {  // vectors of the G_{m+1} problem and its V-cycle
      L.skel = take((size_t)skel_stride(g.nc, g.L) * q * 8);
      // block partials: one per 256 nodes, or per tile of 16 x 16 nodes (at least as many)
      const size_t t16 = ((size_t)g.N(g.L) + 1 + 15) / 16;
      L.skel_parts = take(t16 * t16 * 2 * q * 8);
      L.skel_scal = take(8 * q * 8);
      L.skel_rec = take((MLC_MAX_LEVELS + 1) * 2 * 8);  // per step: iterations, relres
    }
    L.inv_base = P.inv_total;
    P.inv_total += g.inv_total;
    L.sub_item_off = sub_off;
    sub_off += g.sub_x * g.sub_y * (int)q;
  }
  // per-step item tables: every active problem's subdomains x eigenpairs, largest first
  P.steps.assign(P.Lmax + 1, StepTables());
  size_t store_bytes = 0;
  // the reverse sweep runs FP64 solves in the forward pass's items, so a recorded tape
  // sizes them for FP64 whatever the forward precision
  const bool fp64_items = P.precision == 0 || o->record_tape != 0;
  for (int s = 1; s <= P.Lmax; ++s) {
    StepTables& T = P.steps[s];
    T.sub_item.assign((size_t)sub_off, -1);
    T.nodes_l.assign(s, 0);
    std::vector<TileItem> all;
    for (int i = 0; i < n; ++i) {
      const Geometry& g = P.geo[i];
      if (g.L < s) continue;
      T.max_nodes = std::max(T.max_nodes, g.nodes(s));
      for (int l = 0; l < s; ++l) T.nodes_l[l] = std::max(T.nodes_l[l], g.nodes(l));
      for (size_t k = 0; k < g.subs.size(); ++k) {
        const SubBox& sb = g.subs[k];
        for (int r = 0; r < P.q; ++r) {
          TileItem it;
          std::memset(&it, 0, sizeof(it));
          it.prob = i;
          it.sub = sb.id;
          it.rhs = r;
          it.cx0 = sb.Om[0];
          it.cy0 = sb.Om[2];
          it.cw = sb.Om[1] - sb.Om[0];
          it.ch = sb.Om[3] - sb.Om[2];
          it.inv_off = P.pl[i].inv_base + g.inv_off[k];
          all.push_back(it);
        }
      }
    }
    std::stable_sort(all.begin(), all.end(), [](const TileItem& a, const TileItem& b) {
      return a.cw * a.ch > b.cw * b.ch;
    });
    size_t o = 0;
    for (size_t k = 0; k < all.size(); ++k) {
      TileItem& it = all[k];
      it.off = (int64_t)o;
      // tiles hold the nodes of the level's node grid strictly inside Omega_j
      const int sg = s + P.order - 1;
      T.max_tile_nx = std::max(T.max_tile_nx, it.cw * (1 << sg) - 1);
      const int64_t b = fp64_items ? item_bytes_fp64(it.cw, it.ch, sg)
                                   : item_bytes_mixed(it.cw, it.ch, sg);
      o = align_up(o + (size_t)b);
      it.rhs_stride = (int32_t)(align_up((size_t)b));
      T.sub_item[(size_t)P.pl[it.prob].sub_item_off + (size_t)it.sub * P.q + it.rhs] = (int32_t)k;
    }
    // the gluing reaches right-hand side r of a subdomain at rhs_stride * r bytes from its
    // first item: the stable sort keeps a subdomain's q equally sized items adjacent
    for (size_t k = 0; k < all.size(); ++k) {
      const TileItem& it = all[k];
      const int32_t first =
          T.sub_item[(size_t)P.pl[it.prob].sub_item_off + (size_t)it.sub * P.q];
      if (first < 0 || (size_t)first + (size_t)it.rhs != k ||
          all[first].off + (int64_t)it.rhs * it.rhs_stride != it.off) {
        msg = "internal: tile items of a subdomain are not adjacent";
        return MLC_EINVAL;
      }
    }
    store_bytes = std::max(store_bytes, o);
    T.items = all;
    P.max_items = std::max<int64_t>(P.max_items, (int64_t)all.size());
    T.items_off = take(all.size() * sizeof(TileItem));
    T.sub_item_off = take(T.sub_item.size() * 4);
  }
  P.stats = take((size_t)P.max_items * sizeof(ItemStat));
  P.conv = take((MLC_MAX_LEVELS + 1) * 8);  // per step: the largest local relative residual
  P.inv = take((size_t)P.inv_total * 8);
  if (o->record_tape) {
    const Geometry& g = P.geo[0];
    if (n != 1 || P.q != 1 || (P.kind != 1 && P.kind != 2)) {
      msg = "record_tape needs a single problem with n_eig = 1 and coef_kind 1 or 2";
      return MLC_EINVAL;
    }
    TapeLayout& T = P.tape;
    T.on = true;
    T.te_offsets.assign(g.L + 1, {});
    for (int m = 1; m <= g.L; ++m) {
      T.tu[m] = take((size_t)g.nodes(m) * 8);
      T.tut[m] = take((size_t)g.nodes(m) * 8);
      int64_t o = 0;
      for (const TileItem& it : P.steps[m].items) {
        T.te_offsets[m].push_back(o);
        o += (int64_t)(it.cw * (1 << m) - 1) * (it.ch * (1 << m) - 1);
      }
      T.te[m] = take((size_t)o * 8);
      T.te_off[m] = take(P.steps[m].items.size() * 8);
      T.trr[m] = take((size_t)(3 * g.nH + 4) * 8);
    }
    for (int l = 0; l <= g.L; ++l) {
      T.klo[l] = take((size_t)(g.cells(l) * g.cells(l)) * 8);
      T.kup[l] = take((size_t)(g.cells(l) * g.cells(l)) * 8);
    }
    const size_t nnL = (size_t)g.nodes(g.L);
    T.adj_u = take(nnL * 8);
    T.adj_next = take(nnL * 8);
    T.utbar = take(nnL * 8);
    T.shat = take(nnL * 8);
    T.rbar = take(nnL * 8);
    T.ubar = take(nnL * 8);
    T.cbar_H = take((size_t)g.nH * 8);
    T.scal = take((size_t)(g.L + 8) * 8);  // [0] c_bar_u, [1..] lambda_bar per level
    T.ycoef = take((size_t)g.nH * 8);
    T.coef = take(8 * 8);
    T.parts = take(((nnL + 255) / 256) * 8);
    T.a0 = take((size_t)g.nH * 8);
    T.e0 = take((size_t)g.nH * 8);
    T.ygrid = take((size_t)(g.nc + 1) * (g.nc + 1) * 8);
    T.v0grid = take((size_t)(g.nc + 1) * (g.nc + 1) * 8);
  }
  // the device eigensolver of setup works in the local-solve store (unused until the
  // first step): eig_scratch_doubles(n_H) per problem it handles
  size_t eig_bytes = 0;
  for (int i = 0; i < n; ++i) {
    const int nH = P.geo[i].nH;
    if (nH > MLC_JACOBI_MAX_NH) continue;
    P.pl[i].eig_off = (int64_t)eig_bytes;
    eig_bytes = align_up(eig_bytes + (size_t)eig_scratch_doubles(nH) * 8);
  }
  store_bytes = std::max(store_bytes, eig_bytes);
  P.store_bytes = store_bytes;
  P.store = take(store_bytes);
  P.total = p;
  return MLC_OK;
}

}  // namespace

struct mlc_batch {
  Plan plan;
  mlc_solver_opts o{};
  std::vector<std::vector<double>> kappa;
  std::vector<ProbDev> hp;
  hipStream_t st = nullptr;
  char* ws = nullptr;
  ProbDev* dprob = nullptr;
  int step = -1;              // current step (-1 before setup)
  bool can_rewind = false;
  std::vector<int> shift;     // per problem: eigenvector buffer = (level + shift) & 1
  std::vector<int> blocks;    // workgroup size of the local solves per step (index s)
  std::vector<int> nu_s;      // damped Jacobi sweeps per step (index s)
  std::vector<double> inner_s;  // mixed precision: inner FP32 tolerance per step (index s)
  std::vector<hipGraphExec_t> graphs;  // per step
  std::vector<hipGraph_t> graph_defs;
  hipStream_t cap = nullptr;  // capture stream (the caller's may be the null stream)
  std::string err;
  rocblas_handle rb = nullptr;
  std::vector<hipEvent_t> ev_free;
  std::vector<std::array<hipEvent_t, 4>> ev_pending;
  std::vector<double> e0;  // unit coefficient vector (host copy kept for the async upload)
  bool tape_valid = false;  // every taped level comes from steps run from level 0
};

struct mlc_ctx {
  mlc_batch* b = nullptr;
};

namespace {

#define MLC_HIP(bt, expr)                                                         \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      (bt)->err = std::string(#expr) + ": " + hipGetErrorString(e_);              \
      return MLC_EHIP;                                                            \
    }                                                                             \
  } while (0)

hipEvent_t get_event(mlc_batch* c) {
  if (!c->ev_free.empty()) {
    hipEvent_t e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void drop_graphs(mlc_batch* b) {
  for (auto& g : b->graphs)
    if (g) (void)hipGraphExecDestroy(g);
  for (auto& g : b->graph_defs)
    if (g) (void)hipGraphDestroy(g);
  std::fill(b->graphs.begin(), b->graphs.end(), nullptr);
  std::fill(b->graph_defs.begin(), b->graph_defs.end(), nullptr);
}

int problem_level(const mlc_batch* b, int i) { return std::min(b->step, b->plan.geo[i].L); }

mlc_status batch_create(int32_t n, const mlc_problem_desc* descs, const mlc_solver_opts* o,
                        void* ws, size_t bytes, void* stream, mlc_batch** out) {
  if (!out) return MLC_EINVAL;
  *out = nullptr;
  mlc_batch* b = new (std::nothrow) mlc_batch();
  if (!b) return MLC_ENOMEM;
  mlc_status s = make_plan(n, descs, o, b->plan, b->err);
  if (s != MLC_OK) {
    std::fprintf(stderr, "mlc: %s\n", b->err.c_str());
    delete b;
    return s;
  }
  const Plan& P = b->plan;
  if (!ws || bytes < P.total || ((uintptr_t)ws % kAlign) != 0) {
    std::fprintf(stderr, "mlc: workspace missing, misaligned or smaller than %zu bytes\n", P.total);
    delete b;
    return ws && bytes < P.total ? MLC_ENOMEM : MLC_EINVAL;
  }
  b->o = *o;
  b->st = (hipStream_t)stream;
  b->ws = (char*)ws;
  char* w = b->ws;
  b->shift.assign(n, 0);
  b->blocks.assign(P.Lmax + 1, o->block ? o->block : 1024);
  b->nu_s.assign(P.Lmax + 1, o->nu);
  b->inner_s.assign(P.Lmax + 1, o->inner_rtol);
  b->graphs.assign(P.Lmax + 1, nullptr);
  b->graph_defs.assign(P.Lmax + 1, nullptr);
  b->kappa.resize(n);
  b->hp.resize(n);
  for (int i = 0; i < n; ++i) {
    const Geometry& g = P.geo[i];
    const ProbLayout& L = P.pl[i];
    if (g.kind == 1) b->kappa[i].assign(descs[i].kappa, descs[i].kappa + (size_t)g.nc * g.nc);
    if (g.kind == 0) b->kappa[i].assign((size_t)g.nc * g.nc, 1.0);
    if (g.kind == 2)
      b->kappa[i].assign(descs[i].kappa, descs[i].kappa + (size_t)(g.cells(g.L) * g.cells(g.L)));
    if (g.kind == 3)
      b->kappa[i].assign(descs[i].kappa, descs[i].kappa + (size_t)(8 * g.cells(g.L) * g.cells(g.L)));
    ProbDev& D = b->hp[i];
    std::memset(&D, 0, sizeof(D));
    D.domain = g.domain;
    D.n_c = g.nc;
    D.L = g.L;
    D.q = g.q;
    D.coef_kind = g.kind;
    D.sub_x = g.sub_x;
    D.sub_y = g.sub_y;
    D.overlap = g.overlap;
    D.pou = g.pou;
    D.order = g.order;
    D.Lg = g.L + g.order - 1;
    D.c1 = (int)g.N(0) + 1;
    D.nH = g.nH;
    D.side = g.side;
    D.kH = (const double*)(w + L.kH);
    for (int l = 0; l <= g.L; ++l) {
      D.kLR[l] = g.kind == 2 ? (const double*)(w + L.kLR[l]) : nullptr;
      D.kUL[l] = g.kind == 2 ? (const double*)(w + L.kUL[l]) : nullptr;
      D.st7[l] = g.kind == 3 ? (const double*)(w + L.st7[l]) : nullptr;
      D.st7f[l] = g.kind == 3 ? (const float*)(w + L.st7f[l]) : nullptr;
    }
    D.bx = (const int32_t*)(w + L.bx);
    D.by = (const int32_t*)(w + L.by);
    D.sub_item_off = L.sub_item_off;
    D.coarse_nodes = (const int32_t*)(w + L.coarse_nodes);
    D.coarse_index = (const int32_t*)(w + L.coarse_index);
    D.u[0] = (double*)(w + L.u[0]);
    D.u[1] = (double*)(w + L.u[1]);
    D.lam = (double*)(w + L.lam);
    D.ubar = (double*)(w + L.ubar);
    D.res = (double*)(w + L.res);
    D.ut = (double*)(w + L.ut);
    D.rchain = (double*)(w + L.rchain);
    for (int l = 0; l <= g.L; ++l) D.rchain_off[l] = L.rchain_off[l];
    D.Kc = (double*)(w + L.Kc);
    D.V = D.Kc;
    D.Mc = (double*)(w + L.Mc);
    D.VT = D.Mc;
    D.Lam = (double*)(w + L.Lam);
    D.fg = (double*)(w + L.fg);
    D.partials = (double*)(w + L.partials);
    D.nparts = (int)((g.nodes(g.L) + 255) / 256);
    D.rr_y = (double*)(w + L.rr_y);
    D.rr_t = (double*)(w + L.rr_t);
    D.rr_ab = (double*)(w + L.rr_ab);
    D.cH_grid = (double*)(w + L.cH);
    D.sum_parts = (double*)(w + L.out_parts);
    D.conv = (double*)(w + P.conv);
    D.eig_ws = L.eig_off >= 0 ? (double*)(w + P.store + L.eig_off) : nullptr;
    D.info = (int32_t*)(w + L.info);
  }
  b->dprob = (ProbDev*)(w + P.probdev);
  hipStream_t st = b->st;
  auto up = [&](size_t dst, const void* src, size_t nbytes) -> bool {
    return nbytes == 0 ||
           hipMemcpyAsync(w + dst, src, nbytes, hipMemcpyHostToDevice, st) == hipSuccess;
  };
  bool ok = true;
  for (int i = 0; i < n && ok; ++i) {
    const Geometry& g = P.geo[i];
    const ProbLayout& L = P.pl[i];
    ok = ok && up(L.bx, g.bx.data(), g.bx.size() * 4);
    ok = ok && up(L.by, g.by.data(), g.by.size() * 4);
    ok = ok && up(L.coarse_nodes, g.coarse_nodes.data(), g.coarse_nodes.size() * 4);
    ok = ok && up(L.coarse_index, g.coarse_index.data(), g.coarse_index.size() * 4);
    if (g.kind == 2)
      ok = ok && up(L.kLR[g.L], b->kappa[i].data(), b->kappa[i].size() * 8);
    else if (g.kind == 3)
      ok = ok && up(L.coef3, b->kappa[i].data(), b->kappa[i].size() * 8);
    else
      ok = ok && up(L.kH, b->kappa[i].data(), b->kappa[i].size() * 8);
  }
  for (int s = 1; s <= P.Lmax && ok; ++s) {
    const StepTables& T = P.steps[s];
    ok = ok && up(T.items_off, T.items.data(), T.items.size() * sizeof(TileItem));
    ok = ok && up(T.sub_item_off, T.sub_item.data(), T.sub_item.size() * 4);
  }
  if (P.tape.on) {
    for (int m = 1; m <= P.Lmax && ok; ++m)
      ok = ok && up(P.tape.te_off[m], P.tape.te_offsets[m].data(), P.tape.te_offsets[m].size() * 8);
    b->e0.assign((size_t)P.geo[0].nH, 0.0);
    b->e0[0] = 1.0;
    ok = ok && up(P.tape.e0, b->e0.data(), b->e0.size() * 8);
  }
  ok = ok && up(P.probdev, b->hp.data(), b->hp.size() * sizeof(ProbDev));
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  if (!ok) {
    std::fprintf(stderr, "mlc: upload of the geometry tables failed\n");
    delete b;
    return MLC_EHIP;
  }
  *out = b;
  return MLC_OK;
}

mlc_status batch_setup(mlc_batch* b) {
  const Plan& P = b->plan;
  char* w = b->ws;
  hipStream_t st = b->st;
  drop_graphs(b);
  for (int i = 0; i < P.n; ++i) {
    const Geometry& g = P.geo[i];
    const ProbLayout& L = P.pl[i];
    if (g.kind == 2)  // coefficients on every level: children means
      for (int l = g.L - 1; l >= 0; --l)
        MLC_HIP(b, launch_coarsen_kappa(b->hp[i].kLR[l + 1], b->hp[i].kUL[l + 1],
                                        (double*)(w + L.kLR[l]), (double*)(w + L.kUL[l]),
                                        (int)g.N(l), st));
    if (g.kind == 3) {  // seven-point stiffness and mass on every level (Galerkin products)
      const double h = g.side / (double)g.N(g.L);
      MLC_HIP(b, launch_tensor_fine((const double*)(w + L.coef3), (double*)(w + L.st7[g.L]),
                                    (float*)(w + L.st7f[g.L]), (int)g.N(g.L), h * h, st));
      for (int l = g.L - 1; l >= 0; --l)
        MLC_HIP(b, launch_galerkin7((const double*)(w + L.st7[l + 1]), (double*)(w + L.st7[l]),
                                    (float*)(w + L.st7f[l]), (int)g.N(l), st));
    }
    const size_t nH = (size_t)g.nH;
    MLC_HIP(b, hipMemsetAsync(w + L.Kc, 0, nH * nH * 8, st));
    MLC_HIP(b, hipMemsetAsync(w + L.Mc, 0, nH * nH * 8, st));
  }
  if (P.order == 2)
    MLC_HIP(b, launch_p2_coarse_matrices(P.kind, b->dprob, P.n, P.max_nH, st));
  else
    MLC_HIP(b, launch_coarse_matrices(P.kind, b->dprob, P.n, P.max_nH, st));
  // Algorithm 4.2 step 1 on V_0H: K_H V = M_H V Lambda, V^T M_H V = I (full spectrum):
  // coarse spaces up to MLC_JACOBI_MAX_NH nodes on the device, every problem of the batch
  // in one launch; larger ones by rocSOLVER (the choice depends on the problem alone, so a
  // problem's results in a batch equal those of a single run)
  MLC_HIP(b, launch_coarse_eig(b->dprob, P.n, st));
  for (int i = 0; i < P.n; ++i) {
    const Geometry& g = P.geo[i];
    const ProbLayout& L = P.pl[i];
    if (g.nH <= MLC_JACOBI_MAX_NH) continue;
    if (!b->rb && rocblas_create_handle(&b->rb) != rocblas_status_success) {
      b->err = "rocblas_create_handle failed";
      return MLC_EHIP;
    }
    if (rocblas_set_stream(b->rb, st) != rocblas_status_success) {
      b->err = "rocblas_set_stream failed";
      return MLC_EHIP;
    }
    rocblas_status rs = rocsolver_dsygvd(b->rb, rocblas_eform_ax, rocblas_evect_original,
                                         rocblas_fill_upper, g.nH, (double*)(w + L.Kc), g.nH,
                                         (double*)(w + L.Mc), g.nH, (double*)(w + L.Lam),
                                         (double*)(w + L.E), (rocblas_int*)(w + L.info));
    if (rs != rocblas_status_success) {
      b->err = std::string("rocsolver_dsygvd: ") + rocblas_status_to_string(rs);
      return MLC_EHIP;
    }
  }
  MLC_HIP(b, launch_transpose_v(b->dprob, P.n, P.max_nH, st));
  MLC_HIP(b, launch_init_u0(b->dprob, P.n, 0, P.max_nc1sq, st));
  MLC_HIP(b, launch_tile_inverse(P.kind, b->dprob, (const TileItem*)(w + P.steps[1].items_off),
                                 (int)P.steps[1].items.size(), (double*)(w + P.inv), st));
  MLC_HIP(b, hipStreamSynchronize(st));
  for (int i = 0; i < P.n; ++i) {
    int info = 0;
    MLC_HIP(b, hipMemcpy(&info, w + P.pl[i].info, 4, hipMemcpyDeviceToHost));
    if (info != 0) {
      b->err = "coarse generalized eigensolve failed (problem " + std::to_string(i) + ", info " +
               std::to_string(info) + ")";
      return MLC_EHIP;
    }
  }
  MLC_HIP(b, hipMemset(w + P.conv, 0, (MLC_MAX_LEVELS + 1) * 8));
  b->step = 0;
  b->can_rewind = false;
  b->tape_valid = true;
  std::fill(b->shift.begin(), b->shift.end(), 0);
  return MLC_OK;
}

// Enqueue one level step s (src/dst: eigenvector buffers of levels s-1 and s).
mlc_status enqueue_step(mlc_batch* b, int s, int src, int dst, bool timing, bool capture,
                        hipStream_t st) {
  const Plan& P = b->plan;
  const StepTables& T = P.steps[s];
  char* w = b->ws;
  const TileItem* items = (const TileItem*)(w + T.items_off);
  const int32_t* sub_item = (const int32_t*)(w + T.sub_item_off);
  const int nitems = (int)T.items.size();
  std::array<hipEvent_t, 4> ev{};
  if (timing) {
    for (auto& e : ev) {
      e = get_event(b);
      if (!e) {
        b->err = "hipEventCreate failed";
        return MLC_EHIP;
      }
    }
    MLC_HIP(b, hipEventRecord(ev[0], st));
  }
  const bool p2 = P.order == 2;
  if (p2)
    MLC_HIP(b, launch_p2_prolong_residual(P.kind, b->dprob, P.n, s, src, T.max_nodes, P.q, st));
  else
    MLC_HIP(b, launch_prolong_residual(P.kind, b->dprob, P.n, s, src, T.max_nodes, P.q, st));
  if (timing) MLC_HIP(b, hipEventRecord(ev[1], st));
  double w1, w2;
  sweep_weights(b->o, b->nu_s[s], &w1, &w2);
  if (p2) {
    MLC_HIP(b, launch_local_p2(P.kind, b->blocks[s], b->dprob, items, nitems, w + P.store,
                               (const double*)(w + P.inv), s, (ItemStat*)(w + P.stats),
                               b->o.rtol, b->o.max_it, b->nu_s[s], w1, w2, T.max_tile_nx, st));
  } else if (P.precision == 0) {
    MLC_HIP(b, launch_local_pcg(P.kind, b->blocks[s], b->dprob, items, nitems, w + P.store,
                                (const double*)(w + P.inv), s, (ItemStat*)(w + P.stats),
                                b->o.rtol, b->o.max_it, b->nu_s[s], w1, w2, 0, T.max_tile_nx,
                                st));
  } else {
    MLC_HIP(b, launch_local_mixed(P.kind, b->blocks[s], b->dprob, items, nitems, w + P.store,
                                  (const double*)(w + P.inv), s, (ItemStat*)(w + P.stats),
                                  b->o.rtol, b->o.max_it, b->o.max_refine, b->inner_s[s],
                                  b->nu_s[s], w1, w2, T.max_tile_nx, st));
  }
  if (timing) MLC_HIP(b, hipEventRecord(ev[2], st));
  if (P.geo[0].pou == MLC_POU_INTERFACE) {  // single problem (checked at plan time)
    const ProbLayout& L = P.pl[0];
    // eager: CG until every right-hand side has converged (flags polled every 4
    // iterations); captured: a fixed glue_graph_it iterations (converged ones frozen)
    MLC_HIP(b, run_interface_gluing(P.kind, b->dprob, items, sub_item, w + P.store, s, P.q,
                                    P.geo[0].nc, skel_stride(P.geo[0].nc, P.geo[0].L),
                                    b->o.rtol, capture ? b->o.glue_graph_it : kGlueMaxIt,
                                    !capture, (double*)(w + L.skel),
                                    (double*)(w + L.skel_parts), (double*)(w + L.skel_scal),
                                    (double*)(w + L.skel_rec) + 2 * s, st));
  } else {
    // the gluing works on the node grid (level s + order - 1 of the P1 grids)
    MLC_HIP(b, launch_pou_glue(b->dprob, P.n, items, sub_item, w + P.store, s + P.order - 1,
                               T.max_nodes, P.q, st));
  }
  if (p2) {
    MLC_HIP(b, launch_p2_rr_apply(P.kind, b->dprob, P.n, s, T.max_nodes, P.q, st));
    for (int l = s - 1; l >= 0; --l)
      MLC_HIP(b, launch_p2_restrict(b->dprob, P.n, l, s, T.nodes_l[l], P.q, st));
  } else {
    MLC_HIP(b, launch_rr_apply(P.kind, b->dprob, P.n, s, T.max_nodes, P.q, st));
    for (int l = s - 1; l >= 0; --l)
      MLC_HIP(b, launch_restrict(b->dprob, P.n, l, s, T.nodes_l[l], P.q, st));
  }
  MLC_HIP(b, launch_rr_project(b->dprob, P.n, P.max_nH, P.q, st));
  MLC_HIP(b, launch_rr_solve(P.q, b->dprob, P.n, s, P.max_nH, dst, st));
  MLC_HIP(b, launch_rr_combine(b->dprob, P.n, P.max_nc1sq, P.q, st));
  if (p2)
    MLC_HIP(b, launch_p2_assemble(b->dprob, P.n, s, dst, T.max_nodes, P.q, st));
  else
    MLC_HIP(b, launch_assemble(b->dprob, P.n, s, dst, T.max_nodes, P.q, st));
  if (P.tape.on) {  // keep this level's forward state for the reverse sweep
    const TapeLayout& TL = P.tape;
    const ProbDev& D = b->hp[0];
    const int nH = P.geo[0].nH;
    const size_t nn = (size_t)P.geo[0].nodes(s);
    double* rr = (double*)(w + TL.trr[s]);
    MLC_HIP(b, hipMemcpyAsync(w + TL.tu[s], D.u[dst], nn * 8, hipMemcpyDeviceToDevice, st));
    MLC_HIP(b, hipMemcpyAsync(w + TL.tut[s], D.ut, nn * 8, hipMemcpyDeviceToDevice, st));
    MLC_HIP(b, launch_tape_tiles(items, nitems, w + P.store, s, (double*)(w + TL.te[s]),
                                 (const int64_t*)(w + TL.te_off[s]), st));
    MLC_HIP(b, hipMemcpyAsync(rr, D.rr_y, (size_t)nH * 8, hipMemcpyDeviceToDevice, st));
    MLC_HIP(b, hipMemcpyAsync(rr + nH, D.rr_t, 8, hipMemcpyDeviceToDevice, st));
    MLC_HIP(b, hipMemcpyAsync(rr + nH + 1, D.fg, (size_t)2 * nH * 8, hipMemcpyDeviceToDevice, st));
    MLC_HIP(b, hipMemcpyAsync(rr + 3 * nH + 1, D.rr_ab, 16, hipMemcpyDeviceToDevice, st));
    MLC_HIP(b, hipMemcpyAsync(rr + 3 * nH + 3, D.lam + (size_t)dst * MLC_MAX_Q, 8,
                              hipMemcpyDeviceToDevice, st));
  }
  if (timing) {
    MLC_HIP(b, hipEventRecord(ev[3], st));
    b->ev_pending.push_back(ev);
  }
  return MLC_OK;
}

mlc_status batch_step(mlc_batch* b, int use_graph) {
  const Plan& P = b->plan;
  if (b->step < 0 || b->step >= P.Lmax) {
    b->err = "a step needs setup and a level below the finest";
    return MLC_ESTATE;
  }
  const int s = b->step + 1;
  // every problem stepping here holds level s-1 in buffer (s-1+shift)&1; the shift is
  // zero except after mlc_set_state on a single-problem context
  const int src = (s - 1 + b->shift[0]) & 1, dst = 1 - src;
  if (use_graph) {
    if (!b->graphs[s]) {
      // capture on a private stream (default priority); the instantiated graph is then
      // launched on the caller's stream, which orders it with the caller's work
      if (!b->cap) MLC_HIP(b, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
      MLC_HIP(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
      mlc_status e = enqueue_step(b, s, src, dst, false, true, b->cap);
      hipGraph_t g = nullptr;
      hipError_t he = hipStreamEndCapture(b->cap, &g);
      if (e != MLC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return e;
      }
      if (he != hipSuccess) {
        b->err = std::string("hipStreamEndCapture: ") + hipGetErrorString(he);
        return MLC_EHIP;
      }
      hipGraphExec_t ex = nullptr;
      he = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      if (he != hipSuccess) {
        (void)hipGraphDestroy(g);
        b->err = std::string("hipGraphInstantiate: ") + hipGetErrorString(he);
        return MLC_EHIP;
      }
      b->graph_defs[s] = g;
      b->graphs[s] = ex;
    }
    MLC_HIP(b, hipGraphLaunch(b->graphs[s], b->st));
  } else {
    mlc_status e = enqueue_step(b, s, src, dst, b->o.timing != 0, false, b->st);
    if (e != MLC_OK) return e;
  }
  b->step = s;
  b->can_rewind = true;
  return MLC_OK;
}

mlc_status step_stats(mlc_batch* b, mlc_level_stats* stt) {
  const Plan& P = b->plan;
  const int s = b->step;
  if (s < 1) {
    b->err = "no step has run";
    return MLC_ESTATE;
  }
  const StepTables& T = P.steps[s];
  MLC_HIP(b, hipStreamSynchronize(b->st));
  std::vector<ItemStat> is(T.items.size());
  MLC_HIP(b, hipMemcpy(is.data(), b->ws + P.stats, is.size() * sizeof(ItemStat),
                       hipMemcpyDeviceToHost));
  std::memset(stt, 0, sizeof(*stt));
  stt->level = s;
  stt->n_items = (int)T.items.size();
  for (int i = 0; i < P.n; ++i) {
    const Geometry& g = P.geo[i];
    if (g.L < s) continue;
    const int N = (int)g.N(s);
    for (int j = 1; j < N; ++j)
      for (int x = 1; x < N; ++x) stt->n_dofs += is_dof_host(g.domain, N, x, j) ? 1 : 0;
    stt->h = g.side / (double)N;
  }
  for (size_t k = 0; k < T.items.size(); ++k) {
    const TileItem& it = T.items[k];
    const int r = P.order << s;
    const int64_t S = (int64_t)(it.cw * r - 1) * (it.ch * r - 1);
    stt->n_tile_dofs += S;
    stt->it_max = std::max(stt->it_max, is[k].iters);
    stt->refine_max = std::max(stt->refine_max, is[k].refine);
    stt->it_sum += is[k].iters;
    stt->it_dofs += (int64_t)is[k].iters * S;
    stt->refine_dofs += (int64_t)is[k].refine * S;
    stt->relres_max = std::max(stt->relres_max, is[k].relres);
  }
  if (stt->relres_max > b->o.rtol * 1.0000001) {
    b->err = "a local solve did not converge within max_it";
    return MLC_ENOCONV;
  }
  if (P.geo[0].pou == MLC_POU_INTERFACE) {
    double rec[2];
    MLC_HIP(b, hipMemcpy(rec, b->ws + P.pl[0].skel_rec + 2 * s * sizeof(double), sizeof rec,
                         hipMemcpyDeviceToHost));
    stt->glue_it = (int32_t)rec[0];
    stt->glue_relres = rec[1];
    if (!(rec[1] <= b->o.rtol * 1.0000001)) {
      b->err = "the G_{m+1} problem did not converge";
      return MLC_ENOCONV;
    }
  }
  return MLC_OK;
}

mlc_status batch_get(mlc_batch* b, int i, double* lam_host, double* u_dev) {
  const Plan& P = b->plan;
  if (b->step < 0) {
    b->err = "no eigenpairs before setup";
    return MLC_ESTATE;
  }
  if (i < 0 || i >= P.n) return MLC_EINVAL;
  const Geometry& g = P.geo[i];
  const int lvl = problem_level(b, i);
  const int buf = (lvl + b->shift[i]) & 1;
  if (u_dev)
    MLC_HIP(b, launch_output_signed(b->hp[i].u[buf], g.nodes(lvl), g.q,
                                    (double*)(b->ws + P.pl[i].out_parts), u_dev, b->st));
  if (lam_host) {
    MLC_HIP(b, hipStreamSynchronize(b->st));
    MLC_HIP(b, hipMemcpy(lam_host, b->ws + P.pl[i].lam + (size_t)buf * MLC_MAX_Q * 8,
                         (size_t)g.q * 8, hipMemcpyDeviceToHost));
  }
  return MLC_OK;
}

mlc_status phase_times(mlc_batch* b, double* ms, int32_t n) {
  MLC_HIP(b, hipStreamSynchronize(b->st));
  double acc[2] = {0.0, 0.0};
  for (auto& ev : b->ev_pending) {
    float a = 0.f, t = 0.f;
    MLC_HIP(b, hipEventElapsedTime(&a, ev[1], ev[2]));
    MLC_HIP(b, hipEventElapsedTime(&t, ev[0], ev[3]));
    acc[0] += a;
    acc[1] += t;
    for (auto e : ev) b->ev_free.push_back(e);
  }
  b->ev_pending.clear();
  for (int i = 0; ms && i < n; ++i) ms[i] = i < 2 ? acc[i] : 0.0;
  return MLC_OK;
}

// ---- autotuner: per step the workgroup size, nu and (mixed precision) the inner FP32
// tolerance of the local solves; cache lines "<key> <block nu inner_rtol per step>..." ----

struct Tuning {
  int block, nu;
  double inner;
};

// The device architecture, the cache format and a hash (FNV-1a) of everything that
// decides the local-solve work of every step: element order, coefficient kind, precision,
// q, the nu and inner tolerance the batch was created with, and each item's subdomain
// shape.  Two batches with the same key launch the same work.
std::string tune_key(const mlc_batch* b) {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return std::string();
  const Plan& P = b->plan;
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int k = 0; k < 8; ++k) {
      h ^= (uint64_t)((v >> (8 * k)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  mix(P.order);
  mix(P.kind);
  mix(P.precision);
  mix(P.q);
  mix(b->o.nu);
  int64_t bits;
  std::memcpy(&bits, &b->o.inner_rtol, sizeof bits);
  mix(P.precision ? bits : 0);
  mix(P.Lmax);
  for (int s = 1; s <= P.Lmax; ++s) {
    mix((int64_t)P.steps[s].items.size());
    for (const TileItem& it : P.steps[s].items) {
      mix(it.cw);
      mix(it.ch);
    }
  }
  std::string arch(prop.gcnArchName);
  for (char& c : arch)
    if (c == ' ' || c == ':') c = '_';
  char buf[32];
  std::snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
  return arch + "/t2/" + buf;
}

// MLC_AUTOTUNE_CACHE, else $HOME/.cache/mlc_autotune.txt; empty: no cache.
std::string tune_cache_path() {
  if (const char* p = std::getenv("MLC_AUTOTUNE_CACHE")) return std::string(p);
  if (const char* home = std::getenv("HOME")) return std::string(home) + "/.cache/mlc_autotune.txt";
  return std::string();
}

bool valid_tuning(const Tuning& t) {
  return (t.block == 256 || t.block == 512 || t.block == 1024) && t.nu >= 1 && t.nu <= 8 &&
         t.inner > 0.0 && t.inner < 1.0;
}

bool tune_cache_read(const std::string& path, const std::string& key, int L,
                     std::vector<Tuning>& choice) {
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream in(line);
    std::string k;
    if (!(in >> k) || k != key) continue;
    std::vector<Tuning> v(L + 1, Tuning{1024, 2, 1e-4});
    bool ok = true;
    for (int s = 1; s <= L && ok; ++s)
      ok = (bool)(in >> v[s].block >> v[s].nu >> v[s].inner) && valid_tuning(v[s]);
    if (ok) {
      choice = v;
      return true;
    }
  }
  return false;
}

void tune_cache_write(const std::string& path, const std::string& key, int L,
                      const std::vector<Tuning>& choice) {
  std::vector<std::string> keep;
  {
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
      std::istringstream in(line);
      std::string k;
      if ((in >> k) && k != key) keep.push_back(line);
    }
  }
  std::ostringstream o;
  o << key;
  o.precision(17);
  for (int s = 1; s <= L; ++s) o << ' ' << choice[s].block << ' ' << choice[s].nu << ' ' << choice[s].inner;
  keep.push_back(o.str());
  const size_t slash = path.find_last_of('/');
  if (slash != std::string::npos) {
    const std::string dir = path.substr(0, slash);  // create missing directories
    for (size_t i = 1; i <= dir.size(); ++i)
      if (i == dir.size() || dir[i] == '/') (void)::mkdir(dir.substr(0, i).c_str(), 0755);
  }
  std::ofstream f(path, std::ios::trunc);
  for (const std::string& l : keep) f << l << '\n';
}

// After steps from+1 .. to: MLC_ENOCONV if a local solve of one of them (or, with the
// interface gluing, its G_{m+1} problem) ended above the tolerance.  Synchronises.
mlc_status check_converged(mlc_batch* b, int from, int to) {
  if (to <= from) return MLC_OK;
  double worst[MLC_MAX_LEVELS + 1];
  MLC_HIP(b, hipStreamSynchronize(b->st));
  MLC_HIP(b, hipMemcpy(worst, b->ws + b->plan.conv, (MLC_MAX_LEVELS + 1) * 8,
                       hipMemcpyDeviceToHost));
  const double lim = b->o.rtol * 1.0000001;
  double rec[2 * (MLC_MAX_LEVELS + 1)];
  if (b->plan.geo[0].pou == MLC_POU_INTERFACE)
    MLC_HIP(b, hipMemcpy(rec, b->ws + b->plan.pl[0].skel_rec, sizeof rec, hipMemcpyDeviceToHost));
  for (int s = from + 1; s <= to; ++s) {
    if (!(worst[s] <= lim)) {
      char msg[160];
      std::snprintf(msg, sizeof msg,
                    "a local solve of level step %d ended at relative residual %.3e > rtol", s,
                    worst[s]);
      b->err = msg;
      return MLC_ENOCONV;
    }
    if (b->plan.geo[0].pou == MLC_POU_INTERFACE && !(rec[2 * s + 1] <= lim)) {
      b->err = "the G_{m+1} problem of level step " + std::to_string(s) + " did not converge";
      return MLC_ENOCONV;
    }
  }
  return MLC_OK;
}

void batch_destroy(mlc_batch* b) {
  if (b->st) (void)hipStreamSynchronize(b->st);
  drop_graphs(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (auto& ev : b->ev_pending)
    for (auto e : ev) b->ev_free.push_back(e);
  for (auto e : b->ev_free) (void)hipEventDestroy(e);
  if (b->rb) rocblas_destroy_handle(b->rb);
  delete b;
}

}  // namespace

extern "C" {

mlc_status mlc_default_opts(mlc_solver_opts* o) {
  if (!o) return MLC_EINVAL;
  o->precision = 0;
  o->rtol = 1e-12;
  o->max_it = 200;
  o->max_refine = 10;
  o->inner_rtol = 1e-4;
  o->nu = 2;
  o->omega = 0.8;
  o->block = 0;
  o->timing = 0;
  o->record_tape = 0;
  o->glue_graph_it = 24;
  o->smoother = 1;
  return MLC_OK;
}

// ---------------- single problem ----------------

mlc_status mlc_workspace_size(const mlc_problem_desc* d, const mlc_solver_opts* o, size_t* bytes) {
  if (!bytes) return MLC_EINVAL;
  Plan P;
  std::string msg;
  mlc_status s = make_plan(1, d, o, P, msg);
  if (s != MLC_OK) return s;
  *bytes = P.total;
  return MLC_OK;
}

mlc_status mlc_create(const mlc_problem_desc* d, const mlc_solver_opts* o, void* ws, size_t bytes,
                      void* stream, mlc_ctx** out) {
  if (!out) return MLC_EINVAL;
  *out = nullptr;
  mlc_batch* b = nullptr;
  mlc_status s = batch_create(1, d, o, ws, bytes, stream, &b);
  if (s != MLC_OK) return s;
  mlc_ctx* c = new (std::nothrow) mlc_ctx();
  if (!c) {
    batch_destroy(b);
    return MLC_ENOMEM;
  }
  c->b = b;
  *out = c;
  return MLC_OK;
}

mlc_status mlc_coarse_setup(mlc_ctx* c) {
  if (!c) return MLC_EINVAL;
  return batch_setup(c->b);
}

mlc_status mlc_level_correct(mlc_ctx* c, mlc_level_stats* stt) {
  if (!c) return MLC_EINVAL;
  mlc_batch* b = c->b;
  mlc_status s = batch_step(b, 0);
  if (s != MLC_OK || !stt) return s;
  s = step_stats(b, stt);
  if (s != MLC_OK && s != MLC_ENOCONV) return s;
  double lam[MLC_MAX_Q];
  const int buf = (b->step + b->shift[0]) & 1;
  MLC_HIP(b, hipMemcpy(lam, b->ws + b->plan.pl[0].lam + (size_t)buf * MLC_MAX_Q * 8,
                       (size_t)b->plan.q * 8, hipMemcpyDeviceToHost));
  for (int i = 0; i < b->plan.q; ++i) stt->lambda[i] = lam[i];
  return s;
}

mlc_status mlc_run(mlc_ctx* c) {
  if (!c) return MLC_EINVAL;
  if (c->b->step < 0) {
    c->b->err = "run needs coarse_setup";
    return MLC_ESTATE;
  }
  const int from = c->b->step;
  while (c->b->step < c->b->plan.Lmax) {
    mlc_status s = batch_step(c->b, 0);
    if (s != MLC_OK) return s;
  }
  return check_converged(c->b, from, c->b->step);
}

mlc_status mlc_rewind(mlc_ctx* c) {
  if (!c) return MLC_EINVAL;
  return mlc_batch_rewind(c->b);
}

mlc_status mlc_current_level(const mlc_ctx* c, int32_t* level) {
  if (!c || !level) return MLC_EINVAL;
  *level = c->b->step;
  return MLC_OK;
}

mlc_status mlc_get_eigenpairs(mlc_ctx* c, double* lam_host, double* u_dev) {
  if (!c) return MLC_EINVAL;
  return batch_get(c->b, 0, lam_host, u_dev);
}

mlc_status mlc_set_state(mlc_ctx* c, int32_t level, const double* lam_host, const double* u_dev) {
  if (!c || !lam_host || !u_dev) return MLC_EINVAL;
  mlc_batch* b = c->b;
  if (b->step < 0) {
    b->err = "set_state needs coarse_setup";
    return MLC_ESTATE;
  }
  if (level < 0 || level > b->plan.Lmax) {
    b->err = "level out of range";
    return MLC_EINVAL;
  }
  const Geometry& g = b->plan.geo[0];
  // the state goes to buffer 0; the shift makes (level + shift) & 1 == 0
  MLC_HIP(b, launch_set_state(b->dprob, level, 0, u_dev, g.nodes(level), b->st));
  MLC_HIP(b, hipStreamSynchronize(b->st));
  MLC_HIP(b, hipMemcpy(b->ws + b->plan.pl[0].lam, lam_host, (size_t)g.q * 8, hipMemcpyHostToDevice));
  b->step = level;
  b->shift[0] = level & 1;
  b->can_rewind = false;
  b->tape_valid = false;  // the tape below `level` does not belong to this state
  drop_graphs(b);
  return MLC_OK;
}

// Reverse sweep over every level (see kernels_adj.hip for the formulas).
static mlc_status backward_impl(mlc_batch* b, double lambda_bar, double* out, bool hf_only) {
  const Plan& P = b->plan;
  const TapeLayout& T = P.tape;
  const Geometry& g = P.geo[0];
  char* w = b->ws;
  hipStream_t st = b->st;
  const ProbDev* dp = b->dprob;
  const int L = g.L, nH = g.nH;
  const int nc1sq = (g.nc + 1) * (g.nc + 1);
  auto D = [&](size_t off) { return (double*)(w + off); };
  double* scal = D(T.scal);  // [0] c_bar_u, [1 + l] lambda_bar of level l
  for (int l = 0; l <= L; ++l) {
    MLC_HIP(b, hipMemsetAsync(w + T.klo[l], 0, (size_t)(g.N(l) * g.N(l)) * 8, st));
    MLC_HIP(b, hipMemsetAsync(w + T.kup[l], 0, (size_t)(g.N(l) * g.N(l)) * 8, st));
  }
  MLC_HIP(b, hipMemsetAsync(w + T.adj_u, 0, (size_t)g.nodes(L) * 8, st));
  MLC_HIP(b, hipStreamSynchronize(st));
  MLC_HIP(b, hipMemcpy(scal + 1 + L, &lambda_bar, 8, hipMemcpyHostToDevice));
  if (hf_only) {  // Hellmann-Feynman reference: lambda_bar (u, dK u) on the finest level
    MLC_HIP(b, launch_adj_products(dp, L, g.N(L) * g.N(L), D(T.tu[L]), scal + 1 + L, nullptr,
                                   nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                   D(T.klo[L]), D(T.kup[L]), st));
    MLC_HIP(b, launch_adj_out(D(T.klo[L]), D(T.kup[L]), (int)g.N(L), g.kind, g.nc, out, st));
    MLC_HIP(b, hipStreamSynchronize(st));
    return MLC_OK;
  }
  MLC_HIP(b, launch_coarse_combine(dp, nc1sq, D(T.e0), D(T.v0grid), st));
  double* rchain = b->hp[0].rchain;
  for (int m = L; m >= 1; --m) {
    const int k = m - 1;
    const StepTables& S = P.steps[m];
    const TileItem* items = (const TileItem*)(w + S.items_off);
    const int32_t* sub_item = (const int32_t*)(w + S.sub_item_off);
    const int nitems = (int)S.items.size();
    const int64_t nn = g.nodes(m);
    const double* rr = D(T.trr[m]);
    const double* u_m = D(T.tu[m]);
    const double* ut_m = D(T.tut[m]);
    // c_bar = S^T u_bar: restriction of u_bar to the coarse grid, then V^T; and u~ . u_bar
    const double* src = D(T.adj_u);
    for (int l = m - 1; l >= 0; --l) {
      double* dst = rchain + P.pl[0].rchain_off[l];
      MLC_HIP(b, launch_restrict1(dp, src, dst, l, g.nodes(l), st));
      src = dst;
    }
    MLC_HIP(b, launch_coarse_project(dp, nH, src, D(T.cbar_H), st));
    MLC_HIP(b, launch_dot_sum(dp, m, nn, ut_m, D(T.adj_u), false, D(T.parts), scal, st));
    MLC_HIP(b, launch_adj_rr(dp, rr, D(T.cbar_H), scal, scal + 1 + m, D(T.ycoef), D(T.coef), st));
    MLC_HIP(b, launch_coarse_combine(dp, nc1sq, D(T.ycoef), D(T.ygrid), st));
    MLC_HIP(b, launch_adj_shat(dp, m, nn, D(T.ygrid), D(T.coef), ut_m, D(T.shat), st));
    MLC_HIP(b, launch_adj_utbar(g.kind, dp, m, nn, u_m, D(T.shat), D(T.adj_u), D(T.coef), rr,
                                D(T.utbar), st));
    // adjoint local solves z_j = K_j^-1 (chi_j u~_bar)
    MLC_HIP(b, launch_adj_tile_rhs(dp, items, nitems, sub_item, w + P.store, m, D(T.utbar), st));
    double w1, w2;
    sweep_weights(b->o, b->o.nu, &w1, &w2);
    MLC_HIP(b, launch_local_pcg(g.kind, b->blocks[m], dp, items, nitems, w + P.store,
                                (const double*)(w + P.inv), m, (ItemStat*)(w + P.stats),
                                b->o.rtol, b->o.max_it, b->o.nu, w1, w2, 1,
                                P.steps[m].max_tile_nx, st));
    MLC_HIP(b, launch_adj_rbar(dp, items, sub_item, w + P.store, m, nn, D(T.rbar), st));
    const double* u_k = (k == 0) ? D(T.v0grid) : D(T.tu[k]);
    const double* lam_k = (k == 0) ? b->hp[0].Lam : D(T.trr[k]) + 3 * nH + 3;
    MLC_HIP(b, launch_adj_next(g.kind, dp, m, nn, u_k, lam_k, D(T.utbar), D(T.rbar), D(T.ubar),
                               D(T.adj_next), st));
    MLC_HIP(b, launch_dot_sum(dp, m, nn, D(T.rbar), D(T.ubar), true, D(T.parts), scal + 1 + k, st));
    MLC_HIP(b, launch_adj_products(dp, m, g.N(m) * g.N(m), u_m, scal + 1 + m, D(T.shat), D(T.rbar),
                                   D(T.ubar), items, sub_item, w + P.store, D(T.te[m]),
                                   (const int64_t*)(w + T.te_off[m]), D(T.klo[m]), D(T.kup[m]), st));
    MLC_HIP(b, launch_restrict1(dp, D(T.adj_next), D(T.adj_u), k, g.nodes(k), st));
  }
  // level 0: the coarse eigenpair (lambda_0, v_0) of the full eigendecomposition
  MLC_HIP(b, launch_adj_level0(dp, nH, D(T.adj_u), D(T.a0), st));
  MLC_HIP(b, launch_coarse_combine(dp, nc1sq, D(T.a0), D(T.ygrid), st));
  MLC_HIP(b, launch_adj_products(dp, 0, g.N(0) * g.N(0), D(T.v0grid), scal + 1, D(T.ygrid),
                                 nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                 D(T.klo[0]), D(T.kup[0]), st));
  // children-mean coefficients: every triangle passes 1/4 of its adjoint to its children
  for (int l = 1; l <= L; ++l)
    MLC_HIP(b, launch_adj_down(D(T.klo[l - 1]), D(T.kup[l - 1]), D(T.klo[l]), D(T.kup[l]),
                               (int)g.N(l - 1), st));
  MLC_HIP(b, launch_adj_out(D(T.klo[L]), D(T.kup[L]), (int)g.N(L), g.kind, g.nc, out, st));
  MLC_HIP(b, hipStreamSynchronize(st));
  return MLC_OK;
}

mlc_status mlc_backward(mlc_ctx* c, const double* lambda_bar_host, double* kappa_bar_dev) {
  if (!c || !lambda_bar_host || !kappa_bar_dev) return MLC_EINVAL;
  mlc_batch* b = c->b;
  if (!b->plan.tape.on) {
    b->err = "backward needs opts.record_tape = 1";
    return MLC_EINVAL;
  }
  if (b->step != b->plan.Lmax || b->shift[0] != 0 || !b->tape_valid) {
    b->err = "backward needs a complete forward run (coarse_setup, then every level_correct)";
    return MLC_ESTATE;
  }
  return backward_impl(b, *lambda_bar_host, kappa_bar_dev, false);
}

mlc_status mlc_hf_gradient(mlc_ctx* c, double* kappa_bar_dev) {
  if (!c || !kappa_bar_dev) return MLC_EINVAL;
  mlc_batch* b = c->b;
  if (!b->plan.tape.on) {
    b->err = "the Hellmann-Feynman gradient needs opts.record_tape = 1";
    return MLC_EINVAL;
  }
  if (b->step != b->plan.Lmax || b->shift[0] != 0 || !b->tape_valid) {
    b->err = "the Hellmann-Feynman gradient needs a complete forward run";
    return MLC_ESTATE;
  }
  return backward_impl(b, 1.0, kappa_bar_dev, true);
}

mlc_status mlc_phase_times(mlc_ctx* c, double* ms, int32_t n) {
  if (!c || !ms || n < 1) return MLC_EINVAL;
  return phase_times(c->b, ms, n);
}

mlc_status mlc_destroy(mlc_ctx* c) {
  if (!c) return MLC_EINVAL;
  batch_destroy(c->b);
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

const char* mlc_last_error(const mlc_ctx* c) { return c ? c->b->err.c_str() : "null context"; }

// ---------------- without device allocation ----------------

}  // extern "C"

// The workspace of mlc_solve_static: a file-scope device array (every device the library
// runs on holds its own copy until the process ends).  In host code its name is only a
// stand-in: kernels and copies use the address hipGetSymbolAddress returns per device.
#define MLC_STATIC_BYTES ((size_t)64 << 20)
#define MLC_STATIC_DEVICES 64
__device__ __align__(256) char scratch[MLC_STATIC_BYTES];

namespace {
std::mutex g_scratch_mu;
void* g_scratch[MLC_STATIC_DEVICES] = {};
}  // namespace

extern "C" {

mlc_status mlc_solve_static(const mlc_problem_desc* d, const mlc_solver_opts* o, void* stream,
                            double* lam_host, double* u_dev) {
  if (!d || !o || !lam_host) return MLC_EINVAL;
  Plan P;
  std::string msg;
  mlc_status s = make_plan(1, d, o, P, msg);
  if (s != MLC_OK) {
    std::fprintf(stderr, "mlc: %s\n", msg.c_str());
    return s;
  }
  if (P.total > MLC_STATIC_BYTES) {
    std::fprintf(stderr, "mlc: mlc_solve_static needs %zu bytes of workspace, above the static "
                 "scratch of %zu bytes (use mlc_create with a caller's workspace)\n",
                 P.total, (size_t)MLC_STATIC_BYTES);
    return MLC_ENOMEM;
  }
  if (P.geo[0].nH > MLC_JACOBI_MAX_NH || o->record_tape || o->timing) {
    std::fprintf(stderr, "mlc: mlc_solve_static needs a coarse space of at most %d nodes (the "
                 "device eigensolver), no tape and no timing events\n", MLC_JACOBI_MAX_NH);
    return MLC_EINVAL;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MLC_STATIC_DEVICES) return MLC_EHIP;
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        std::fprintf(stderr, "mlc: hipGetSymbolAddress(scratch): %s\n", hipGetErrorString(e));
        return MLC_EHIP;
      }
      g_scratch[dev] = p;
    }
    ws = g_scratch[dev];
  }
  mlc_batch* b = nullptr;
  s = batch_create(1, d, o, ws, MLC_STATIC_BYTES, stream, &b);
  if (s != MLC_OK) return s;
  s = batch_setup(b);
  if (s == MLC_OK) {
    while (s == MLC_OK && b->step < b->plan.Lmax) s = batch_step(b, 0);
    if (s == MLC_OK) s = check_converged(b, 0, b->step);
    if (s == MLC_OK || s == MLC_ENOCONV) {
      const mlc_status g = batch_get(b, 0, lam_host, u_dev);
      if (g != MLC_OK) s = g;
    }
  }
  if (s != MLC_OK && s != MLC_ENOCONV) std::fprintf(stderr, "mlc: %s\n", b->err.c_str());
  batch_destroy(b);
  return s;
}

// ---------------- batches ----------------

mlc_status mlc_batch_workspace_size(int32_t n, const mlc_problem_desc* descs,
                                    const mlc_solver_opts* o, size_t* bytes) {
  if (!bytes) return MLC_EINVAL;
  Plan P;
  std::string msg;
  mlc_status s = make_plan(n, descs, o, P, msg);
  if (s != MLC_OK) return s;
  *bytes = P.total;
  return MLC_OK;
}

mlc_status mlc_batch_create(int32_t n, const mlc_problem_desc* descs, const mlc_solver_opts* o,
                            void* ws, size_t bytes, void* stream, mlc_batch** out) {
  return batch_create(n, descs, o, ws, bytes, stream, out);
}

mlc_status mlc_batch_setup(mlc_batch* b) { return b ? batch_setup(b) : MLC_EINVAL; }

mlc_status mlc_batch_step(mlc_batch* b, int32_t use_graph) {
  return b ? batch_step(b, use_graph) : MLC_EINVAL;
}

mlc_status mlc_batch_run(mlc_batch* b, int32_t use_graph) {
  if (!b) return MLC_EINVAL;
  if (b->step < 0) {
    b->err = "run needs setup";
    return MLC_ESTATE;
  }
  const int from = b->step;
  while (b->step < b->plan.Lmax) {
    mlc_status s = batch_step(b, use_graph);
    if (s != MLC_OK) return s;
  }
  return check_converged(b, from, b->step);
}

mlc_status mlc_batch_rewind(mlc_batch* b) {
  if (!b) return MLC_EINVAL;
  if (b->step < 1 || !b->can_rewind) {
    b->err = "nothing to rewind";
    return MLC_ESTATE;
  }
  b->step -= 1;
  b->can_rewind = false;
  return MLC_OK;
}

mlc_status mlc_batch_restart(mlc_batch* b) {
  if (!b) return MLC_EINVAL;
  if (b->step < 0) {
    b->err = "restart needs setup";
    return MLC_ESTATE;
  }
  MLC_HIP(b, launch_init_u0(b->dprob, b->plan.n, 0, b->plan.max_nc1sq, b->st));
  b->step = 0;
  b->can_rewind = false;
  b->tape_valid = true;  // the next steps record every level again from level 0
  std::fill(b->shift.begin(), b->shift.end(), 0);
  return MLC_OK;
}

mlc_status mlc_batch_current_step(const mlc_batch* b, int32_t* step) {
  if (!b || !step) return MLC_EINVAL;
  *step = b->step;
  return MLC_OK;
}

mlc_status mlc_batch_get(mlc_batch* b, int32_t i, double* lam_host, double* u_dev) {
  return b ? batch_get(b, i, lam_host, u_dev) : MLC_EINVAL;
}

mlc_status mlc_batch_step_stats(mlc_batch* b, mlc_level_stats* st) {
  if (!b || !st) return MLC_EINVAL;
  return step_stats(b, st);
}

mlc_status mlc_batch_autotune(mlc_batch* b, int32_t* blocks_out, int32_t n) {
  if (!b) return MLC_EINVAL;
  if (b->step < 0) {
    b->err = "autotune needs setup";
    return MLC_ESTATE;
  }
  const Plan& P = b->plan;
  const Tuning base{b->blocks[1], b->o.nu, b->o.inner_rtol};
  std::vector<Tuning> choice(P.Lmax + 1, base);
  const std::string key = tune_key(b);
  const std::string path = tune_cache_path();
  bool cached = !key.empty() && !path.empty() && tune_cache_read(path, key, P.Lmax, choice);
  if (!cached) {
    // Coordinate search, each candidate timed over kReps full runs from level 0 (per step
    // the median local-solve time): the workgroup size at the batch's nu and tolerance;
    // then nu in 1..3 at the chosen sizes; then (mixed precision) the inner tolerance
    // 1e-3, 3e-4, .. 1e-5 at the chosen sizes and nu (the inner solves stop after whole
    // iterations, so the best tolerance varies with the problem).  Every setting solves
    // to the same rtol.
    constexpr int kReps = 3;
    std::vector<double> best(P.Lmax + 1, 1e300);
    const int saved_timing = b->o.timing;
    b->o.timing = 1;
    drop_graphs(b);
    mlc_status e = phase_times(b, nullptr, 0);  // drop stale events
    auto trial = [&](auto&& set) {
      std::vector<Tuning> t = choice;
      for (int s = 1; s <= P.Lmax; ++s) set(t[s]);
      for (int s = 1; s <= P.Lmax; ++s) {
        b->blocks[s] = t[s].block;
        b->nu_s[s] = t[s].nu;
        b->inner_s[s] = t[s].inner;
      }
      std::vector<std::vector<double>> ms_s(P.Lmax + 1);
      for (int rep = 0; rep < kReps && e == MLC_OK; ++rep) {
        if (launch_init_u0(b->dprob, P.n, 0, P.max_nc1sq, b->st) != hipSuccess) {
          b->err = "launch_init_u0 failed";
          e = MLC_EHIP;
          break;
        }
        b->step = 0;
        std::fill(b->shift.begin(), b->shift.end(), 0);
        for (int s = 1; s <= P.Lmax && e == MLC_OK; ++s) {
          e = batch_step(b, 0);
          double ms[2] = {0.0, 0.0};
          if (e == MLC_OK) e = phase_times(b, ms, 2);
          ms_s[s].push_back(ms[0]);
        }
      }
      for (int s = 1; s <= P.Lmax && e == MLC_OK; ++s) {
        std::vector<double> v = ms_s[s];
        std::sort(v.begin(), v.end());
        const double med = v[v.size() / 2];
        if (med < best[s]) {
          best[s] = med;
          choice[s] = t[s];
        }
      }
    };
    for (int blk : {256, 512, 1024})
      if (e == MLC_OK) trial([&](Tuning& t) { t = Tuning{blk, base.nu, base.inner}; });
    for (int nu : {1, 2, 3})
      if (e == MLC_OK && nu != base.nu) trial([&](Tuning& t) { t.nu = nu; });
    if (P.precision == 1)
      for (double tol : {1e-3, 3e-4, 1e-4, 3e-5, 1e-5})
        if (e == MLC_OK && tol != base.inner) trial([&](Tuning& t) { t.inner = tol; });
    b->o.timing = saved_timing;
    if (e != MLC_OK) return e;
    if (!key.empty() && !path.empty()) tune_cache_write(path, key, P.Lmax, choice);
  }
  for (int s = 1; s <= P.Lmax; ++s) {
    b->blocks[s] = choice[s].block;
    b->nu_s[s] = choice[s].nu;
    b->inner_s[s] = choice[s].inner;
  }
  for (int s = 1; s <= P.Lmax && blocks_out && s - 1 < n; ++s) blocks_out[s - 1] = choice[s].block;
  drop_graphs(b);
  MLC_HIP(b, launch_init_u0(b->dprob, P.n, 0, P.max_nc1sq, b->st));
  MLC_HIP(b, hipStreamSynchronize(b->st));
  b->step = 0;
  b->can_rewind = false;
  std::fill(b->shift.begin(), b->shift.end(), 0);
  return MLC_OK;
}

mlc_status mlc_batch_get_tuning(const mlc_batch* b, int32_t* blocks, int32_t* nu,
                                double* inner_rtol, int32_t n) {
  if (!b || n < 0) return MLC_EINVAL;
  for (int s = 1; s <= b->plan.Lmax && s - 1 < n; ++s) {
    if (blocks) blocks[s - 1] = b->blocks[s];
    if (nu) nu[s - 1] = b->nu_s[s];
    if (inner_rtol) inner_rtol[s - 1] = b->inner_s[s];
  }
  return MLC_OK;
}

mlc_status mlc_batch_set_tuning(mlc_batch* b, const int32_t* blocks, const int32_t* nu,
                                const double* inner_rtol, int32_t n) {
  if (!b || !blocks || !nu || !inner_rtol) return MLC_EINVAL;
  for (int s = 1; s <= b->plan.Lmax && s - 1 < n; ++s) {
    if (!valid_tuning(Tuning{blocks[s - 1], nu[s - 1], inner_rtol[s - 1]})) {
      b->err = "tuning: block 256, 512 or 1024, nu in 1..8, inner_rtol in (0, 1)";
      return MLC_EINVAL;
    }
  }
  for (int s = 1; s <= b->plan.Lmax && s - 1 < n; ++s) {
    b->blocks[s] = blocks[s - 1];
    b->nu_s[s] = nu[s - 1];
    b->inner_s[s] = inner_rtol[s - 1];
  }
  drop_graphs(b);
  return MLC_OK;
}

mlc_status mlc_batch_set_blocks(mlc_batch* b, const int32_t* blocks, int32_t n) {
  if (!b || !blocks) return MLC_EINVAL;
  for (int s = 1; s <= b->plan.Lmax && s - 1 < n; ++s) {
    const int v = blocks[s - 1];
    if (v != 256 && v != 512 && v != 1024) {
      b->err = "block sizes must be 256, 512 or 1024";
      return MLC_EINVAL;
    }
  }
  for (int s = 1; s <= b->plan.Lmax && s - 1 < n; ++s) b->blocks[s] = blocks[s - 1];
  drop_graphs(b);
  return MLC_OK;
}

mlc_status mlc_batch_phase_times(mlc_batch* b, double* ms, int32_t n) {
  if (!b || !ms || n < 1) return MLC_EINVAL;
  return phase_times(b, ms, n);
}

mlc_status mlc_batch_destroy(mlc_batch* b) {
  if (!b) return MLC_EINVAL;
  batch_destroy(b);
  return MLC_OK;
}

const char* mlc_batch_last_error(const mlc_batch* b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
