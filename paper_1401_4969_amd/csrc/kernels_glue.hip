// Algorithm 4.1 step 2 as the paper states it (gluing MLC_GLUE_INTERFACE): u~ = u~^j on
// G_j, and on G_{m+1} = Omega minus the closed G_j the solution of
//   a(u~, v) = lambda_k b(u_k, v) for all v in V_0h(G_{m+1}),
// with u~ = u~^j on the boundary of each G_j and 0 on the boundary of Omega (equation
// (G_m+1_Problem)).  G_j is D_j shrunk by half a coarse cell on every side, so the closed
// G_j are disjoint and lie inside the tiles.  In correction form (u~ = I u + e): e = e^j
// on each closed G_j, and on the remaining dofs S ("skeleton") K_SS e_S = r_S - K_SG e_G.
//
// The skeleton is one connected region of the whole grid, so it is solved by a global
// preconditioned CG over full-grid vectors that vanish off S: one thread per node, a few
// launches per iteration for all q right-hand sides at once (blockIdx.y), scalars kept in
// device memory (no host round trip per iteration), block partial sums reduced in a fixed
// order (deterministic).  A right-hand side that has converged is frozen by a flag its
// reduction sets; the host polls the flags every few iterations.
//
// Preconditioner: a geometric multigrid V-cycle on the same region.  G_{m+1} is bounded by
// lines of the grid of half coarse cells, so it is a union of cells of every level l >= 1
// and its Dirichlet spaces on levels l = 1..m are nested: the level-l operator (the level's
// stencil with the nodes outside the region held at 0) is the Galerkin product of the
// level above, and interpolation and restriction are the P1 ones with the nodes outside
// the region dropped.  Damped Jacobi (omega = 0.8, two sweeps before and after each coarse
// correction); on level 1 the region's interior nodes lie on the block-boundary lines, an
// operator with a bounded condition number, where eight sweeps serve as the coarse solve.
// The strips of G_{m+1} are a coarse cell wide, so a diagonal preconditioner needs
// O(H / h) iterations; the V-cycle keeps the count bounded in h.
//
// Per right-hand side i, at vec + i * stride: vectors E, W, Z, P (two, used alternately),
// Q, T on the level-m grid, then for l = m-1 down to 1 the level's b, x, y; block partials
// at parts + i*2*nblk; scalars at scal + i*SKEL_NS: rho, alpha, beta, ||w||^2, ||w_0||^2,
// done, tol^2, iterations.
#include "mlc_launch.h"

namespace {

constexpr int NTS = 256;
constexpr int SKEL_NS = 8;  // scalars per right-hand side
constexpr int SKEL_VEC = 7; // level-m vectors per right-hand side: E, W, Z, P0, P1, Q, T
constexpr double kMgOmega = 0.8;
constexpr int kMgCoarseSweeps = 8;

// Closed G_b along one axis holding fine index g (r fine cells per coarse cell, r >= 2),
// or -1.  G_b lies inside D_b, so only the block of g's coarse cell can hold it.
__device__ __forceinline__ int g_block(int nc, int nb, int g, int r) {
  const int half = r >> 1;
  const int b = block_of_cell(min(g / r, nc - 1), nc, nb);
  return (g >= block_bound(b, nc, nb) * r + half && g <= block_bound(b + 1, nc, nb) * r - half) ? b : -1;
}

// Skeleton dof: a dof of the domain outside every closed G_j.
__device__ __forceinline__ bool skel_dof(const ProbDev& P, int N, int r, int gx, int gy) {
  if (!is_dof(P.domain, N, gx, gy)) return false;
  return g_block(P.n_c, P.sub_x, gx, r) < 0 || g_block(P.n_c, P.sub_y, gy, r) < 0;
}

template <int KIND>
__device__ __forceinline__ double apply_masked(const ProbDev& P, int m, int N, int n1, int gx,
                                               int gy, int64_t idx, const double* v, double& d) {
  const Weights W = edge_weights<KIND>(P, m, N, gx, gy);
  double ne = 0.0, sw = 0.0;
  if constexpr (KIND == 3) {
    ne = v[idx + n1 + 1];
    sw = v[idx - n1 - 1];
  }
  return apply_k<KIND, double>(W, v[idx], v[idx + 1], v[idx - 1], v[idx + n1], v[idx - n1], ne,
                               sw, d);
}

__device__ __forceinline__ void block_partials(double a, double b, double* parts) {
  __shared__ double red[2 * (NTS / 64)];
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[wid] = a;
    red[NTS / 64 + wid] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < NTS / 64; ++w) {
      sa += red[w];
      sb += red[NTS / 64 + w];
    }
    parts[2 * blockIdx.x] = sa;
    parts[2 * blockIdx.x + 1] = sb;
  }
}

// e = e^j on the closed G_j (item of subdomain j and right-hand side i), 0 elsewhere.
__global__ __launch_bounds__(NTS) void k_skel_fill(const ProbDev* probs, const TileItem* items,
                                                   const int32_t* sub_item, const char* store,
                                                   int m, double* vec, int64_t stride,
                                                   double* scal_all) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1, r = 1 << m;
  const int64_t nn = (int64_t)n1 * n1;
  const int i_rhs = blockIdx.y;
  // the preconditioner of the first iteration runs before the scalars are set: clear the
  // flag a previous solve left
  if (blockIdx.x == 0 && threadIdx.x == 0) scal_all[i_rhs * SKEL_NS + 5] = 0.0;
  double* E = vec + (int64_t)i_rhs * stride;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  if (idx >= nn) return;
  const int gy = (int)(idx / n1), gx = (int)(idx - (int64_t)gy * n1);
  double v = 0.0;
  if (is_dof(P.domain, N, gx, gy)) {
    const int bx = g_block(P.n_c, P.sub_x, gx, r), by = g_block(P.n_c, P.sub_y, gy, r);
    if (bx >= 0 && by >= 0) {
      const int item = sub_item[P.sub_item_off + (by * P.sub_x + bx) * P.q + i_rhs];
      if (item >= 0) {
        const TileItem& it = items[item];
        const int nx = it.cw * r - 1;
        const int lx = gx - (it.cx0 * r + 1), ly = gy - (it.cy0 * r + 1);
        v = reinterpret_cast<const double*>(store + it.off)[(int64_t)ly * nx + lx];
      }
    }
  }
  E[idx] = v;
}

// w = r - K e on S (0 elsewhere).
template <int KIND>
__global__ __launch_bounds__(NTS) void k_skel_init(const ProbDev* probs, int m, double* vec,
                                                   int64_t stride) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1, r = 1 << m;
  const int64_t nn = (int64_t)n1 * n1;
  const int i_rhs = blockIdx.y;
  double* base = vec + (int64_t)i_rhs * stride;
  const double* E = base;
  double* Wv = base + nn;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  if (idx >= nn) return;
  const int gy = (int)(idx / n1), gx = (int)(idx - (int64_t)gy * n1);
  double w = 0.0;
  if (skel_dof(P, N, r, gx, gy)) {
    double d;
    w = P.res[(int64_t)i_rhs * nn + idx] - apply_masked<KIND>(P, m, N, n1, gx, gy, idx, E, d);
  }
  Wv[idx] = w;
}

// Partial sums (w.z, w.w) after the preconditioner.
__global__ __launch_bounds__(NTS) void k_skel_dot(const ProbDev* probs, int m, const double* vec,
                                                  int64_t stride, const double* scal_all,
                                                  double* parts_all) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1;
  const int64_t nn = (int64_t)n1 * n1;
  const int i_rhs = blockIdx.y;
  if (scal_all[i_rhs * SKEL_NS + 5] != 0.0) return;  // converged: frozen
  const double* Wv = vec + (int64_t)i_rhs * stride + nn;
  const double* Z = Wv + nn;
  double* parts = parts_all + (int64_t)i_rhs * 2 * gridDim.x;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  double wz = 0.0, ww = 0.0;
  if (idx < nn) {
    const double w = Wv[idx];
    wz = w * Z[idx];
    ww = w * w;
  }
  block_partials(wz, ww, parts);
}

// ---- the V-cycle on G_{m+1} (one thread per node of the level, blockIdx.y = rhs) ----

// Level-l vectors of right-hand side i: b, x, y (level m: W, T, Z).
struct MgLevel {
  double* b;
  double* x;
  double* y;
};
__device__ __forceinline__ MgLevel mg_level(double* vec, int64_t stride, int i_rhs, int nc, int m,
                                            int l) {
  double* base = vec + (int64_t)i_rhs * stride;
  const int64_t nnm = (int64_t)((nc << m) + 1) * ((nc << m) + 1);
  MgLevel L;
  if (l == m) {
    L.b = base + nnm;
    L.x = base + 6 * nnm;
    L.y = base + 2 * nnm;
    return L;
  }
  int64_t off = SKEL_VEC * nnm;
  for (int k = m - 1; k > l; --k) off += 3 * (int64_t)((nc << k) + 1) * ((nc << k) + 1);
  const int64_t nl = (int64_t)((nc << l) + 1) * ((nc << l) + 1);
  L.b = base + off;
  L.x = base + off + nl;
  L.y = base + off + 2 * nl;
  return L;
}

// out = in + omega D^-1 (b - A in) on the region's nodes of level l (first: in = 0), 0
// elsewhere.  sel: 0 x -> y, 1 y -> x, 2 first sweep into x.
template <int KIND>
__global__ __launch_bounds__(NTS) void k_mg_smooth(const ProbDev* probs, int m, int l, double* vec,
                                                   int64_t stride, int sel, const double* scal_all) {
  const ProbDev& P = probs[0];
  const int i_rhs = blockIdx.y;
  if (scal_all[i_rhs * SKEL_NS + 5] != 0.0) return;  // converged: frozen
  const int N = P.n_c << l, n1 = N + 1, r = 1 << l;
  const int64_t nn = (int64_t)n1 * n1;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  if (idx >= nn) return;
  const MgLevel L = mg_level(vec, stride, i_rhs, P.n_c, m, l);
  const double* in = sel == 1 ? L.y : L.x;
  double* out = sel == 0 ? L.y : L.x;
  const int gy = (int)(idx / n1), gx = (int)(idx - (int64_t)gy * n1);
  double v = 0.0;
  if (skel_dof(P, N, r, gx, gy)) {
    double d;
    if (sel == 2) {
      const Weights W = edge_weights<KIND>(P, l, N, gx, gy);
      v = kMgOmega * L.b[idx] / diag_of<KIND>(W);
    } else {
      const double a = apply_masked<KIND>(P, l, N, n1, gx, gy, idx, in, d);
      v = in[idx] + kMgOmega * (L.b[idx] - a) / d;
    }
  }
  out[idx] = v;
}

// b_{l-1} = P^T (b_l - A_l y_l) on the region's nodes of level l-1 (full weighting on the
// SW-NE mesh: the coarse node's fine twin 1, its six neighbours 1/2), 0 elsewhere.
template <int KIND>
__global__ __launch_bounds__(NTS) void k_mg_restrict(const ProbDev* probs, int m, int l,
                                                     double* vec, int64_t stride,
                                                     const double* scal_all) {
  const ProbDev& P = probs[0];
  const int i_rhs = blockIdx.y;
  if (scal_all[i_rhs * SKEL_NS + 5] != 0.0) return;
  const int Nc = P.n_c << (l - 1), nc1 = Nc + 1;
  const int64_t nnc = (int64_t)nc1 * nc1;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  if (idx >= nnc) return;
  const MgLevel F = mg_level(vec, stride, i_rhs, P.n_c, m, l);
  const MgLevel Cl = mg_level(vec, stride, i_rhs, P.n_c, m, l - 1);
  const int Iy = (int)(idx / nc1), Ix = (int)(idx - (int64_t)Iy * nc1);
  double val = 0.0;
  if (skel_dof(P, Nc, 1 << (l - 1), Ix, Iy)) {
    const int N = 2 * Nc, n1 = N + 1, r = 1 << l;
    const int fx = 2 * Ix, fy = 2 * Iy;
    const int dx[7] = {0, 1, -1, 0, 0, 1, -1}, dy[7] = {0, 0, 0, 1, -1, 1, -1};
    for (int k = 0; k < 7; ++k) {
      const int gx = fx + dx[k], gy = fy + dy[k];
      if (!skel_dof(P, N, r, gx, gy)) continue;
      const int64_t f = (int64_t)gy * n1 + gx;
      double d;
      const double res = F.b[f] - apply_masked<KIND>(P, l, N, n1, gx, gy, f, F.y, d);
      val += (k == 0 ? 1.0 : 0.5) * res;
    }
  }
  Cl.b[idx] = val;
}

// y_l += P y_{l-1} on the region's nodes of level l (P1 interpolation on the SW-NE mesh).
__global__ __launch_bounds__(NTS) void k_mg_prolong(const ProbDev* probs, int m, int l, double* vec,
                                                    int64_t stride, const double* scal_all) {
  const ProbDev& P = probs[0];
  const int i_rhs = blockIdx.y;
  if (scal_all[i_rhs * SKEL_NS + 5] != 0.0) return;
  const int N = P.n_c << l, n1 = N + 1, r = 1 << l;
  const int64_t nn = (int64_t)n1 * n1;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  if (idx >= nn) return;
  const int gy = (int)(idx / n1), gx = (int)(idx - (int64_t)gy * n1);
  if (!skel_dof(P, N, r, gx, gy)) return;
  const MgLevel F = mg_level(vec, stride, i_rhs, P.n_c, m, l);
  const MgLevel Cl = mg_level(vec, stride, i_rhs, P.n_c, m, l - 1);
  const int nc1 = N / 2 + 1;
  // the fine node's value of the coarse P1 function: the average of the coarse nodes at the
  // ends of the coarse edge it halves (or the coarse node it coincides with)
  const int x0 = gx >> 1, y0 = gy >> 1, x1 = (gx + 1) >> 1, y1 = (gy + 1) >> 1;
  const double v = 0.5 * (Cl.y[(int64_t)y0 * nc1 + x0] + Cl.y[(int64_t)y1 * nc1 + x1]);
  F.y[idx] += v;
}

// p_new = z + beta p_old on S (formed on the fly at the stencil points; 0 off S), stored
// in Pn; q = A p_new on S; partial sums (p.q, 0).  first: beta = 0, p_old unread.
template <int KIND>
__global__ __launch_bounds__(NTS) void k_skel_dir(const ProbDev* probs, int m, double* vec,
                                                  int64_t stride, int po, const double* scal_all,
                                                  int first, double* parts_all) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1, r = 1 << m;
  const int64_t nn = (int64_t)n1 * n1;
  const int i_rhs = blockIdx.y;
  const double* scal = scal_all + i_rhs * SKEL_NS;
  if (scal[5] != 0.0) return;  // converged: frozen (uniform over the workgroup)
  double* base = vec + (int64_t)i_rhs * stride;
  const double* Z = base + 2 * nn;
  const double* Po = base + (3 + po) * nn;
  double* Pn = base + (4 - po) * nn;
  double* Q = base + 5 * nn;
  double* parts = parts_all + (int64_t)i_rhs * 2 * gridDim.x;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  const double beta = first ? 0.0 : scal[2];
  const double* Pold = first ? Z : Po;  // any valid vector: multiplied by 0
  double pq = 0.0;
  if (idx < nn) {
    const int gy = (int)(idx / n1), gx = (int)(idx - (int64_t)gy * n1);
    double pc = 0.0, q = 0.0;
    if (skel_dof(P, N, r, gx, gy)) {
      auto pv = [&](int64_t j) -> double { return Z[j] + beta * Pold[j]; };
      const Weights W = edge_weights<KIND>(P, m, N, gx, gy);
      pc = pv(idx);
      double ne = 0.0, sw = 0.0, d;
      if constexpr (KIND == 3) {
        ne = pv(idx + n1 + 1);
        sw = pv(idx - n1 - 1);
      }
      q = apply_k<KIND, double>(W, pc, pv(idx + 1), pv(idx - 1), pv(idx + n1), pv(idx - n1), ne,
                                sw, d);
      pq = pc * q;
    }
    Pn[idx] = pc;
    Q[idx] = q;
  }
  block_partials(pq, 0.0, parts);
}

// e += alpha p, w -= alpha q on S.
__global__ __launch_bounds__(NTS) void k_skel_upd(const ProbDev* probs, int m, double* vec,
                                                  int64_t stride, int pn,
                                                  const double* scal_all) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1, r = 1 << m;
  const int64_t nn = (int64_t)n1 * n1;
  const int i_rhs = blockIdx.y;
  const double* scal = scal_all + i_rhs * SKEL_NS;
  if (scal[5] != 0.0) return;  // converged: frozen
  double* base = vec + (int64_t)i_rhs * stride;
  double* E = base;
  double* Wv = base + nn;
  const double* Pv = base + (3 + pn) * nn;
  const double* Q = base + 5 * nn;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  const double alpha = scal[1];
  if (idx < nn) {
    const int gy = (int)(idx / n1), gx = (int)(idx - (int64_t)gy * n1);
    if (skel_dof(P, N, r, gx, gy)) {
      E[idx] += alpha * Pv[idx];
      Wv[idx] = Wv[idx] - alpha * Q[idx];
    }
  }
}

// Fixed-order sum of the block partials of right-hand side blockIdx.x, then its CG scalars:
//   stage 0 (after init):  rho = w.z, ||w||^2 = ||w_0||^2 = w.w, tol^2 = rtol^2 ||w_0||^2,
//                          iterations 0, done when w_0 = 0
//   stage 1 (after dir):   alpha = rho / p.q
//   stage 2 (after upd):   beta = (w.z) / rho, rho = w.z, ||w||^2 = w.w, iterations + 1,
//                          done when ||w||^2 <= tol^2
// Stages 1 and 2 leave a converged right-hand side untouched.
__global__ __launch_bounds__(1024) void k_skel_reduce(const double* parts_all, int nblk, int stage,
                                                      double rtol, double* scal_all) {
  __shared__ double red[2 * 16];
  const int i_rhs = blockIdx.x;
  double* scal = scal_all + i_rhs * SKEL_NS;
  if (stage != 0 && scal[5] != 0.0) return;
  const double* parts = parts_all + (int64_t)i_rhs * 2 * nblk;
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nblk; k += 1024) {
    a += parts[2 * k];
    b += parts[2 * k + 1];
  }
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[wid] = a;
    red[16 + wid] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < 16; ++w) {
      sa += red[w];
      sb += red[16 + w];
    }
    if (stage == 0) {
      scal[0] = sa;
      scal[3] = sb;
      scal[4] = sb;
      scal[6] = rtol * rtol * sb;
      scal[7] = 0.0;
      scal[5] = sb > 0.0 ? 0.0 : 1.0;
    } else if (stage == 1) {
      scal[1] = sa != 0.0 ? scal[0] / sa : 0.0;
    } else {
      scal[2] = scal[0] != 0.0 ? sa / scal[0] : 0.0;
      scal[0] = sa;
      scal[3] = sb;
      scal[7] += 1.0;
      if (sb <= scal[6]) scal[5] = 1.0;
    }
  }
}

// u~ = I u + e for right-hand side i (0 off the domain).
__global__ __launch_bounds__(NTS) void k_skel_finish(const ProbDev* probs, int m,
                                                     const double* vec, int64_t stride) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1;
  const int64_t nn = (int64_t)n1 * n1;
  const int i_rhs = blockIdx.y;
  const double* E = vec + (int64_t)i_rhs * stride;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  if (idx >= nn) return;
  const int gy = (int)(idx / n1), gx = (int)(idx - (int64_t)gy * n1);
  const int64_t o = (int64_t)i_rhs * nn + idx;
  P.ut[o] = is_dof(P.domain, N, gx, gy) ? P.ubar[o] + E[idx] : 0.0;
}

}  // namespace

hipError_t run_interface_gluing(int kind, const ProbDev* dprob, const TileItem* items,
                                const int32_t* sub_item, const char* store, int m, int q, int nc,
                                int64_t stride, double rtol, int max_it, double* vec,
                                double* parts, double* scal, hipStream_t s, int* iters_out,
                                double* relres_out) {
  auto nodes_of = [&](int l) { return (int64_t)((nc << l) + 1) * ((nc << l) + 1); };
  auto grid_of = [&](int l) { return dim3((unsigned)((nodes_of(l) + NTS - 1) / NTS), (unsigned)q); };
  const unsigned nblk = (unsigned)((nodes_of(m) + NTS - 1) / NTS);
  const dim3 g(nblk, (unsigned)q);
#define MLC_SKEL(K, G, ...)                                                               \
  do {                                                                                    \
    if (kind == 0)                                                                        \
      hipLaunchKernelGGL(K<0>, G, dim3(NTS), 0, s, __VA_ARGS__);                          \
    else if (kind == 1)                                                                   \
      hipLaunchKernelGGL(K<1>, G, dim3(NTS), 0, s, __VA_ARGS__);                          \
    else if (kind == 2)                                                                   \
      hipLaunchKernelGGL(K<2>, G, dim3(NTS), 0, s, __VA_ARGS__);                          \
    else                                                                                  \
      hipLaunchKernelGGL(K<3>, G, dim3(NTS), 0, s, __VA_ARGS__);                          \
  } while (0)
  // z = B w: the V-cycle on G_{m+1}, levels m .. 1 (result in Z)
  auto vcycle = [&]() {
    for (int l = m; l >= 2; --l) {
      MLC_SKEL(k_mg_smooth, grid_of(l), dprob, m, l, vec, stride, 2, scal);
      MLC_SKEL(k_mg_smooth, grid_of(l), dprob, m, l, vec, stride, 0, scal);
      MLC_SKEL(k_mg_restrict, grid_of(l - 1), dprob, m, l, vec, stride, scal);
    }
    MLC_SKEL(k_mg_smooth, grid_of(1), dprob, m, 1, vec, stride, 2, scal);
    for (int k = 1; k < kMgCoarseSweeps; ++k)
      MLC_SKEL(k_mg_smooth, grid_of(1), dprob, m, 1, vec, stride, (k & 1) ? 0 : 1, scal);
    for (int l = 2; l <= m; ++l) {
      hipLaunchKernelGGL(k_mg_prolong, grid_of(l), dim3(NTS), 0, s, dprob, m, l, vec, stride, scal);
      MLC_SKEL(k_mg_smooth, grid_of(l), dprob, m, l, vec, stride, 1, scal);
      MLC_SKEL(k_mg_smooth, grid_of(l), dprob, m, l, vec, stride, 0, scal);
    }
  };
  hipLaunchKernelGGL(k_skel_fill, g, dim3(NTS), 0, s, dprob, items, sub_item, store, m, vec,
                     stride, scal);
  MLC_SKEL(k_skel_init, g, dprob, m, vec, stride);
  vcycle();
  hipLaunchKernelGGL(k_skel_dot, g, dim3(NTS), 0, s, dprob, m, vec, stride, scal, parts);
  hipLaunchKernelGGL(k_skel_reduce, dim3(q), dim3(1024), 0, s, parts, (int)nblk, 0, rtol, scal);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double h[SKEL_NS * MLC_MAX_Q];
  int it = 0;
  while (it < max_it) {
    // four iterations between polls of the convergence flags
    for (int k = 0; k < 4 && it < max_it; ++k, ++it) {
      const int po = it & 1;  // the two direction buffers alternate
      MLC_SKEL(k_skel_dir, g, dprob, m, vec, stride, po, scal, it == 0 ? 1 : 0, parts);
      hipLaunchKernelGGL(k_skel_reduce, dim3(q), dim3(1024), 0, s, parts, (int)nblk, 1, rtol, scal);
      hipLaunchKernelGGL(k_skel_upd, g, dim3(NTS), 0, s, dprob, m, vec, stride, 1 - po, scal);
      vcycle();
      hipLaunchKernelGGL(k_skel_dot, g, dim3(NTS), 0, s, dprob, m, vec, stride, scal, parts);
      hipLaunchKernelGGL(k_skel_reduce, dim3(q), dim3(1024), 0, s, parts, (int)nblk, 2, rtol, scal);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(h, scal, sizeof(double) * SKEL_NS * q, hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    bool all = true;
    for (int i = 0; i < q; ++i) all = all && h[i * SKEL_NS + 5] != 0.0;
    if (all) break;
  }
#undef MLC_SKEL
  hipLaunchKernelGGL(k_skel_finish, g, dim3(NTS), 0, s, dprob, m, vec, stride);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(h, scal, sizeof(double) * SKEL_NS * q, hipMemcpyDeviceToHost, s)) !=
      hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  int it_max = 0;
  double rel_max = 0.0;
  for (int i = 0; i < q; ++i) {
    const double* c = h + i * SKEL_NS;
    it_max = (int)c[7] > it_max ? (int)c[7] : it_max;
    const double rel = c[4] > 0.0 ? sqrt(c[3] / c[4]) : 0.0;
    rel_max = rel > rel_max ? rel : rel_max;
  }
  *iters_out = it_max;
  *relres_out = rel_max;
  return hipSuccess;
}

// Doubles per right-hand side of the interface problem's vectors at finest level L.
int64_t skel_stride(int nc, int L) {
  auto nodes_of = [&](int l) { return (int64_t)((nc << l) + 1) * ((nc << l) + 1); };
  int64_t s = SKEL_VEC * nodes_of(L);
  for (int l = 1; l < L; ++l) s += 3 * nodes_of(l);
  return s;
}
