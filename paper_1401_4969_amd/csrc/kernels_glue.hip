// Algorithm 4.1 step 2 as the paper states it (gluing MLC_GLUE_INTERFACE): u~ = u~^j on
// G_j, and on G_{m+1} = Omega minus the closed G_j the solution of
//   a(u~, v) = lambda_k b(u_k, v) for all v in V_0h(G_{m+1}),
// with u~ = u~^j on the boundary of each G_j and 0 on the boundary of Omega (equation
// (G_m+1_Problem)).  G_j is D_j shrunk by half a coarse cell on every side, so the closed
// G_j are disjoint and lie inside the tiles.  In correction form (u~ = I u + e): e = e^j
// on each closed G_j, and on the remaining dofs S ("skeleton") K_SS e_S = r_S - K_SG e_G.
//
// The skeleton is one connected region of the whole grid, so it is solved by a global
// preconditioned CG over full-grid vectors that vanish off S, all q right-hand sides at once
// (blockIdx.y), scalars kept in device memory (no host round trip per iteration), block
// partial sums reduced in a fixed order (deterministic).  A right-hand side that has
// converged is frozen by a flag its reduction sets, so a fixed launch sequence (a hipGraph)
// can run more iterations than it needs; the eager path polls the flags every few
// iterations.
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
// Each level l >= 2 of the cycle is two launches over tiles of 32 x 32 (or 16 x 16) nodes staged in LDS
// with a halo of three nodes (recomputed by the neighbouring tiles, so no tile waits on
// another): the down leg (both pre-sweeps, the residual and its restriction) and the up leg
// (the interpolated coarse correction and both post-sweeps).  The CG update of w and e is
// fused into the down leg of level m and the dot products into its up leg; level 1 runs its
// eight sweeps in one workgroup per right-hand side with the level in LDS.  One CG
// iteration is 2 m + 2 launches.
//
// Per right-hand side i, at vec + i * stride: vectors E, W0, W1 (the residual, alternating
// between iterations), Z, P0, P1 (the direction, alternating), Q, Y (the pre-smoothed
// level-m iterate) on the level-m grid, then for l = m-1 down to 1 the level's b, y (after
// the pre-sweeps) and x (the level's correction); block partials at parts + i*2*nblk;
// scalars at scal + i*SKEL_NS: rho, alpha, beta, ||w||^2, ||w_0||^2, done, tol^2,
// iterations.
#include "mlc_launch.h"

namespace {

constexpr int NTS = 256;
constexpr int SKEL_NS = 8;  // scalars per right-hand side
constexpr int SKEL_VEC = 8; // level-m vectors per right-hand side: E, W0, W1, Z, P0, P1, Q, Y
constexpr int V_E = 0, V_W = 1, V_Z = 3, V_P = 4, V_Q = 6, V_Y = 7;
constexpr double kMgOmega = 0.8;
constexpr int kMgCoarseSweeps = 8;
static_assert(kMgCoarseSweeps % 2 == 0, "the coarse sweeps end in their second buffer");

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

// e = e^j on the closed G_j (item of subdomain j and right-hand side i), 0 elsewhere; clears
// the solve's flags and record.
__global__ __launch_bounds__(NTS) void k_skel_fill(const ProbDev* probs, const TileItem* items,
                                                   const int32_t* sub_item, const char* store,
                                                   int m, double* vec, int64_t stride,
                                                   double* scal_all, double* rec) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1, r = 1 << m;
  const int64_t nn = (int64_t)n1 * n1;
  const int i_rhs = blockIdx.y;
  // the preconditioner of the first iteration runs before the scalars are set: clear the
  // flag a previous solve left
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal_all[i_rhs * SKEL_NS + 5] = 0.0;
    if (i_rhs == 0) rec[0] = rec[1] = 0.0;  // the solve's record (finished by k_skel_finish)
  }
  double* E = vec + (int64_t)i_rhs * stride;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  if (idx >= nn) return;
  const int gy = grid_row(idx, n1), gx = (int)(idx - (int64_t)gy * n1);
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
  const int gy = grid_row(idx, n1), gx = (int)(idx - (int64_t)gy * n1);
  double w = 0.0;
  if (skel_dof(P, N, r, gx, gy)) {
    double d;
    w = P.res[(int64_t)i_rhs * nn + idx] - apply_masked<KIND>(P, m, N, n1, gx, gy, idx, E, d);
  }
  Wv[idx] = w;
}

// Partial sums (w.z, w.w) after the preconditioner (level m = 1, where no tiled leg runs).
__global__ __launch_bounds__(NTS) void k_skel_dot(const ProbDev* probs, int m, const double* vec,
                                                  int64_t stride, int64_t w_off, int64_t z_off,
                                                  const double* scal_all, double* parts_all) {
  const ProbDev& P = probs[0];
  const int n1 = (P.n_c << m) + 1;
  const int64_t nn = (int64_t)n1 * n1;
  const int i_rhs = blockIdx.y;
  if (scal_all[i_rhs * SKEL_NS + 5] != 0.0) return;  // converged: frozen
  const double* Wv = vec + (int64_t)i_rhs * stride + w_off;
  const double* Z = vec + (int64_t)i_rhs * stride + z_off;
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

// e += alpha p, w_new = w - alpha q on S (0 elsewhere) (level m = 1).
__global__ __launch_bounds__(NTS) void k_skel_upd(const ProbDev* probs, int m, double* vec,
                                                  int64_t stride, int64_t w_off, int64_t wn_off,
                                                  int64_t p_off, const double* scal_all) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1, r = 1 << m;
  const int64_t nn = (int64_t)n1 * n1;
  const int i_rhs = blockIdx.y;
  const double* scal = scal_all + i_rhs * SKEL_NS;
  if (scal[5] != 0.0) return;  // converged: frozen
  double* base = vec + (int64_t)i_rhs * stride;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  if (idx >= nn) return;
  const double alpha = scal[1];
  const int gy = grid_row(idx, n1), gx = (int)(idx - (int64_t)gy * n1);
  double w = 0.0;
  if (skel_dof(P, N, r, gx, gy)) {
    base[V_E * nn + idx] += alpha * base[p_off + idx];
    w = base[w_off + idx] - alpha * base[V_Q * nn + idx];
  }
  base[wn_off + idx] = w;
}

// ---- the V-cycle on G_{m+1}; vectors are offsets (doubles) from vec + i * stride ----

// Tiles of TT x TT owned nodes (TT even, so coarse twins align): 32 on levels with many
// tiles, 16 where fewer tiles would leave compute units idle.
constexpr int TH = 3;  // halo: two sweeps and a residual reach three nodes out

// Skeleton membership of the staged square of side R at grid origin (ox, oy): per axis,
// whether the index lies in the closed G_b of its block (both axes in: inside a G_j), so a
// node's test is two LDS reads and is_dof instead of six integer divisions.
template <int R>
__device__ __forceinline__ void stage_axes(const ProbDev& P, int N, int r, int ox, int oy,
                                           unsigned char* ax, unsigned char* ay) {
  for (int t = threadIdx.x; t < 2 * R; t += NTS) {
    if (t < R) {
      const int g = ox + t;
      ax[t] = (g > 0 && g < N && g_block(P.n_c, P.sub_x, g, r) >= 0) ? 1 : 0;
    } else {
      const int g = oy + t - R;
      ay[t - R] = (g > 0 && g < N && g_block(P.n_c, P.sub_y, g, r) >= 0) ? 1 : 0;
    }
  }
}

// K v at the staged node li of a square of row length ld (its neighbours are staged too);
// d receives the diagonal.
template <int KIND>
__device__ __forceinline__ double lds_apply(const ProbDev& P, int l, int N, int gx, int gy,
                                            const double* v, int li, int ld, double& d) {
  const Weights W = edge_weights<KIND>(P, l, N, gx, gy);
  double ne = 0.0, sw = 0.0;
  if constexpr (KIND == 3) {
    ne = v[li + ld + 1];
    sw = v[li - ld - 1];
  }
  return apply_k<KIND, double>(W, v[li], v[li + 1], v[li - 1], v[li + ld], v[li - ld], ne, sw,
                               d);
}

// Down leg on level l >= 2, one tile of TT x TT nodes per workgroup (blockIdx.x, row-major
// over the level's tiles): x = omega D^-1 b (the first sweep, from zero), y = x + omega D^-1
// (b - A x), the residual b - A y and b_{l-1} = P^T (b - A y) (full weighting on the SW-NE
// mesh: the coarse node's fine twin 1, its six neighbours 1/2) at the coarse nodes whose
// twins the tile owns.  Stores y on the owned nodes.  With upd (level m) the CG update is
// fused in: b = w - alpha q wherever it is read, stored as w_new (and e += alpha p) on the
// owned nodes.
template <int KIND, int TT>
__global__ __launch_bounds__(NTS) void k_mg_down(const ProbDev* probs, int l, double* vec,
                                                 int64_t stride, int64_t b_off, int64_t y_off,
                                                 int64_t bc_off, int upd, int64_t wn_off,
                                                 int64_t p_off, const double* scal_all) {
  const ProbDev& P = probs[0];
  const int i_rhs = blockIdx.y;
  const double* scal = scal_all + i_rhs * SKEL_NS;
  if (scal[5] != 0.0) return;  // converged: frozen (uniform over the workgroup)
  constexpr int TR = TT + 2 * TH, S2 = TT + 4, S1 = TT + 2;
  __shared__ double sb[TR * TR], sx[TR * TR], sy[TR * TR];
  __shared__ unsigned char sm[TR * TR], ax[TR], ay[TR];
  const int N = P.n_c << l, n1 = N + 1, r = 1 << l;
  const int64_t nn = (int64_t)n1 * n1;
  const int tiles_x = (n1 + TT - 1) / TT;
  // grid coordinates of staged node (0, 0)
  const int ox = (int)(blockIdx.x % tiles_x) * TT - TH, oy = (int)(blockIdx.x / tiles_x) * TT - TH;
  double* base = vec + (int64_t)i_rhs * stride;
  const double alpha = upd ? scal[1] : 0.0;
  stage_axes<TR>(P, N, r, ox, oy, ax, ay);
  __syncthreads();
  for (int t = threadIdx.x; t < TR * TR; t += NTS) {
    const int lx = t % TR, ly = t / TR, gx = ox + lx, gy = oy + ly;
    const bool mk = is_dof(P.domain, N, gx, gy) && !(ax[lx] && ay[ly]);
    const int64_t g = (int64_t)gy * n1 + gx;
    double b = 0.0, x = 0.0;
    if (mk) {
      b = base[b_off + g];
      if (upd) b -= alpha * base[V_Q * nn + g];
      x = kMgOmega * b / diag_of<KIND>(edge_weights<KIND>(P, l, N, gx, gy));
    }
    if (upd && lx >= TH && lx < TH + TT && ly >= TH && ly < TH + TT && gx <= N && gy <= N) {
      base[wn_off + g] = b;
      if (mk) base[V_E * nn + g] += alpha * base[p_off + g];
    }
    sb[t] = b;
    sx[t] = x;
    sm[t] = mk ? 1 : 0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < S2 * S2; t += NTS) {
    const int lx = 1 + t % S2, ly = 1 + t / S2, li = ly * TR + lx;
    double y = 0.0;
    if (sm[li]) {
      double d;
      const double a = lds_apply<KIND>(P, l, N, ox + lx, oy + ly, sx, li, TR, d);
      y = sx[li] + kMgOmega * (sb[li] - a) / d;
    }
    sy[li] = y;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < S1 * S1; t += NTS) {  // the residual, into sx
    const int lx = 2 + t % S1, ly = 2 + t / S1, li = ly * TR + lx;
    double res = 0.0;
    if (sm[li]) {
      double d;
      res = sb[li] - lds_apply<KIND>(P, l, N, ox + lx, oy + ly, sy, li, TR, d);
    }
    sx[li] = res;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < TT * TT; t += NTS) {
    const int lx = TH + t % TT, ly = TH + t / TT, gx = ox + lx, gy = oy + ly;
    if (gx <= N && gy <= N) base[y_off + (int64_t)gy * n1 + gx] = sy[ly * TR + lx];
  }
  const int Nc = N >> 1, nc1 = Nc + 1;
  for (int t = threadIdx.x; t < (TT / 2) * (TT / 2); t += NTS) {
    const int Ix = (ox + TH) / 2 + t % (TT / 2), Iy = (oy + TH) / 2 + t / (TT / 2);
    if (Ix > Nc || Iy > Nc) continue;
    double val = 0.0;
    if (skel_dof(P, Nc, r >> 1, Ix, Iy)) {
      const int li = (2 * Iy - oy) * TR + (2 * Ix - ox);  // the fine twin (owned by the tile)
      val = sx[li];
      val += 0.5 * sx[li + 1];
      val += 0.5 * sx[li - 1];
      val += 0.5 * sx[li + TR];
      val += 0.5 * sx[li - TR];
      val += 0.5 * sx[li + TR + 1];
      val += 0.5 * sx[li - TR - 1];
    }
    base[bc_off + (int64_t)Iy * nc1 + Ix] = val;
  }
}

// Up leg on level l >= 2, one tile per workgroup: y^ = y + P x_{l-1} (P1 interpolation on the
// SW-NE mesh: the average of the coarse nodes at the ends of the coarse edge the node halves,
// or of the coarse node it coincides with), then x = y^ + omega D^-1 (b - A y^) and
// out = x + omega D^-1 (b - A x) on the owned nodes.  With dot (level m): the block partials
// (w.z, w.w) of b = w and z = out.
template <int KIND, int TT>
__global__ __launch_bounds__(NTS) void k_mg_up(const ProbDev* probs, int l, double* vec,
                                               int64_t stride, int64_t b_off, int64_t y_off,
                                               int64_t xc_off, int64_t out_off, int dot,
                                               double* parts_all, const double* scal_all) {
  const ProbDev& P = probs[0];
  const int i_rhs = blockIdx.y;
  if (scal_all[i_rhs * SKEL_NS + 5] != 0.0) return;  // converged: frozen
  constexpr int TR = TT + 2 * TH, S2 = TT + 4, S1 = TT + 2;
  __shared__ double sb[TR * TR], sx[TR * TR], sy[TR * TR];
  __shared__ unsigned char sm[TR * TR], ax[TR], ay[TR];
  const int N = P.n_c << l, n1 = N + 1, r = 1 << l, nc1 = (N >> 1) + 1;
  const int tiles_x = (n1 + TT - 1) / TT;
  const int ox = (int)(blockIdx.x % tiles_x) * TT - TH, oy = (int)(blockIdx.x / tiles_x) * TT - TH;
  double* base = vec + (int64_t)i_rhs * stride;
  const double* Xc = base + xc_off;
  stage_axes<TR>(P, N, r, ox, oy, ax, ay);
  __syncthreads();
  for (int t = threadIdx.x; t < S2 * S2; t += NTS) {
    const int lx = 1 + t % S2, ly = 1 + t / S2, li = ly * TR + lx;
    const int gx = ox + lx, gy = oy + ly;
    const bool mk = is_dof(P.domain, N, gx, gy) && !(ax[lx] && ay[ly]);
    double yh = 0.0, b = 0.0;
    if (mk) {
      const int64_t g = (int64_t)gy * n1 + gx;
      const int x0 = gx >> 1, y0 = gy >> 1, x1 = (gx + 1) >> 1, y1 = (gy + 1) >> 1;
      yh = base[y_off + g] + 0.5 * (Xc[(int64_t)y0 * nc1 + x0] + Xc[(int64_t)y1 * nc1 + x1]);
      b = base[b_off + g];
    }
    sy[li] = yh;
    sb[li] = b;
    sm[li] = mk ? 1 : 0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < S1 * S1; t += NTS) {
    const int lx = 2 + t % S1, ly = 2 + t / S1, li = ly * TR + lx;
    double x = 0.0;
    if (sm[li]) {
      double d;
      const double a = lds_apply<KIND>(P, l, N, ox + lx, oy + ly, sy, li, TR, d);
      x = sy[li] + kMgOmega * (sb[li] - a) / d;
    }
    sx[li] = x;
  }
  __syncthreads();
  double wz = 0.0, ww = 0.0;
  for (int t = threadIdx.x; t < TT * TT; t += NTS) {
    const int lx = TH + t % TT, ly = TH + t / TT, li = ly * TR + lx;
    const int gx = ox + lx, gy = oy + ly;
    if (gx > N || gy > N) continue;
    double z = 0.0;
    if (sm[li]) {
      double d;
      const double a = lds_apply<KIND>(P, l, N, gx, gy, sx, li, TR, d);
      z = sx[li] + kMgOmega * (sb[li] - a) / d;
    }
    base[out_off + (int64_t)gy * n1 + gx] = z;
    wz += sb[li] * z;
    ww += sb[li] * sb[li];
  }
  if (dot) block_partials(wz, ww, parts_all + (int64_t)i_rhs * 2 * gridDim.x);
}

// The bottom of the cycle: kMgCoarseSweeps damped Jacobi sweeps on level l from zero
// (x = omega D^-1 b, then sweeps alternating between two buffers), the level staged in LDS,
// one workgroup per right-hand side (blockIdx.x); the result goes to out.
constexpr int NTC = 1024;
constexpr int kCoarseLdsNodes = 6400;  // 3 vectors and a mask: 160000 bytes of LDS

__host__ __device__ inline size_t coarse_lds_bytes(int64_t nn) {
  return (size_t)(3 * nn) * sizeof(double) + (size_t)((nn + 7) / 8 * 8);
}

template <int KIND>
__global__ __launch_bounds__(NTC) void k_mg_coarse(const ProbDev* probs, int l, double* vec,
                                                   int64_t stride, int64_t b_off, int64_t out_off,
                                                   const double* scal_all) {
  const ProbDev& P = probs[0];
  const int i_rhs = blockIdx.x;
  if (scal_all[i_rhs * SKEL_NS + 5] != 0.0) return;  // converged: frozen
  extern __shared__ double coarse_lds[];
  const int N = P.n_c << l, n1 = N + 1, nn = n1 * n1, r = 1 << l;
  double* sb = coarse_lds;
  double* s0 = coarse_lds + nn;
  double* s1 = coarse_lds + 2 * nn;
  unsigned char* sm = reinterpret_cast<unsigned char*>(coarse_lds + 3 * nn);
  double* base = vec + (int64_t)i_rhs * stride;
  for (int idx = threadIdx.x; idx < nn; idx += NTC) {
    const int gy = grid_row(idx, n1), gx = idx - gy * n1;
    const bool mk = skel_dof(P, N, r, gx, gy);
    double b = 0.0, x = 0.0;
    if (mk) {
      b = base[b_off + idx];
      x = kMgOmega * b / diag_of<KIND>(edge_weights<KIND>(P, l, N, gx, gy));
    }
    sb[idx] = b;
    s0[idx] = x;
    sm[idx] = mk ? 1 : 0;
  }
  __syncthreads();
  for (int k = 1; k < kMgCoarseSweeps; ++k) {
    const double* in = (k & 1) ? s0 : s1;
    double* out = (k & 1) ? s1 : s0;
    for (int idx = threadIdx.x; idx < nn; idx += NTC) {
      double v = 0.0;
      if (sm[idx]) {  // an interior node: its neighbours are in the square
        const int gy = grid_row(idx, n1), gx = idx - gy * n1;
        double d;
        const double a = lds_apply<KIND>(P, l, N, gx, gy, in, idx, n1, d);
        v = in[idx] + kMgOmega * (sb[idx] - a) / d;
      }
      out[idx] = v;
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < nn; idx += NTC) base[out_off + idx] = s1[idx];
}

// One sweep of the bottom level with a thread per node, for levels too large for LDS:
// out = in + omega D^-1 (b - A in) (first: omega D^-1 b) on the region, 0 elsewhere.
template <int KIND>
__global__ __launch_bounds__(NTS) void k_mg_sweep(const ProbDev* probs, int l, double* vec,
                                                  int64_t stride, int64_t b_off, int64_t in_off,
                                                  int64_t out_off, int first,
                                                  const double* scal_all) {
  const ProbDev& P = probs[0];
  const int i_rhs = blockIdx.y;
  if (scal_all[i_rhs * SKEL_NS + 5] != 0.0) return;  // converged: frozen
  const int N = P.n_c << l, n1 = N + 1, r = 1 << l;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  if (idx >= (int64_t)n1 * n1) return;
  double* base = vec + (int64_t)i_rhs * stride;
  const int gy = grid_row(idx, n1), gx = (int)(idx - (int64_t)gy * n1);
  double v = 0.0;
  if (skel_dof(P, N, r, gx, gy)) {
    const double b = base[b_off + idx];
    if (first) {
      v = kMgOmega * b / diag_of<KIND>(edge_weights<KIND>(P, l, N, gx, gy));
    } else {
      const double* in = base + in_off;
      double d;
      const double a = apply_masked<KIND>(P, l, N, n1, gx, gy, idx, in, d);
      v = in[idx] + kMgOmega * (b - a) / d;
    }
  }
  base[out_off + idx] = v;
}

// p_new = z + beta p_old on S (formed on the fly at the stencil points; 0 off S), stored
// in Pn; q = A p_new on S; partial sums (p.q, 0).  first: beta = 0, p_old unread.
template <int KIND>
__global__ __launch_bounds__(NTS) void k_skel_dir(const ProbDev* probs, int m, double* vec,
                                                  int64_t stride, int64_t po_off, int64_t pn_off,
                                                  const double* scal_all, int first,
                                                  double* parts_all) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1, r = 1 << m;
  const int64_t nn = (int64_t)n1 * n1;
  const int i_rhs = blockIdx.y;
  const double* scal = scal_all + i_rhs * SKEL_NS;
  if (scal[5] != 0.0) return;  // converged: frozen (uniform over the workgroup)
  double* base = vec + (int64_t)i_rhs * stride;
  const double* Z = base + V_Z * nn;
  const double* Po = base + po_off;
  double* Pn = base + pn_off;
  double* Q = base + V_Q * nn;
  double* parts = parts_all + (int64_t)i_rhs * 2 * gridDim.x;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  const double beta = first ? 0.0 : scal[2];
  const double* Pold = first ? Z : Po;  // any valid vector: multiplied by 0
  double pq = 0.0;
  if (idx < nn) {
    const int gy = grid_row(idx, n1), gx = (int)(idx - (int64_t)gy * n1);
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

// Fixed-order sum of the block partials of right-hand side blockIdx.x, then its CG scalars:
//   stage 0 (after the first preconditioning):  rho = w.z, ||w||^2 = ||w_0||^2 = w.w,
//                          tol^2 = rtol^2 ||w_0||^2, iterations 0, done when w_0 = 0
//   stage 1 (after dir):   alpha = rho / p.q
//   stage 2 (after the update and preconditioning):  beta = (w.z) / rho, rho = w.z,
//                          ||w||^2 = w.w, iterations + 1, done when ||w||^2 <= tol^2
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

// u~ = I u + e for right-hand side i (0 off the domain); the solve's record takes the
// maximum over right-hand sides of the iterations and of ||w|| / ||w_0||.
__global__ __launch_bounds__(NTS) void k_skel_finish(const ProbDev* probs, int m,
                                                     const double* vec, int64_t stride,
                                                     const double* scal_all, double* rec) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1;
  const int64_t nn = (int64_t)n1 * n1;
  const int i_rhs = blockIdx.y;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double* c = scal_all + i_rhs * SKEL_NS;
    const double rel = c[4] > 0.0 ? sqrt(c[3] / c[4]) : 0.0;
    atomicMax(reinterpret_cast<unsigned long long*>(rec),
              (unsigned long long)__double_as_longlong(c[7]));
    atomicMax(reinterpret_cast<unsigned long long*>(rec + 1),
              (unsigned long long)__double_as_longlong(rel));
  }
  const double* E = vec + (int64_t)i_rhs * stride;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  if (idx >= nn) return;
  const int gy = grid_row(idx, n1), gx = (int)(idx - (int64_t)gy * n1);
  const int64_t o = (int64_t)i_rhs * nn + idx;
  P.ut[o] = is_dof(P.domain, N, gx, gy) ? P.ubar[o] + E[idx] : 0.0;
}

}  // namespace

hipError_t run_interface_gluing(int kind, const ProbDev* dprob, const TileItem* items,
                                const int32_t* sub_item, const char* store, int m, int q, int nc,
                                int64_t stride, double rtol, int max_it, bool poll, double* vec,
                                double* parts, double* scal, double* rec, hipStream_t s) {
  auto nodes_of = [&](int l) { return (int64_t)((nc << l) + 1) * ((nc << l) + 1); };
  auto grid_of = [&](int l) { return dim3((unsigned)((nodes_of(l) + NTS - 1) / NTS), (unsigned)q); };
  // tile side per level: 32 when that gives at least 8 workgroups per compute unit
  auto tile_side = [&](int l) {
    const int64_t t = ((nc << l) + 1 + 31) / 32;
    return t * t * q >= 2048 ? 32 : 16;
  };
  auto tiles_of = [&](int l) {
    const int tt = tile_side(l);
    const unsigned t = (unsigned)(((nc << l) + 1 + tt - 1) / tt);
    return dim3(t * t, (unsigned)q);
  };
  const int64_t nnm = nodes_of(m);
  // level-l (< m) vectors: b, y, x
  auto off = [&](int l, int which) {
    int64_t o = SKEL_VEC * nnm;
    for (int k = m - 1; k > l; --k) o += 3 * nodes_of(k);
    return o + which * nodes_of(l);
  };
  const unsigned nblk = (unsigned)((nnm + NTS - 1) / NTS);
  const unsigned ntile = tiles_of(m).x;
#define MLC_LEG(K, l, ...)                                                                \
  do {                                                                                    \
    if (tile_side(l) == 32)                                                               \
      MLC_SKEL2(K, 32, tiles_of(l), __VA_ARGS__);                                         \
    else                                                                                  \
      MLC_SKEL2(K, 16, tiles_of(l), __VA_ARGS__);                                         \
  } while (0)
#define MLC_SKEL2(K, T, G, ...)                                                           \
  do {                                                                                    \
    if (kind == 0)                                                                        \
      hipLaunchKernelGGL((K<0, T>), G, dim3(NTS), 0, s, __VA_ARGS__);                     \
    else if (kind == 1)                                                                   \
      hipLaunchKernelGGL((K<1, T>), G, dim3(NTS), 0, s, __VA_ARGS__);                     \
    else if (kind == 2)                                                                   \
      hipLaunchKernelGGL((K<2, T>), G, dim3(NTS), 0, s, __VA_ARGS__);                     \
    else                                                                                  \
      hipLaunchKernelGGL((K<3, T>), G, dim3(NTS), 0, s, __VA_ARGS__);                     \
  } while (0)
  const dim3 g(nblk, (unsigned)q);
#define MLC_SKEL(K, G, B, L, ...)                                                         \
  do {                                                                                    \
    if (kind == 0)                                                                        \
      hipLaunchKernelGGL(K<0>, G, dim3(B), L, s, __VA_ARGS__);                            \
    else if (kind == 1)                                                                   \
      hipLaunchKernelGGL(K<1>, G, dim3(B), L, s, __VA_ARGS__);                            \
    else if (kind == 2)                                                                   \
      hipLaunchKernelGGL(K<2>, G, dim3(B), L, s, __VA_ARGS__);                            \
    else                                                                                  \
      hipLaunchKernelGGL(K<3>, G, dim3(B), L, s, __VA_ARGS__);                            \
  } while (0)
  // the bottom of the cycle on level lc: b at b_off, the result to out_off (s0 a spare
  // vector of the level, used only when the level does not fit in LDS)
  auto coarse = [&](int lc, int64_t b_off, int64_t s0_off, int64_t out_off) {
    if (nodes_of(lc) <= kCoarseLdsNodes) {
      MLC_SKEL(k_mg_coarse, dim3((unsigned)q), NTC, coarse_lds_bytes(nodes_of(lc)), dprob, lc,
               vec, stride, b_off, out_off, scal);
    } else {
      MLC_SKEL(k_mg_sweep, grid_of(lc), NTS, 0, dprob, lc, vec, stride, b_off, b_off, s0_off, 1,
               scal);
      for (int k = 1; k < kMgCoarseSweeps; ++k) {
        const int64_t in = (k & 1) ? s0_off : out_off, out = (k & 1) ? out_off : s0_off;
        MLC_SKEL(k_mg_sweep, grid_of(lc), NTS, 0, dprob, lc, vec, stride, b_off, in, out, 0,
                 scal);
      }
    }
  };
  // z = B w (into Z) with w at w_off; upd: the CG update first (w_new to wn_off, e += alpha
  // p with p at p_off), and B applied to w_new; then the partials (w.z, w.w)
  auto precondition = [&](int64_t w_off, int upd, int64_t wn_off, int64_t p_off) {
    const int64_t wz = upd ? wn_off : w_off;  // the residual the cycle works on
    if (m == 1) {
      if (upd)
        hipLaunchKernelGGL(k_skel_upd, g, dim3(NTS), 0, s, dprob, m, vec, stride, w_off, wn_off,
                           p_off, scal);
      coarse(1, wz, V_Y * nnm, V_Z * nnm);
      hipLaunchKernelGGL(k_skel_dot, g, dim3(NTS), 0, s, dprob, m, vec, stride, wz, V_Z * nnm,
                         scal, parts);
      return nblk;
    }
    for (int l = m; l >= 2; --l) {
      const bool top = l == m;
      MLC_LEG(k_mg_down, l, dprob, l, vec, stride, top ? w_off : off(l, 0),
               top ? V_Y * nnm : off(l, 1), off(l - 1, 0), top ? upd : 0, wn_off, p_off, scal);
    }
    coarse(1, off(1, 0), off(1, 1), off(1, 2));
    for (int l = 2; l <= m; ++l) {
      const bool top = l == m;
      MLC_LEG(k_mg_up, l, dprob, l, vec, stride, top ? wz : off(l, 0),
               top ? V_Y * nnm : off(l, 1), off(l - 1, 2), top ? V_Z * nnm : off(l, 2),
               top ? 1 : 0, parts, scal);
    }
    return ntile;
  };
  hipLaunchKernelGGL(k_skel_fill, g, dim3(NTS), 0, s, dprob, items, sub_item, store, m, vec,
                     stride, scal, rec);
  MLC_SKEL(k_skel_init, g, NTS, 0, dprob, m, vec, stride);
  unsigned np = precondition(V_W * nnm, 0, 0, 0);
  hipLaunchKernelGGL(k_skel_reduce, dim3(q), dim3(1024), 0, s, parts, (int)np, 0, rtol, scal);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double h[SKEL_NS * MLC_MAX_Q];
  int it = 0;
  while (it < max_it) {
    // four iterations between polls of the convergence flags
    for (int k = 0; k < 4 && it < max_it; ++k, ++it) {
      const int c = it & 1;  // W_c and P_c hold the current residual and direction
      MLC_SKEL(k_skel_dir, g, NTS, 0, dprob, m, vec, stride, (V_P + c) * nnm,
               (V_P + 1 - c) * nnm, scal, it == 0 ? 1 : 0, parts);
      hipLaunchKernelGGL(k_skel_reduce, dim3(q), dim3(1024), 0, s, parts, (int)nblk, 1, rtol, scal);
      np = precondition((V_W + c) * nnm, 1, (V_W + 1 - c) * nnm, (V_P + 1 - c) * nnm);
      hipLaunchKernelGGL(k_skel_reduce, dim3(q), dim3(1024), 0, s, parts, (int)np, 2, rtol, scal);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (!poll) continue;
    if ((e = hipMemcpyAsync(h, scal, sizeof(double) * SKEL_NS * q, hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
      return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    bool all = true;
    for (int i = 0; i < q; ++i) all = all && h[i * SKEL_NS + 5] != 0.0;
    if (all) break;
  }
#undef MLC_SKEL
#undef MLC_SKEL2
#undef MLC_LEG
  hipLaunchKernelGGL(k_skel_finish, g, dim3(NTS), 0, s, dprob, m, vec, stride, scal, rec);
  return hipGetLastError();
}

// Doubles per right-hand side of the interface problem's vectors at finest level L.
int64_t skel_stride(int nc, int L) {
  auto nodes_of = [&](int l) { return (int64_t)((nc << l) + 1) * ((nc << l) + 1); };
  int64_t s = SKEL_VEC * nodes_of(L);
  for (int l = 1; l < L; ++l) s += 3 * nodes_of(l);
  return s;
}
