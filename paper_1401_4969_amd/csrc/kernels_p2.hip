// The correction step of Algorithm 4.1 with P2 elements (Section 2.1 with k = 2; Example
// 6.1 runs P1 and P2).  A level-m vector holds the P2 nodes of the mesh with n_c 2^m cells
// per side, i.e. the nodes of the grid with n_c 2^(m+1) intervals (p2_ops.h).  The
// gluing, the Rayleigh-Ritz solve and the output kernels are the P1 ones on that grid;
// this file holds what the element changes:
//   step 1: quadratic interpolation of u_k onto level k+1 (nested P2 spaces), the
//           residual lambda M u - K u with the P2 stencils, and the local solves:
//           conjugate gradients on the P2 stiffness of each tile, preconditioned by the P1
//           V-cycle on the same nodes (the P1 stiffness of the half-cell mesh is
//           spectrally equivalent to the P2 one, so the iteration count stays bounded in h);
//   step 3: K u~, M u~ and the transposed interpolation chain to the coarse P2 space, and
//           the coarse P2 part of the new eigenvector evaluated on the fine nodes;
//   setup (Algorithm 4.2 step 1): the coarse P2 stiffness and mass.
#include "p2_ops.h"
#include "pcg_ops.h"

namespace {

constexpr int NTP = 256;

inline unsigned nblk(int64_t n) { return (unsigned)((n + NTP - 1) / NTP); }

// Algorithm 4.1, step 1 (u_{h_k} in the finer space): u_bar = I u_k on P2 level m from
// level m-1: the coarse quadratic at every fine node.
__global__ __launch_bounds__(NTP) void k_p2_prolong(const ProbDev* probs, int m, int src) {
  const ProbDev& P = probs[blockIdx.y];
  if (m > P.L) return;
  const int i = blockIdx.z;
  if (i >= P.q) return;
  const int N = P.n_c << (m + 1);  // fine node grid
  const int n1 = N + 1;
  const int64_t nn = (int64_t)n1 * n1;
  const int64_t idx = (int64_t)blockIdx.x * NTP + threadIdx.x;
  if (idx >= nn) return;
  const int y = grid_row(idx, n1), x = (int)(idx - (int64_t)y * n1);
  double v = 0.0;
  if (is_dof(P.domain, N, x, y)) {
    const int nc1 = N / 2 + 1;  // coarse node grid
    const double* uc = P.u[src] + (int64_t)i * nc1 * nc1;
    // the fine node in units of 1/4 of a coarse cell (n_c 2^(m-1) cells per side)
    const p2::Loc L = p2::locate(x, y, 4, 2, P.n_c << (m - 1));
    double f[6];
    p2::shape(L.l0, L.l1, L.l2, f);
#pragma unroll
    for (int b = 0; b < 6; ++b)
      v += f[b] * uc[(int64_t)(2 * L.J + p2::node_dy_rt(L.up, b)) * nc1 + 2 * L.I +
                     p2::node_dx_rt(L.up, b)];
  }
  P.ubar[(int64_t)i * nn + idx] = v;
}

// Algorithm 4.1, step 1: r = lambda_k M u_bar - K u_bar (the right-hand side of
// (Aux_Problem)).
template <int KIND>
__global__ __launch_bounds__(NTP) void k_p2_residual(const ProbDev* probs, int m, int src) {
  // the step's convergence record starts empty (the local solves follow on the stream)
  if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0)
    probs[0].conv[m] = 0.0;
  const ProbDev& P = probs[blockIdx.y];
  if (m > P.L) return;
  const int i = blockIdx.z;
  if (i >= P.q) return;
  const int N = P.n_c << (m + 1);
  const int n1 = N + 1;
  const int64_t nn = (int64_t)n1 * n1;
  const int64_t idx = (int64_t)blockIdx.x * NTP + threadIdx.x;
  if (idx >= nn) return;
  const int y = grid_row(idx, n1), x = (int)(idx - (int64_t)y * n1);
  double r = 0.0;
  if (is_dof(P.domain, N, x, y)) {
    const double* ub = P.ubar + (int64_t)i * nn;
    // a dof's triangles lie inside the grid, so every offset node exists
    auto u = [&](int dx, int dy) -> double { return ub[idx + (int64_t)dy * n1 + dx]; };
    const double h = P.side / (double)(P.n_c << m);
    const double Ku = p2::apply_k<KIND>(P, m, x, y, u);
    const double Mu = p2::apply_m(x, y, h * h, u);
    r = P.lam[src * MLC_MAX_Q + i] * Mu - Ku;
  }
  P.res[(int64_t)i * nn + idx] = r;
}

// Algorithm 4.1, step 3 (the border of (Eigen_Augment_Problem)): y_K = K u~ (into res),
// y_M = M u~ (into ubar), and per-block partial sums of alpha_ij = u~_i . y_K,j,
// beta_ij = u~_i . y_M,j and s_i = sum u~_i (the layout the Rayleigh-Ritz solve reads).
constexpr int RNV2 = 2 * MLC_MAX_Q * MLC_MAX_Q + MLC_MAX_Q;

template <int KIND, int QM>
__global__ __launch_bounds__(NTP) void k_p2_rr_apply(const ProbDev* probs, int m) {
  __shared__ double red[(NTP / 64) * RNV2];
  const ProbDev& P = probs[blockIdx.y];
  if (m > P.L) return;
  const int N = P.n_c << (m + 1);
  const int n1 = N + 1;
  const int64_t nn = (int64_t)n1 * n1;
  const int64_t nb = (nn + NTP - 1) / NTP;
  if ((int64_t)blockIdx.x >= nb) return;
  const int64_t idx = (int64_t)blockIdx.x * NTP + threadIdx.x;
  const int q = P.q;
  const bool inr = idx < nn;
  int x = 0, y = 0;
  if (inr) {
    y = grid_row(idx, n1);
    x = (int)(idx - (int64_t)y * n1);
  }
  const bool dof = inr && is_dof(P.domain, N, x, y);
  const double h = P.side / (double)(P.n_c << m);
  double uv[QM], yk[QM], ym[QM];
#pragma unroll
  for (int i = 0; i < QM; ++i) {
    uv[i] = yk[i] = ym[i] = 0.0;
    if (i < q && dof) {
      const double* ut = P.ut + (int64_t)i * nn;
      auto u = [&](int dx, int dy) -> double { return ut[idx + (int64_t)dy * n1 + dx]; };
      uv[i] = ut[idx];
      yk[i] = p2::apply_k<KIND>(P, m, x, y, u);
      ym[i] = p2::apply_m(x, y, h * h, u);
    }
  }
#pragma unroll
  for (int i = 0; i < QM; ++i)
    if (i < q && inr) {
      P.res[(int64_t)i * nn + idx] = yk[i];
      P.ubar[(int64_t)i * nn + idx] = ym[i];
    }
  const int nv = 2 * q * q + q;
  double* out = P.partials + (int64_t)blockIdx.x * nv;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < QM; ++i) {
    if (i >= q) break;
#pragma unroll
    for (int j = 0; j < QM; ++j) {
      if (j >= q) break;
      const double a = wave_sum(uv[i] * yk[j]);
      const double c = wave_sum(uv[i] * ym[j]);
      if (lane == 0) {
        red[wid * RNV2 + i * q + j] = a;
        red[wid * RNV2 + q * q + i * q + j] = c;
      }
    }
    const double s = wave_sum(uv[i]);
    if (lane == 0) red[wid * RNV2 + 2 * q * q + i] = s;
  }
  __syncthreads();
  for (int v = threadIdx.x; v < nv; v += NTP) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NTP / 64; ++w) s += red[w * RNV2 + v];
    out[v] = s;
  }
}

// Algorithm 4.1, step 3 (continued): one level of the transposed interpolation, P2 level
// l+1 -> l, for the 2q border vectors: every coarse node gathers the fine values in its
// basis function's support (fine nodes within two coarse half steps), each weighted by
// that basis function at the fine node.  The coarse basis functions of one node class
// (vertex, x-, y- or diagonal-edge midpoint) are translates of each other on the uniform
// mesh, so each workgroup first tabulates the four classes' weights at the 9 x 9 fine
// offsets in LDS, evaluated at a coarse node away from the boundary (its triangles located
// as the interpolation locates them; exact dyadic values), and every node then reads its
// class's row.
__global__ __launch_bounds__(NTP) void k_p2_restrict(const ProbDev* probs, int l, int m) {
  __shared__ double wt[4][81];
  const ProbDev& P = probs[blockIdx.y];
  if (m > P.L) return;
  const int q = P.q;
  const int v = blockIdx.z;
  if (v >= 2 * q) return;
  for (int e = threadIdx.x; e < 4 * 81; e += NTP) {
    const int c = e / 81, k = e - 81 * c;
    const int dy = k / 9 - 4, dx = k - 9 * (k / 9) - 4;
    const int cx = 4 + (c & 1), cy = 4 + (c >> 1);  // a class-c node of an unbounded mesh
    const p2::Loc L = p2::locate(2 * cx + dx, 2 * cy + dy, 4, 2, 1 << 20);
    double sh[6];
    p2::shape(L.l0, L.l1, L.l2, sh);
    double w = 0.0;
#pragma unroll
    for (int bb = 0; bb < 6; ++bb)
      if (2 * L.I + p2::node_dx_rt(L.up, bb) == cx && 2 * L.J + p2::node_dy_rt(L.up, bb) == cy)
        w = sh[bb];
    wt[c][k] = w;
  }
  __syncthreads();
  const int Nc = P.n_c << (l + 1);  // coarse node grid
  const int nc1 = Nc + 1;
  const int64_t nnc = (int64_t)nc1 * nc1;
  const int64_t idx = (int64_t)blockIdx.x * NTP + threadIdx.x;
  if (idx >= nnc) return;
  const int cy = grid_row(idx, nc1), cx = (int)(idx - (int64_t)cy * nc1);
  const int Nf = 2 * Nc;
  const int nf1 = Nf + 1;
  const int64_t nnf = (int64_t)nf1 * nf1;
  double* outb = P.rchain + P.rchain_off[l];
  const double* f;
  if (l + 1 == m)
    f = (v < q ? P.res + (int64_t)v * nnf : P.ubar + (int64_t)(v - q) * nnf);
  else
    f = P.rchain + P.rchain_off[l + 1] + (int64_t)v * nnf;
  double val = 0.0;
  if (is_dof(P.domain, Nc, cx, cy)) {
    const double* w = wt[(cx & 1) | ((cy & 1) << 1)];
    for (int dy = -4; dy <= 4; ++dy) {
      const int fy = 2 * cy + dy;
      if (fy < 0 || fy > Nf) continue;
#pragma unroll
      for (int dx = -4; dx <= 4; ++dx) {
        const int fx = 2 * cx + dx;
        const double ww = w[9 * (dy + 4) + dx + 4];
        if (fx >= 0 && fx <= Nf && ww != 0.0) val += ww * f[(int64_t)fy * nf1 + fx];
      }
    }
  }
  outb[(int64_t)v * nnc + idx] = val;
}

// Algorithm 4.1, step 3 (the new eigenfunction): u_{k+1} = P_{0->m} c_H + sum_i t_i u~_i on
// P2 level m, the coarse quadratic evaluated at every fine node (a coarse cell spans
// 2^(m+1) fine half steps).
__global__ __launch_bounds__(NTP) void k_p2_assemble(const ProbDev* probs, int m, int dst) {
  const ProbDev& P = probs[blockIdx.y];
  if (m > P.L) return;
  const int k = blockIdx.z;
  if (k >= P.q) return;
  const int N = P.n_c << (m + 1);
  const int n1 = N + 1;
  const int64_t nn = (int64_t)n1 * n1;
  const int64_t idx = (int64_t)blockIdx.x * NTP + threadIdx.x;
  if (idx >= nn) return;
  const int y = grid_row(idx, n1), x = (int)(idx - (int64_t)y * n1);
  double val = 0.0;
  if (is_dof(P.domain, N, x, y)) {
    const p2::Loc L = p2::locate(x, y, 2 << m, m + 1, P.n_c);
    double f[6];
    p2::shape(L.l0, L.l1, L.l2, f);
    const double* c = P.cH_grid + (int64_t)k * P.c1 * P.c1;
#pragma unroll
    for (int b = 0; b < 6; ++b)
      val += f[b] * c[(2 * L.J + p2::node_dy_rt(L.up, b)) * P.c1 + 2 * L.I + p2::node_dx_rt(L.up, b)];
    for (int i = 0; i < P.q; ++i) val += P.rr_t[k * P.q + i] * P.ut[(int64_t)i * nn + idx];
  }
  P.u[dst][(int64_t)k * nn + idx] = val;
}

// setup: the coarse P2 stiffness K_H and mass M_H (column-major, one column per thread:
// the entries of coarse dof r against every node within two half steps, each found by
// applying the stencils to that node's unit vector).
template <int KIND>
__global__ __launch_bounds__(NTP) void k_p2_coarse_matrices(const ProbDev* probs) {
  const ProbDev& P = probs[blockIdx.y];
  const int r = blockIdx.x * NTP + threadIdx.x;
  if (r >= P.nH) return;
  const int n1 = P.c1;
  const int node = P.coarse_nodes[r];
  const int y = node / n1, x = node - y * n1;
  const double H = P.side / (double)P.n_c;
  const int nH = P.nH;
  for (int dy = -2; dy <= 2; ++dy)
    for (int dx = -2; dx <= 2; ++dx) {
      const int jx = x + dx, jy = y + dy;
      if (jx < 0 || jy < 0 || jx >= n1 || jy >= n1) continue;
      const int c = P.coarse_index[jy * n1 + jx];
      if (c < 0) continue;
      auto e = [&](int ox, int oy) -> double { return (ox == dx && oy == dy) ? 1.0 : 0.0; };
      P.Kc[(int64_t)c * nH + r] = p2::apply_k<KIND>(P, 0, x, y, e);
      P.Mc[(int64_t)c * nH + r] = p2::apply_m(x, y, H * H, e);
    }
}

// ---- Algorithm 4.1, step 1: local solves ----

// Tile vectors: the value at the node offset by (dx, dy), 0 off the tile (the Dirichlet
// boundary of Omega_j); loads are issued from clamped indices and then selected.
template <typename V>
__device__ __forceinline__ double tile_at(const LevelDesc& l0, int ix, int iy, int dx, int dy,
                                          const V& val) {
  const int jx = ix + dx, jy = iy + dy;
  const bool in = jx >= 0 && jx < l0.nx && jy >= 0 && jy < l0.ny;
  const unsigned j = (unsigned)((in ? jy : iy) * l0.nx + (in ? jx : ix));
  const double v = val(j);
  return in ? v : 0.0;
}

// p = z + beta p_old (beta = 0 and p_old unread on the first iteration): a streaming pass.
template <int NT>
__device__ void pass_dir_p2(const LevelDesc& l0, const double* Z, const double* Po, double* Pn,
                            double beta, bool first) {
  const double bet = first ? 0.0 : beta;
  const double* Pold = first ? Z : Po;  // any valid vector: its values are multiplied by 0
  FOR_TILE(l0) {
    const unsigned i = (unsigned)(iy * l0.nx + ix);
    Pn[i] = Z[i] + bet * Pold[i];
  }
}

// q = K2 p (the P2 stiffness of the tile), stored, and this thread's share of p . q.  The
// P2 stencil gathers up to 19 nodes, so q is kept for the update pass instead of being
// formed again there.
template <int NT, int KIND>
__device__ void pass_apply_p2(const ProbDev& P, const LevelDesc& l0, const double* Pn, double* Q,
                              double* acc) {
  const int lm = l0.l - 1;  // P2 mesh level of the tile's node grid
  FOR_TILE(l0) {
    const unsigned i = (unsigned)(iy * l0.nx + ix);
    double q = 0.0;
    if (is_dof(P.domain, l0.N, l0.gx0 + ix, l0.gy0 + iy)) {
      auto pv = [&](unsigned j) -> double { return Pn[j]; };
      auto u = [&](int dx, int dy) -> double { return tile_at(l0, ix, iy, dx, dy, pv); };
      q = p2::apply_k<KIND>(P, lm, l0.gx0 + ix, l0.gy0 + iy, u);
      *acc += Pn[i] * q;
    }
    Q[i] = q;
  }
}

// x += alpha p, r -= alpha q: a streaming pass (x_0 = 0 is not read).
template <int NT>
__device__ void pass_xr_p2(const LevelDesc& l0, double* X, double* R, const double* Pn,
                           const double* Q, double alpha, bool first, double* acc) {
  FOR_TILE(l0) {
    const unsigned i = (unsigned)(iy * l0.nx + ix);
    X[i] = (first ? 0.0 : X[i]) + alpha * Pn[i];
    const double r = R[i] - alpha * Q[i];
    R[i] = r;
    *acc += r * r;
  }
}

// Banded forms of the CG passes (tile rows of at most RING_CHUNKS * 64 nodes): the
// workgroup walks the tile in bands of BH = RW * NW rows (RW rows per wave) with one LDS
// ring of BH + 4 rows of p (the P2 stencil reaches two rows; rows -2, -1, ny and ny + 1
// hold zeros, the Dirichlet values).  At step k the waves form or stage rows k BH - 2 to
// k BH + BH - 3 of p in the ring (first stage), and after a barrier apply K2 to the rows
// two above them from the ring (second stage), so K2 p needs no global gathers and
// q = K2 p is not stored.  A ring row is overwritten only after the barrier that follows
// its last reader.  BH + 4 rows fit the three-ring space of the smoothing passes
// (3 (NW + 2) rows) for RW = 3; tall bands keep the barriers per pass few.
template <int NT>
struct P2Ring {
  static constexpr int NW = NT / 64, RW = 3, BH = RW * NW, RING = BH + 4, CM = RING_CHUNKS;
  double* ring;
  int nx;
  __device__ double* row(int y) const { return ring + ((y + 2) % RING) * nx; }
  // row j of wave w in the first stage of step k
  __device__ static int row_a(int k, int j, int w) { return k * BH + j * NW + w - 2; }
  __device__ static bool more(int k, int ny) { return k * BH - 4 < ny; }
};

// K2 p at tile node (ix, y) (a dof) from the ring.
template <int NT, int KIND>
__device__ __forceinline__ double ring_k2(const ProbDev& P, const LevelDesc& l0, int lm,
                                          const P2Ring<NT>& rg, int ix, int y) {
  auto u = [&](int dx, int dy) -> double {
    const int jx = ix + dx;
    const bool in = jx >= 0 && jx < l0.nx;
    const double v = rg.row(y + dy)[in ? jx : ix];
    return in ? v : 0.0;
  };
  return p2::apply_k<KIND>(P, lm, l0.gx0 + ix, l0.gy0 + y, u);
}

// p_new = z + beta p_old (stored) and this thread's share of p_new . K2 p_new.
template <int NT, int KIND>
__device__ void pass_dir_p2_banded(const ProbDev& P, const LevelDesc& l0, const double* Z,
                                   const double* Po, double* Pn, double beta, bool first,
                                   double* ring, double* acc) {
  using RG = P2Ring<NT>;
  constexpr int RW = RG::RW, CM = RG::CM;
  const RG rg{ring, l0.nx};
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nx = l0.nx, ny = l0.ny, nch = (nx + 63) >> 6, lm = l0.l - 1;
  const double bet = first ? 0.0 : beta;
  const double* Pold = first ? Z : Po;  // any valid vector: its values are multiplied by 0
  for (int k = 0; RG::more(k, ny); ++k) {
#pragma unroll 1
    for (int j = 0; j < RW; ++j) {
      const int ya = RG::row_a(k, j, w);
      if (ya > ny + 1) break;
      const bool inA = ya >= 0 && ya < ny;
      double zv[CM], pv[CM];
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        if (c < nch) {
          const int ix = lane + 64 * c;
          const unsigned i = (inA && ix < nx) ? (unsigned)(ya * nx + ix) : 0u;
          zv[c] = Z[i];
          pv[c] = Pold[i];
        }
      }
      double* dst = rg.row(ya);
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        const int ix = lane + 64 * c;
        if (c < nch && ix < nx) {
          double v = 0.0;
          if (inA) {
            v = zv[c] + bet * pv[c];
            Pn[(unsigned)(ya * nx + ix)] = v;
          }
          dst[ix] = v;
        }
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int j = 0; j < RW; ++j) {
      const int yb = RG::row_a(k, j, w) - 2;
      if (yb < 0 || yb >= ny) continue;
      const double* rc = rg.row(yb);
#pragma unroll 1
      for (int ix = lane; ix < nx; ix += 64) {
        if (is_dof(P.domain, l0.N, l0.gx0 + ix, l0.gy0 + yb))
          *acc += rc[ix] * ring_k2<NT, KIND>(P, l0, lm, rg, ix, yb);
      }
    }
    __syncthreads();
  }
}

// x += alpha p, r -= alpha K2 p and this thread's share of ||r||^2, with p staged in the
// ring.
template <int NT, int KIND>
__device__ void pass_xr_p2_banded(const ProbDev& P, const LevelDesc& l0, double* X, double* R,
                                  const double* Pn, double alpha, bool first, double* ring,
                                  double* acc) {
  using RG = P2Ring<NT>;
  constexpr int RW = RG::RW, CM = RG::CM;
  const RG rg{ring, l0.nx};
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nx = l0.nx, ny = l0.ny, nch = (nx + 63) >> 6, lm = l0.l - 1;
  for (int k = 0; RG::more(k, ny); ++k) {
#pragma unroll 1
    for (int j = 0; j < RW; ++j) {
      const int ya = RG::row_a(k, j, w);
      if (ya > ny + 1) break;
      const bool inA = ya >= 0 && ya < ny;
      double pv[CM];
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        if (c < nch) {
          const int ix = lane + 64 * c;
          const int jx = ix < nx ? ix : nx - 1;
          pv[c] = Pn[inA ? (unsigned)(ya * nx + jx) : 0u];
        }
      }
      double* dst = rg.row(ya);
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        const int ix = lane + 64 * c;
        if (c < nch && ix < nx) dst[ix] = inA ? pv[c] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int j = 0; j < RW; ++j) {
      const int yb = RG::row_a(k, j, w) - 2;
      if (yb < 0 || yb >= ny) continue;
      const double* rc = rg.row(yb);
#pragma unroll 1
      for (int ix = lane; ix < nx; ix += 64) {
        const unsigned i = (unsigned)(yb * nx + ix);
        const double xo = first ? 0.0 : X[i], ro = R[i];  // x_0 = 0 is not read
        double q = 0.0;
        if (is_dof(P.domain, l0.N, l0.gx0 + ix, l0.gy0 + yb))
          q = ring_k2<NT, KIND>(P, l0, lm, rg, ix, yb);
        X[i] = xo + alpha * rc[ix];
        const double r = ro - alpha * q;
        R[i] = r;
        *acc += r * r;
      }
    }
    __syncthreads();
  }
}

// Conjugate gradients on the P2 tile problem K2 e = r, preconditioned by the P1 V-cycle
// on the same nodes (levels: the tile's node grid, then the coarser P1 grids down to the
// coarse-cell grid of Omega_j, solved exactly); the same loop as the P1 solver.
template <int NT, int KIND>
__device__ int pcg_solve_p2(const ProbDev& P, const Levels& lev, double* base, int mg,
                            const double* Kinv, double bb, double tol2, int max_it, int nu,
                            double omega, double omega2, double* red, double* ring, int ring_rows,
                            double* tail, double& rr) {
  const LevelDesc l0 = lev[0];
  const int64_t S0 = (int64_t)l0.nx * l0.ny;
  double* X = base;
  double* R = base + l0.ob;
  double* Po = base + 4 * S0;
  double* Pn = base + 5 * S0;
  double* Q = base + l0.ot;  // the V-cycle's level-0 temporary, free between V-cycles
  int iters = 0;
  rr = bb;
  double acc[2];
  const double* Z = nullptr;
  double rho = 0.0, beta = 0.0;
  bool first = true;
  for (;;) {
    if (Z != nullptr) {
      if (iters >= max_it) break;
      ++iters;
      acc[0] = acc[1] = 0.0;
      const bool banded = ring != nullptr && l0.nx <= 64 * RING_CHUNKS;
      if (banded) {
        pass_dir_p2_banded<NT, KIND>(P, l0, Z, Po, Pn, beta, first, ring, &acc[0]);
      } else {
        pass_dir_p2<NT>(l0, Z, Po, Pn, beta, first);
        __syncthreads();
        pass_apply_p2<NT, KIND>(P, l0, Pn, Q, &acc[0]);
      }
      block_sum<NT, 2>(acc, red);
      // a zero right-hand side gives p = 0: alpha = 0 writes x_1 = 0 and r stays 0
      const double alpha = acc[0] > 0.0 ? rho / acc[0] : 0.0;
      acc[0] = acc[1] = 0.0;
      if (banded)
        pass_xr_p2_banded<NT, KIND>(P, l0, X, R, Pn, alpha, first, ring, &acc[0]);
      else
        pass_xr_p2<NT>(l0, X, R, Pn, Q, alpha, first, &acc[0]);
      block_sum<NT, 2>(acc, red);
      rr = acc[0];
      if (rr <= tol2) break;
    }
    acc[0] = acc[1] = 0.0;
    const bool init = Z == nullptr;
    Z = vcycle<NT, KIND, double, 2>(P, lev, base, mg, Kinv, nu, omega, omega2, &acc[0], ring,
                                    ring_rows,
                                    tail);
    block_sum<NT, 2>(acc, red);
    if (init) {
      rho = acc[0];
      continue;
    }
    beta = acc[0] / rho;
    rho = acc[0];
    first = false;
    double* tmp = Po;
    Po = Pn;
    Pn = tmp;
  }
  return iters;
}

template <int NT, int KIND>
__global__ __launch_bounds__(NT) void k_local_p2(const ProbDev* probs, const TileItem* items,
                                                  char* store, const double* inv, int m,
                                                  ItemStat* stats, double rtol, int max_it,
                                                  int nu, double omega, double omega2, int ring_cap,
                                                  int ring_cap2) {
  __shared__ double red[2 * (NT / 64)];
  extern __shared__ double ring_lds_p2[];
  const TileItem it = items[blockIdx.x];
  const ProbDev& P = probs[it.prob];
  const int mg = m + 1;  // the tile's node grid is P1 level m + 1 of the same cells
  const Levels lev(it, P, mg, 2);
  double* base = reinterpret_cast<double*>(store + it.off);
  const LevelDesc l0 = lev[0];
  double* X = base;
  double* R = base + l0.ob;
  const int n1 = l0.N + 1;
  const double* bglob = P.res + (int64_t)it.rhs * n1 * n1;
  double acc[2] = {0.0, 0.0};
  FOR_TILE(l0) {
    const unsigned i = (unsigned)(iy * l0.nx + ix);
    const double v = bglob[(int64_t)(l0.gy0 + iy) * n1 + (l0.gx0 + ix)];
    R[i] = v;  // x is written by the first update, without being read
    acc[0] += v * v;
  }
  block_sum<NT, 2>(acc, red);
  const double bb = acc[0];
  double rr = bb;
  const int rows = l0.nx <= ring_cap2 ? 2 : (l0.nx <= ring_cap ? 1 : 0);
  double* ring = rows ? ring_lds_p2 : nullptr;
  double* tail =
      (rows && NT == 1024) ? ring_lds_p2 + ring_elems(NT / 64, ring_cap, ring_cap2) : nullptr;
  const int iters = pcg_solve_p2<NT, KIND>(P, lev, base, mg, inv + it.inv_off, bb,
                                           rtol * rtol * bb, max_it, nu, omega, omega2, red, ring, rows,
                                           tail, rr);
  if (threadIdx.x == 0) {
    ItemStat s;
    s.iters = iters;
    s.refine = 0;
    s.relres = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    stats[blockIdx.x] = s;
    atomicMax(reinterpret_cast<unsigned long long*>(P.conv + m),
              (unsigned long long)__double_as_longlong(s.relres));
  }
}

}  // namespace

hipError_t launch_p2_prolong_residual(int kind, const ProbDev* probs, int nprob, int m, int src,
                                      int64_t max_nodes, int max_q, hipStream_t s) {
  const dim3 g(nblk(max_nodes), nprob, max_q);
  hipLaunchKernelGGL(k_p2_prolong, g, dim3(NTP), 0, s, probs, m, src);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (kind == 0)
    hipLaunchKernelGGL(k_p2_residual<0>, g, dim3(NTP), 0, s, probs, m, src);
  else
    hipLaunchKernelGGL(k_p2_residual<1>, g, dim3(NTP), 0, s, probs, m, src);
  return hipGetLastError();
}

hipError_t launch_p2_rr_apply(int kind, const ProbDev* probs, int nprob, int m, int64_t max_nodes,
                              int max_q, hipStream_t s) {
  const dim3 g(nblk(max_nodes), nprob);
#define MLC_P2A(K, QM) hipLaunchKernelGGL((k_p2_rr_apply<K, QM>), g, dim3(NTP), 0, s, probs, m)
#define MLC_P2A_Q(K)   \
  if (max_q <= 1)      \
    MLC_P2A(K, 1);     \
  else if (max_q <= 2) \
    MLC_P2A(K, 2);     \
  else if (max_q <= 4) \
    MLC_P2A(K, 4);     \
  else                 \
    MLC_P2A(K, 8)
  if (kind == 0) {
    MLC_P2A_Q(0);
  } else {
    MLC_P2A_Q(1);
  }
#undef MLC_P2A_Q
#undef MLC_P2A
  return hipGetLastError();
}

hipError_t launch_p2_restrict(const ProbDev* probs, int nprob, int l, int m, int64_t max_nodes_l,
                              int max_q, hipStream_t s) {
  hipLaunchKernelGGL(k_p2_restrict, dim3(nblk(max_nodes_l), nprob, 2 * max_q), dim3(NTP), 0, s,
                     probs, l, m);
  return hipGetLastError();
}

hipError_t launch_p2_assemble(const ProbDev* probs, int nprob, int m, int dst, int64_t max_nodes,
                              int max_q, hipStream_t s) {
  hipLaunchKernelGGL(k_p2_assemble, dim3(nblk(max_nodes), nprob, max_q), dim3(NTP), 0, s, probs,
                     m, dst);
  return hipGetLastError();
}

hipError_t launch_p2_coarse_matrices(int kind, const ProbDev* probs, int nprob, int max_nH,
                                     hipStream_t s) {
  const dim3 g(nblk(max_nH), nprob);
  if (kind == 0)
    hipLaunchKernelGGL(k_p2_coarse_matrices<0>, g, dim3(NTP), 0, s, probs);
  else
    hipLaunchKernelGGL(k_p2_coarse_matrices<1>, g, dim3(NTP), 0, s, probs);
  return hipGetLastError();
}

hipError_t launch_local_p2(int kind, int nt, const ProbDev* probs, const TileItem* items,
                           int nitems, char* store, const double* inv, int m, ItemStat* stats,
                           double rtol, int max_it, int nu, double omega, double omega2,
                           int max_tile_nx,
                           hipStream_t s) {
  const int ntv = nt == 256 ? 256 : (nt == 512 ? 512 : 1024);
  size_t lds = 0;
  int cap2 = 0;
  const int cap = ring_capacity(ntv, nu, max_tile_nx, 8, ntv == 1024, &lds, &cap2);
#define MLC_LP2(NTV, KV)                                                                    \
  hipLaunchKernelGGL((k_local_p2<NTV, KV>), dim3(nitems), dim3(NTV), lds, s, probs, items, \
                     store, inv, m, stats, rtol, max_it, nu, omega, omega2, cap, cap2)
#define MLC_LP2_NT(NTV) \
  if (kind == 0)        \
    MLC_LP2(NTV, 0);    \
  else                  \
    MLC_LP2(NTV, 1);
  if (nt == 256) {
    MLC_LP2_NT(256)
  } else if (nt == 512) {
    MLC_LP2_NT(512)
  } else {
    MLC_LP2_NT(1024)
  }
#undef MLC_LP2_NT
#undef MLC_LP2
  return hipGetLastError();
}
