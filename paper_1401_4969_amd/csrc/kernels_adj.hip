// Reverse sweep (adjoint) of the multilevel correction for d lambda_1 / d kappa.
//
// The derivative is that of the computed finest eigenvalue lambda_L(kappa) through every
// level: the Rayleigh-Ritz steps (equation (Eigen_Augment_Problem)), the gluing, the local
// solves of (Aux_Problem), the residuals, the coarse eigenproblem of Algorithm 4.2 step 1
// and the children-mean coefficients of the coarser levels.  Per level m (k = m-1), with
// the adjoints lambda_bar_m and u_bar_m of the level's eigenpair (u = S c, S = [P V, u~],
// A = S^T K S, B = S^T M S, A c = mu B c, c^T B c = 1):
//   c_bar = S^T u_bar;  [A - mu B, B c; (B c)^T, 0] [g; nu] = [c_bar; 0]  (bordered solve)
//   K_bar = lambda_bar u u^T - (s u^T + u s^T)/2,  s = S g
//   u~_bar = (2 lambda_bar c_u - g_u)(K u - mu M u) - c_u (K s - mu M s) - nu c_u M u + c_u u_bar
//   e_bar_j = chi_j u~_bar;  z_j = K_j^-1 e_bar_j;  kappa_bar -= z_j^T dK e_j;  r_bar = sum_j z_j
//   lambda_bar_k = r_bar^T M u_bar_k-interp;  u_bar_k = P^T (u~_bar + lambda_k M r_bar - K r_bar)
//   kappa_bar += lambda_bar u^T dK u - s^T dK u - r_bar^T dK (P u_k)
// and at level 0 the eigenvector derivative through the full coarse eigenbasis.  The
// per-triangle products are a^T dK_T b = (1/2) sum over the two legs of T of the
// products of the differences of a and b along the leg; the coarser-level kappa of a
// triangle is the mean of its four children, so its adjoint passes 1/4 to each child.
#include "mlc_launch.h"

namespace {

constexpr int NTA = 256;

inline unsigned nb(int64_t n) { return (unsigned)((n + NTA - 1) / NTA); }

__device__ __forceinline__ double interp2(const double* uc, int nc1, int x, int y) {
  const int ix = x >> 1, iy = y >> 1;
  const double a = uc[iy * nc1 + ix];
  if (x & 1) {
    if (y & 1) return 0.5 * (a + uc[(iy + 1) * nc1 + ix + 1]);
    return 0.5 * (a + uc[iy * nc1 + ix + 1]);
  }
  if (y & 1) return 0.5 * (a + uc[(iy + 1) * nc1 + ix]);
  return a;
}

__device__ __forceinline__ double interp_coarse(const double* c, int nc, int m, int gx, int gy) {
  const int nc1 = nc + 1;
  const int I = min(gx >> m, nc - 1), J = min(gy >> m, nc - 1);
  const int a = gx - (I << m), b = gy - (J << m);
  const double inv_r = 1.0 / (double)(1 << m);
  const double c00 = c[J * nc1 + I], c10 = c[J * nc1 + I + 1];
  const double c01 = c[(J + 1) * nc1 + I], c11 = c[(J + 1) * nc1 + I + 1];
  if (a >= b) return c00 + (a * (c10 - c00) + b * (c11 - c10)) * inv_r;
  return c00 + (b * (c01 - c00) + a * (c11 - c01)) * inv_r;
}

template <int KIND>
__device__ __forceinline__ void K_and_M(const ProbDev& P, int m, int N, const double* u, int64_t i,
                                        int gx, int gy, double& Ku, double& Mu) {
  const int n1 = N + 1;
  const Weights W = edge_weights<KIND>(P, m, N, gx, gy);
  const double c = u[i], e = u[i + 1], w = u[i - 1], n = u[i + n1], s = u[i - n1];
  Ku = (W.e + W.w + W.n + W.s) * c - W.e * e - W.w * w - W.n * n - W.s * s;
  const double h = P.side / N;
  Mu = h * h / 12.0 * (6.0 * c + e + w + n + s + u[i + n1 + 1] + u[i - n1 - 1]);
}

// Copy the local corrections e_j of a level into the tape (item order, contiguous).
__global__ __launch_bounds__(NTA) void k_tape_tiles(const TileItem* items, const char* store,
                                                    int m, double* te, const int64_t* te_off) {
  const TileItem it = items[blockIdx.x];
  const int r = 1 << m;
  const int64_t S = (int64_t)(it.cw * r - 1) * (it.ch * r - 1);
  const double* x = reinterpret_cast<const double*>(store + it.off);
  double* out = te + te_off[blockIdx.x];
  for (int64_t i = threadIdx.x; i < S; i += NTA) out[i] = x[i];
}

// out (level l) = P^T in (level l+1), on interior nodes.
__global__ __launch_bounds__(NTA) void k_restrict1(const ProbDev* probs, const double* in,
                                                   double* out, int l) {
  const ProbDev& P = probs[0];
  const int Nc = P.n_c << l, nc1 = Nc + 1, nf1 = 2 * Nc + 1;
  const int64_t idx = (int64_t)blockIdx.x * NTA + threadIdx.x;
  if (idx >= (int64_t)nc1 * nc1) return;
  const int Iy = grid_row(idx, nc1), Ix = (int)(idx - (int64_t)Iy * nc1);
  double v = 0.0;
  if (is_dof(P.domain, Nc, Ix, Iy)) {
    const int64_t c = (int64_t)(2 * Iy) * nf1 + 2 * Ix;
    v = in[c] + 0.5 * (in[c + 1] + in[c - 1] + in[c + nf1] + in[c - nf1] + in[c + nf1 + 1] +
                       in[c - nf1 - 1]);
  }
  out[idx] = v;
}

// out[c] = sum_r V[r, c] a[node r] (one wave per coarse eigenvector c)
__global__ __launch_bounds__(NTA) void k_coarse_project(const ProbDev* probs, const double* a,
                                                        double* out) {
  const ProbDev& P = probs[0];
  const int c = blockIdx.x * (NTA / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= P.nH) return;
  const double* col = P.V + (int64_t)c * P.nH;
  double s = 0.0;
  for (int r = lane; r < P.nH; r += 64) s += col[r] * a[P.coarse_nodes[r]];
  s = wave_sum(s);
  if (lane == 0) out[c] = s;
}

// grid (coarse) = V y: one wave per coarse node over a row of V^T
__global__ __launch_bounds__(NTA) void k_coarse_combine(const ProbDev* probs, const double* y,
                                                        double* grid) {
  const ProbDev& P = probs[0];
  const int nc1 = P.n_c + 1;
  const int node = blockIdx.x * (NTA / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (node >= nc1 * nc1) return;
  const int r = P.coarse_index[node];
  double s = 0.0;
  if (r >= 0) {
    const double* row = P.VT + (int64_t)r * P.nH;
    for (int c = lane; c < P.nH; c += 64) s += row[c] * y[c];
    s = wave_sum(s);
  }
  if (lane == 0) grid[node] = s;
}

// Per-block partial sums of a . b (plain) or a . (M b) (mass) on level m.
template <bool MASS>
__global__ __launch_bounds__(NTA) void k_dot(const ProbDev* probs, int m, const double* a,
                                             const double* b, double* parts) {
  __shared__ double red[NTA / 64];
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1;
  const int64_t nn = (int64_t)n1 * n1;
  const int64_t idx = (int64_t)blockIdx.x * NTA + threadIdx.x;
  double v = 0.0;
  if (idx < nn) {
    const int gy = grid_row(idx, n1), gx = (int)(idx - (int64_t)gy * n1);
    if (is_dof(P.domain, N, gx, gy)) {
      if (MASS) {
        const double h = P.side / N;
        const double mb = h * h / 12.0 *
                          (6.0 * b[idx] + b[idx + 1] + b[idx - 1] + b[idx + n1] + b[idx - n1] +
                           b[idx + n1 + 1] + b[idx - n1 - 1]);
        v = a[idx] * mb;
      } else {
        v = a[idx] * b[idx];
      }
    }
  }
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < NTA / 64; ++w) s += red[w];
    parts[blockIdx.x] = s;
  }
}

// out[0] = sum of parts[0..n) in a fixed order (one workgroup)
__global__ __launch_bounds__(NTA) void k_sum_to(const double* parts, int n, double* out) {
  __shared__ double red[NTA / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += NTA) s += parts[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NTA / 64; ++w) t += red[w];
    out[0] = t;
  }
}

// Bordered solve of the Rayleigh-Ritz adjoint in the [P V, u~] basis (one workgroup).
// rr: c_H[nH], c_u, f[nH], g[nH], alpha, beta, mu.  cbar_H[nH], cbar_u (scalar),
// lam_bar (scalar).  Out: y_H[nH] (y), coef[0..5] = {2 lam_bar c_u - y_u, -c_u,
// -nu c_u, c_u, y_u, nu}.
__global__ __launch_bounds__(NTA) void k_adj_rr(const ProbDev* probs, const double* rr,
                                                const double* cbar_H, const double* cbar_u,
                                                const double* lam_bar, double* y, double* coef) {
  __shared__ double red[5 * (NTA / 64)];
  __shared__ double sol[2];
  const ProbDev& P = probs[0];
  const int nH = P.nH;
  const double* cH = rr;
  const double cu = rr[nH];
  const double* f = rr + nH + 1;
  const double* g = rr + 2 * nH + 1;
  const double alpha = rr[3 * nH + 1], beta = rr[3 * nH + 2], mu = rr[3 * nH + 3];
  // A - mu B = [[D, h], [h^T, d]], D = Lambda - mu, h = f - mu g, d = alpha - mu beta;
  // B c = [p; pi], p = c_H + g c_u, pi = g^T c_H + beta c_u.
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // h'Dh, h'Dp, p'Dp, h'Dcb, p'Dcb ; and g'cH
  double gch = 0.0;
  for (int r = threadIdx.x; r < nH; r += NTA) {
    const double D = P.Lam[r] - mu;
    const double h = f[r] - mu * g[r];
    const double p = cH[r] + g[r] * cu;
    const double cb = cbar_H[r];
    acc[0] += h * h / D;
    acc[1] += h * p / D;
    acc[2] += p * p / D;
    acc[3] += h * cb / D;
    acc[4] += p * cb / D;
    gch += g[r] * cH[r];
  }
  double tot[6];
  {
    double v[6] = {acc[0], acc[1], acc[2], acc[3], acc[4], gch};
    __shared__ double lds6[6 * (NTA / 64)];
    for (int k = 0; k < 6; ++k) {
      const double w = wave_sum(v[k]);
      if ((threadIdx.x & 63) == 0) lds6[k * (NTA / 64) + (threadIdx.x >> 6)] = w;
    }
    __syncthreads();
    for (int k = 0; k < 6; ++k) {
      double s = 0.0;
      for (int w = 0; w < NTA / 64; ++w) s += lds6[k * (NTA / 64) + w];
      tot[k] = s;
    }
  }
  (void)red;
  const double d = alpha - mu * beta;
  const double pi = tot[5] + beta * cu;
  const double cbu = cbar_u[0];
  if (threadIdx.x == 0) {
    // [d - h'D^-1 h, pi - h'D^-1 p; pi - p'D^-1 h, -p'D^-1 p] [y_u; nu] = [cbu - h'D^-1 cb; -p'D^-1 cb]
    const double a11 = d - tot[0], a12 = pi - tot[1], a21 = pi - tot[1], a22 = -tot[2];
    const double b1 = cbu - tot[3], b2 = -tot[4];
    const double det = a11 * a22 - a12 * a21;
    sol[0] = (b1 * a22 - a12 * b2) / det;
    sol[1] = (a11 * b2 - a21 * b1) / det;
  }
  __syncthreads();
  const double yu = sol[0], nu = sol[1];
  for (int r = threadIdx.x; r < nH; r += NTA) {
    const double D = P.Lam[r] - mu;
    const double h = f[r] - mu * g[r];
    const double p = cH[r] + g[r] * cu;
    y[r] = (cbar_H[r] - h * yu - p * nu) / D;
  }
  if (threadIdx.x == 0) {
    const double lb = lam_bar[0];
    coef[0] = 2.0 * lb * cu - yu;
    coef[1] = -cu;
    coef[2] = -nu * cu;
    coef[3] = cu;
    coef[4] = yu;
    coef[5] = nu;
  }
}

// s = (coarse function ygrid interpolated) + y_u u~ on level m
__global__ __launch_bounds__(NTA) void k_adj_shat(const ProbDev* probs, int m, const double* ygrid,
                                                  const double* coef, const double* ut, double* s) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1;
  const int64_t idx = (int64_t)blockIdx.x * NTA + threadIdx.x;
  if (idx >= (int64_t)n1 * n1) return;
  const int gy = grid_row(idx, n1), gx = (int)(idx - (int64_t)gy * n1);
  double v = 0.0;
  if (is_dof(P.domain, N, gx, gy)) v = interp_coarse(ygrid, P.n_c, m, gx, gy) + coef[4] * ut[idx];
  s[idx] = v;
}

// u~_bar = c0 (K u - mu M u) + c1 (K s - mu M s) + c2 M u + c3 u_bar
template <int KIND>
__global__ __launch_bounds__(NTA) void k_adj_utbar(const ProbDev* probs, int m, const double* u,
                                                   const double* s, const double* ubar_m,
                                                   const double* coef, const double* rr,
                                                   double* out) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1;
  const int64_t idx = (int64_t)blockIdx.x * NTA + threadIdx.x;
  if (idx >= (int64_t)n1 * n1) return;
  const int gy = grid_row(idx, n1), gx = (int)(idx - (int64_t)gy * n1);
  double v = 0.0;
  if (is_dof(P.domain, N, gx, gy)) {
    const double mu = rr[3 * P.nH + 3];
    double Ku, Mu, Ks, Ms;
    K_and_M<KIND>(P, m, N, u, idx, gx, gy, Ku, Mu);
    K_and_M<KIND>(P, m, N, s, idx, gx, gy, Ks, Ms);
    v = coef[0] * (Ku - mu * Mu) + coef[1] * (Ks - mu * Ms) + coef[2] * Mu + coef[3] * ubar_m[idx];
  }
  out[idx] = v;
}

// Right-hand side of the adjoint local solve of each item: chi_j u~_bar on its tile,
// written into the item's residual buffer (the local solver then starts from it).
__global__ __launch_bounds__(NTA) void k_adj_tile_rhs(const ProbDev* probs, const TileItem* items,
                                                      const int32_t* sub_item, char* store, int m,
                                                      const double* utbar) {
  const ProbDev& P = probs[0];
  const TileItem it = items[blockIdx.y];
  const int r = 1 << m;
  const int nx = it.cw * r - 1, ny = it.ch * r - 1;
  const int64_t S = (int64_t)nx * ny;
  const int N = P.n_c << m, n1 = N + 1;
  double* R = reinterpret_cast<double*>(store + it.off) + S;
  const int sxb = it.sub % P.sub_x, syb = it.sub / P.sub_x;
  for (int64_t i = (int64_t)blockIdx.x * NTA + threadIdx.x; i < S; i += (int64_t)gridDim.x * NTA) {
    const int iy = (int)(i / nx), ix = (int)(i - (int64_t)iy * nx);
    const int gx = it.cx0 * r + 1 + ix, gy = it.cy0 * r + 1 + iy;
    double v = 0.0;
    if (is_dof(P.domain, N, gx, gy)) {
      int cx[MLC_MAX_CAND], cy[MLC_MAX_CAND];
      double rx[MLC_MAX_CAND], ry[MLC_MAX_CAND];
      const int nxc = pou_axis(P.n_c, P.sub_x, gx, r, P.overlap, P.pou, cx, rx);
      const int nyc = pou_axis(P.n_c, P.sub_y, gy, r, P.overlap, P.pou, cy, ry);
      double tot = 0.0, mine = 0.0;
      for (int a = 0; a < nyc; ++a)
        for (int b = 0; b < nxc; ++b) {
          if (sub_item[P.sub_item_off + (cy[a] * P.sub_x + cx[b]) * P.q] < 0) continue;
          const double phi = rx[b] * ry[a];
          tot += phi;
          if (cx[b] == sxb && cy[a] == syb) mine = phi;
        }
      v = tot > 0.0 ? mine / tot * utbar[(int64_t)gy * n1 + gx] : 0.0;
    }
    R[i] = v;
  }
}

// r_bar = sum over the tiles covering a node of the adjoint local solutions z_j
__global__ __launch_bounds__(NTA) void k_adj_rbar(const ProbDev* probs, const TileItem* items,
                                                  const int32_t* sub_item, const char* store, int m,
                                                  double* rbar) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1;
  const int64_t idx = (int64_t)blockIdx.x * NTA + threadIdx.x;
  if (idx >= (int64_t)n1 * n1) return;
  const int gy = grid_row(idx, n1), gx = (int)(idx - (int64_t)gy * n1);
  double v = 0.0;
  if (is_dof(P.domain, N, gx, gy)) {
    const int r = 1 << m;
    int cx[MLC_MAX_CAND], cy[MLC_MAX_CAND];
    double rx[MLC_MAX_CAND], ry[MLC_MAX_CAND];
    const int nxc = pou_axis(P.n_c, P.sub_x, gx, r, P.overlap, P.pou, cx, rx);
    const int nyc = pou_axis(P.n_c, P.sub_y, gy, r, P.overlap, P.pou, cy, ry);
    for (int a = 0; a < nyc; ++a)
      for (int b = 0; b < nxc; ++b) {
        const int item = sub_item[P.sub_item_off + (cy[a] * P.sub_x + cx[b]) * P.q];
        if (item < 0) continue;
        const TileItem& it = items[item];
        const int nx = it.cw * r - 1;
        const double* z = reinterpret_cast<const double*>(store + it.off);
        v += z[(int64_t)(gy - (it.cy0 * r + 1)) * nx + (gx - (it.cx0 * r + 1))];
      }
  }
  rbar[idx] = v;
}

// ubar_i = (P u_k)(node); next = u~_bar + lambda_k M r_bar - K r_bar (level m)
template <int KIND>
__global__ __launch_bounds__(NTA) void k_adj_next(const ProbDev* probs, int m, const double* uk,
                                                  const double* lam_k, const double* utbar,
                                                  const double* rbar, double* ubar, double* next) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1;
  const int64_t idx = (int64_t)blockIdx.x * NTA + threadIdx.x;
  if (idx >= (int64_t)n1 * n1) return;
  const int gy = grid_row(idx, n1), gx = (int)(idx - (int64_t)gy * n1);
  double ub = 0.0, nx = 0.0;
  if (is_dof(P.domain, N, gx, gy)) {
    ub = interp2(uk, (N >> 1) + 1, gx, gy);
    double Kr, Mr;
    K_and_M<KIND>(P, m, N, rbar, idx, gx, gy, Kr, Mr);
    nx = utbar[idx] + lam_k[0] * Mr - Kr;
  }
  ubar[idx] = ub;
  next[idx] = nx;
}

__device__ __forceinline__ void tri_prods(double a_sw, double a_se, double a_ne, double a_nw,
                                          double b_sw, double b_se, double b_ne, double b_nw,
                                          double& lo, double& up) {
  lo = 0.5 * ((a_sw - a_se) * (b_sw - b_se) + (a_se - a_ne) * (b_se - b_ne));
  up = 0.5 * ((a_sw - a_nw) * (b_sw - b_nw) + (a_nw - a_ne) * (b_nw - b_ne));
}

// kappa_bar of every triangle of level m:
//   c_uu * (u, u) - (s, u) - (r_bar, ubar) - sum_j (z_j, e_j)
// (s, r_bar, ubar, tiles optional: null pointers skip them).
__global__ __launch_bounds__(NTA) void k_adj_products(const ProbDev* probs, int m, const double* u,
                                                      const double* c_uu, const double* s,
                                                      const double* rbar, const double* ubar,
                                                      const TileItem* items, const int32_t* sub_item,
                                                      const char* store, const double* te,
                                                      const int64_t* te_off, double* klo,
                                                      double* kup) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1;
  const int64_t idx = (int64_t)blockIdx.x * NTA + threadIdx.x;
  if (idx >= (int64_t)N * N) return;
  const int J = grid_row(idx, N), I = (int)(idx - (int64_t)J * N);
  const int64_t sw = (int64_t)J * n1 + I, se = sw + 1, nw = sw + n1, ne = nw + 1;
  double lo, up, l2, u2;
  tri_prods(u[sw], u[se], u[ne], u[nw], u[sw], u[se], u[ne], u[nw], lo, up);
  const double cu = c_uu[0];
  double alo = cu * lo, aup = cu * up;
  if (s) {
    tri_prods(s[sw], s[se], s[ne], s[nw], u[sw], u[se], u[ne], u[nw], l2, u2);
    alo -= l2;
    aup -= u2;
  }
  if (rbar) {
    tri_prods(rbar[sw], rbar[se], rbar[ne], rbar[nw], ubar[sw], ubar[se], ubar[ne], ubar[nw], l2, u2);
    alo -= l2;
    aup -= u2;
  }
  if (items) {
    const int r = 1 << m;
    const int d = P.overlap * r;
    for (int by = 0; by < P.sub_y; ++by) {
      const int y0 = max(0, P.by[by] * r - d), y1 = min(N, P.by[by + 1] * r + d);
      if (J < y0 || J + 1 > y1) continue;
      for (int bx = 0; bx < P.sub_x; ++bx) {
        const int x0 = max(0, P.bx[bx] * r - d), x1 = min(N, P.bx[bx + 1] * r + d);
        if (I < x0 || I + 1 > x1) continue;
        const int item = sub_item[P.sub_item_off + (by * P.sub_x + bx) * P.q];
        if (item < 0) continue;
        const TileItem& it = items[item];
        const int nx = it.cw * r - 1, ny = it.ch * r - 1;
        const double* z = reinterpret_cast<const double*>(store + it.off);
        const double* e = te + te_off[item];
        const int lx = I - it.cx0 * r - 1, ly = J - it.cy0 * r - 1;  // tile index of sw
        auto at = [&](const double* v, int x, int y) -> double {
          return (x >= 0 && y >= 0 && x < nx && y < ny) ? v[(int64_t)y * nx + x] : 0.0;
        };
        tri_prods(at(z, lx, ly), at(z, lx + 1, ly), at(z, lx + 1, ly + 1), at(z, lx, ly + 1),
                  at(e, lx, ly), at(e, lx + 1, ly), at(e, lx + 1, ly + 1), at(e, lx, ly + 1), l2, u2);
        alo -= l2;
        aup -= u2;
      }
    }
  }
  klo[idx] += alo;
  kup[idx] += aup;
}

// Level 0: a_i = (v_i^T u_bar_0) / (Lambda_i - Lambda_0) for i >= 1, a_0 = 0.
__global__ __launch_bounds__(NTA) void k_adj_level0(const ProbDev* probs, const double* ubar0,
                                                    double* a) {
  const ProbDev& P = probs[0];
  const int c = blockIdx.x * (NTA / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= P.nH) return;
  const double* col = P.V + (int64_t)c * P.nH;
  double s = 0.0;
  for (int r = lane; r < P.nH; r += 64) s += col[r] * ubar0[P.coarse_nodes[r]];
  s = wave_sum(s);
  if (lane == 0) a[c] = (c == 0) ? 0.0 : s / (P.Lam[c] - P.Lam[0]);
}

// kappa_bar on level l gets 1/4 of its parent's (level l-1) adjoint (children means).
__global__ __launch_bounds__(NTA) void k_adj_down(const double* plo, const double* pup, double* clo,
                                                  double* cup, int Nc) {
  const int Nf = 2 * Nc;
  const int64_t idx = (int64_t)blockIdx.x * NTA + threadIdx.x;
  if (idx >= (int64_t)Nf * Nf) return;
  const int j = grid_row(idx, Nf), i = (int)(idx - (int64_t)j * Nf);
  const int64_t p = (int64_t)(j >> 1) * Nc + (i >> 1);
  const bool xi = i & 1, yj = j & 1;
  // parents: lower(I,J) <- lower(2I,2J), lower(2I+1,2J), upper(2I+1,2J), lower(2I+1,2J+1)
  //          upper(I,J) <- upper(2I,2J), upper(2I,2J+1), lower(2I,2J+1), upper(2I+1,2J+1)
  const double lo_parent = (!xi && !yj) || xi ? plo[p] : pup[p];
  const double up_parent = (xi && !yj) ? plo[p] : pup[p];
  clo[idx] += 0.25 * lo_parent;
  cup[idx] += 0.25 * up_parent;
}

// Output: kind 2 per finest cell (both triangles); kind 1 per coarse cell (sum of its cells).
__global__ __launch_bounds__(NTA) void k_adj_out(const double* lo, const double* up, int N, int kind,
                                                 int nc, double* out) {
  const int64_t idx = (int64_t)blockIdx.x * NTA + threadIdx.x;
  if (kind == 2) {
    if (idx < (int64_t)N * N) out[idx] = lo[idx] + up[idx];
    return;
  }
  if (idx >= (int64_t)nc * nc) return;
  const int J = grid_row(idx, nc), I = (int)(idx - (int64_t)J * nc);
  const int r = N / nc;
  double s = 0.0;
  for (int y = J * r; y < (J + 1) * r; ++y)
    for (int x = I * r; x < (I + 1) * r; ++x) s += lo[(int64_t)y * N + x] + up[(int64_t)y * N + x];
  out[idx] = s;
}

}  // namespace

#define MLC_CHK()                                   \
  do {                                              \
    hipError_t e_ = hipGetLastError();              \
    if (e_ != hipSuccess) return e_;                \
  } while (0)

hipError_t launch_tape_tiles(const TileItem* items, int nitems, const char* store, int m, double* te,
                             const int64_t* te_off, hipStream_t s) {
  hipLaunchKernelGGL(k_tape_tiles, dim3(nitems), dim3(NTA), 0, s, items, store, m, te, te_off);
  return hipGetLastError();
}

hipError_t launch_restrict1(const ProbDev* p, const double* in, double* out, int l, int64_t nodes_l,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_restrict1, dim3(nb(nodes_l)), dim3(NTA), 0, s, p, in, out, l);
  return hipGetLastError();
}

hipError_t launch_coarse_project(const ProbDev* p, int nH, const double* a, double* out,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_project, dim3((nH + 3) / 4), dim3(NTA), 0, s, p, a, out);
  return hipGetLastError();
}

hipError_t launch_coarse_combine(const ProbDev* p, int nc1sq, const double* y, double* grid,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_combine, dim3((nc1sq + 3) / 4), dim3(NTA), 0, s, p, y, grid);
  return hipGetLastError();
}

hipError_t launch_dot_sum(const ProbDev* p, int m, int64_t nodes, const double* a, const double* b,
                          bool mass, double* parts, double* out, hipStream_t s) {
  const unsigned g = nb(nodes);
  if (mass)
    hipLaunchKernelGGL(k_dot<true>, dim3(g), dim3(NTA), 0, s, p, m, a, b, parts);
  else
    hipLaunchKernelGGL(k_dot<false>, dim3(g), dim3(NTA), 0, s, p, m, a, b, parts);
  MLC_CHK();
  hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(NTA), 0, s, parts, (int)g, out);
  return hipGetLastError();
}

hipError_t launch_adj_rr(const ProbDev* p, const double* rr, const double* cbar_H,
                         const double* cbar_u, const double* lam_bar, double* y, double* coef,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_adj_rr, dim3(1), dim3(NTA), 0, s, p, rr, cbar_H, cbar_u, lam_bar, y, coef);
  return hipGetLastError();
}

hipError_t launch_adj_shat(const ProbDev* p, int m, int64_t nodes, const double* ygrid,
                           const double* coef, const double* ut, double* shat, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_shat, dim3(nb(nodes)), dim3(NTA), 0, s, p, m, ygrid, coef, ut, shat);
  return hipGetLastError();
}

hipError_t launch_adj_utbar(int kind, const ProbDev* p, int m, int64_t nodes, const double* u,
                            const double* shat, const double* ubar_m, const double* coef,
                            const double* rr, double* out, hipStream_t s) {
  if (kind == 1)
    hipLaunchKernelGGL(k_adj_utbar<1>, dim3(nb(nodes)), dim3(NTA), 0, s, p, m, u, shat, ubar_m,
                       coef, rr, out);
  else
    hipLaunchKernelGGL(k_adj_utbar<2>, dim3(nb(nodes)), dim3(NTA), 0, s, p, m, u, shat, ubar_m,
                       coef, rr, out);
  return hipGetLastError();
}

hipError_t launch_adj_tile_rhs(const ProbDev* p, const TileItem* items, int nitems,
                               const int32_t* sub_item, char* store, int m, const double* utbar,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_adj_tile_rhs, dim3(32, nitems), dim3(NTA), 0, s, p, items, sub_item, store,
                     m, utbar);
  return hipGetLastError();
}

hipError_t launch_adj_rbar(const ProbDev* p, const TileItem* items, const int32_t* sub_item,
                           const char* store, int m, int64_t nodes, double* rbar, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_rbar, dim3(nb(nodes)), dim3(NTA), 0, s, p, items, sub_item, store, m,
                     rbar);
  return hipGetLastError();
}

hipError_t launch_adj_next(int kind, const ProbDev* p, int m, int64_t nodes, const double* uk,
                           const double* lam_k, const double* utbar, const double* rbar,
                           double* ubar, double* next, hipStream_t s) {
  if (kind == 1)
    hipLaunchKernelGGL(k_adj_next<1>, dim3(nb(nodes)), dim3(NTA), 0, s, p, m, uk, lam_k, utbar,
                       rbar, ubar, next);
  else
    hipLaunchKernelGGL(k_adj_next<2>, dim3(nb(nodes)), dim3(NTA), 0, s, p, m, uk, lam_k, utbar,
                       rbar, ubar, next);
  return hipGetLastError();
}

hipError_t launch_adj_products(const ProbDev* p, int m, int64_t cells, const double* u,
                               const double* c_uu, const double* shat, const double* rbar,
                               const double* ubar, const TileItem* items, const int32_t* sub_item,
                               const char* store, const double* te, const int64_t* te_off,
                               double* klo, double* kup, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_products, dim3(nb(cells)), dim3(NTA), 0, s, p, m, u, c_uu, shat, rbar,
                     ubar, items, sub_item, store, te, te_off, klo, kup);
  return hipGetLastError();
}

hipError_t launch_adj_level0(const ProbDev* p, int nH, const double* ubar0, double* a,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_adj_level0, dim3((nH + 3) / 4), dim3(NTA), 0, s, p, ubar0, a);
  return hipGetLastError();
}

hipError_t launch_adj_down(const double* plo, const double* pup, double* clo, double* cup, int Nc,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_adj_down, dim3(nb((int64_t)4 * Nc * Nc)), dim3(NTA), 0, s, plo, pup, clo,
                     cup, Nc);
  return hipGetLastError();
}

hipError_t launch_adj_out(const double* lo, const double* up, int N, int kind, int nc, double* out,
                          hipStream_t s) {
  const int64_t n = kind == 2 ? (int64_t)N * N : (int64_t)nc * nc;
  hipLaunchKernelGGL(k_adj_out, dim3(nb(n)), dim3(NTA), 0, s, lo, up, N, kind, nc, out);
  return hipGetLastError();
}
