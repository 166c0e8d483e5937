// Global-grid kernels of one correction step (Algorithm 4.1) and of the coarse setup
// (Algorithm 4.2 step 1).  One thread per node of a level grid; blockIdx.y selects the
// problem of a batch.  All are plain streaming sweeps bound by HBM bandwidth.
#include "mlc_launch.h"

namespace {

constexpr int NTG = 256;

__device__ __forceinline__ double interp2(const double* uc, int nc1, int x, int y) {
  // P1 nodal interpolation from the grid one level coarser (SW-NE diagonals):
  // coinciding nodes copy, edge midpoints average the two ends of their edge (E, N or NE
  // of the first).  Branch-free: a coinciding node averages its value with itself, which
  // is exact, so neighbouring lanes of either parity issue their loads together.
  const int ix = x >> 1, iy = y >> 1;
  const double a = uc[iy * nc1 + ix];
  const double b = uc[(iy + (y & 1)) * nc1 + ix + (x & 1)];
  return 0.5 * (a + b);
}

// Algorithm 4.1, step 1: u_bar = I u_k on level m and the right-hand side of (Aux_Problem),
// r = lambda_k M u_bar - K u_bar, for eigenpair i = blockIdx.z (one grid slice per
// eigenpair, so the loads of all of them are in flight together).
template <int KIND>
__global__ __launch_bounds__(NTG) void k_prolong_residual(const ProbDev* probs, int m, int src) {
  // the step's convergence record starts empty (the local solves follow on the stream)
  if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0)
    probs[0].conv[m] = 0.0;
  const ProbDev& P = probs[blockIdx.y];
  if (m > P.L) return;
  const int i = blockIdx.z;
  if (i >= P.q) return;
  const int N = P.n_c << m;
  const int n1 = N + 1;
  const int64_t nn = (int64_t)n1 * n1;
  const int64_t idx = (int64_t)blockIdx.x * NTG + threadIdx.x;
  if (idx >= nn) return;
  const int gy = grid_row(idx, n1), gx = (int)(idx - (int64_t)gy * n1);
  const int nc1 = (N >> 1) + 1;
  const bool dof = is_dof(P.domain, N, gx, gy);
  const double h = P.side / N;
  const double mh = h * h * (1.0 / 12.0);
  Weights W;
  MassW Mw;
  if (dof) {
    W = edge_weights<KIND>(P, m, N, gx, gy);
    Mw = mass_weights<KIND>(P, m, N, gx, gy, mh);
  }
  double* ub = P.ubar + (int64_t)i * nn;
  double* r = P.res + (int64_t)i * nn;
  if (!dof) {
    ub[idx] = 0.0;
    r[idx] = 0.0;
    return;
  }
  const double* uc = P.u[src] + (int64_t)i * nc1 * nc1;
  const double c = interp2(uc, nc1, gx, gy);
  const double e = interp2(uc, nc1, gx + 1, gy), w = interp2(uc, nc1, gx - 1, gy);
  const double n = interp2(uc, nc1, gx, gy + 1), s = interp2(uc, nc1, gx, gy - 1);
  const double ne = interp2(uc, nc1, gx + 1, gy + 1), sw = interp2(uc, nc1, gx - 1, gy - 1);
  double d;
  const double Ku = apply_k<KIND, double>(W, c, e, w, n, s, ne, sw, d);
  const double Mu = apply_mass<KIND>(Mw, mh, c, e, w, n, s, ne, sw);
  const double lam = P.lam[src * MLC_MAX_Q + i];
  ub[idx] = c;
  r[idx] = lam * Mu - Ku;
}

// floor(a / b) for 0 <= a < 2^22 and b >= 1 from a float reciprocal of b: the estimate is
// within one of the quotient (relative error below 2^-22), and one step each way makes it
// exact.  Integer division costs tens of instructions on the vector unit.
__device__ __forceinline__ int div_small(int a, int b, float rb) {
  int q = (int)((float)a * rb);
  q -= (q * b > a) ? 1 : 0;
  q += ((q + 1) * b <= a) ? 1 : 0;
  return q;
}

// pou_axis with r = 2^m and the block divisions by reciprocals (nc * nb < 2^22, checked by
// the caller): the same candidates, factors and order.
__device__ __forceinline__ int pou_axis_fast(int nc, int nb, int g, int m, int ov, int pou,
                                             int (&id)[MLC_MAX_CAND], double (&rho)[MLC_MAX_CAND]) {
  const int r = 1 << m, d = ov * r;
  const float rnb = 1.0f / (float)nb, rnc = 1.0f / (float)nc;
  const int b0 = div_small((min(g >> m, nc - 1) + 1) * nb - 1, nc, rnc);
  const int blo = max(0, b0 - ov - 1), bhi = min(nb - 1, b0 + ov + 1);
  int n = 0;
  int lo = div_small(blo * nc, nb, rnb) * r;
  for (int b = blo; b <= bhi && n < MLC_MAX_CAND; ++b) {
    const int hi = div_small((b + 1) * nc, nb, rnb) * r;
    const int v = min(g - lo + d, hi + d - g);
    if (v > 0) {
      id[n] = b;
      rho[n] = pou == 0 ? (double)min(v, d) / (double)d : (g >= lo && g <= hi ? 1.0 : 0.0);
      ++n;
    }
    lo = hi;
  }
  return n;
}

// pou_axis_fast for nodes with at most two covering blocks, without the candidate arrays
// (their run-time indices cost a conditional move per slot and candidate).  A block's
// Omega range holds g strictly inside when lo - d < g < hi + d, and lo, hi grow with the
// block, so the covering blocks run from the block holding fine position g - d to the one
// holding g + d - 1 (coarse cells (g >> m) - ov and ((g - 1) >> m) + ov, clamped; g is an
// interior node).  Returns their number (0 on a block boundary without overlap) and the
// first in *b0; rho[0..1] receive the factors of the first two, the values pou_axis_fast
// gives (with an overlap of a power of two coarse cells the division by d is a scaling by a
// power of two, which is exact, so it is done as one).
__device__ __forceinline__ int pou_axis2(int nc, int nb, int g, int m, int ov, int pou, int* b0,
                                         double (&rho)[2]) {
  const int r = 1 << m, d = ov * r;
  const float rnb = 1.0f / (float)nb, rnc = 1.0f / (float)nc;
  const int c1 = max(0, (g >> m) - ov), c2 = min(nc - 1, ((g - 1) >> m) + ov);
  const int bf = div_small((c1 + 1) * nb - 1, nc, rnc);
  const int bl = div_small((c2 + 1) * nb - 1, nc, rnc);
  const int n = max(0, bl - bf + 1);
  *b0 = bf;
  const int l0 = div_small(bf * nc, nb, rnb) * r;
  const int l1 = div_small(min(bf + 1, nb) * nc, nb, rnb) * r;
  const int l2 = div_small(min(bf + 2, nb) * nc, nb, rnb) * r;
  const int sh = pou == 0 ? m + __builtin_ctz((unsigned)max(ov, 1)) : 0;
  const bool pow2 = (ov & (ov - 1)) == 0;
  auto factor = [&](int lo, int hi) -> double {
    if (pou != 0) return (g >= lo && g <= hi) ? 1.0 : 0.0;
    const double v = (double)min(min(g - lo + d, hi + d - g), d);
    return pow2 ? ldexp(v, -sh) : v / (double)d;
  };
  rho[0] = n > 0 ? factor(l0, l1) : 0.0;
  rho[1] = n > 1 ? factor(l1, l2) : 0.0;
  return n;
}

// Algorithm 4.1, step 2 in its partition-of-unity form: the gluing
//   u~ = u_bar + sum_j chi_j e^j,  chi_j = phi_j / sum_l phi_l.
// QM: a bound on q (1, 2, 4 or 8) that sizes the per-eigenpair registers.
template <int QM>
__global__ __launch_bounds__(NTG) void k_pou_glue(const ProbDev* probs, const TileItem* items,
                                                   const int32_t* sub_item, const char* store,
                                                   int m) {
  // m: level of the node grid (the mesh level for P1, one more for P2)
  const ProbDev& P = probs[blockIdx.y];
  if (m > P.Lg) return;
  const int N = P.n_c << m;
  const int n1 = N + 1;
  const int64_t nn = (int64_t)n1 * n1;
  const int64_t idx = (int64_t)blockIdx.x * NTG + threadIdx.x;
  if (idx >= nn) return;
  const int gy = grid_row(idx, n1), gx = (int)(idx - (int64_t)gy * n1);
  if (!is_dof(P.domain, N, gx, gy)) {
    for (int i = 0; i < P.q; ++i) P.ut[(int64_t)i * nn + idx] = 0.0;
    return;
  }
  const int r = 1 << m;
  const bool fast = P.n_c * max(P.sub_x, P.sub_y) < (1 << 22);
  // one item lookup per covering subdomain: its q right-hand sides follow at rhs_stride
  double acc[QM], tot = 0.0;
#pragma unroll
  for (int i = 0; i < QM; ++i) acc[i] = 0.0;
  int bx0 = 0, by0 = 0;
  double rx[2], ry[2];
  const int sx = fast ? pou_axis2(P.n_c, P.sub_x, gx, m, P.overlap, P.pou, &bx0, rx) : 3;
  const int sy = fast ? pou_axis2(P.n_c, P.sub_y, gy, m, P.overlap, P.pou, &by0, ry) : 3;
  if (sx <= 2 && sy <= 2) {
    const int nxc = sx, nyc = sy;
    const int ix[2] = {bx0, bx0 + 1}, iy[2] = {by0, by0 + 1};
    // at most 2 x 2 covering subdomains (overlap 1 on blocks of two or more coarse cells):
    // every index load first, then every item, then every tile value, so the three
    // dependent loads of the subdomains overlap instead of following one another.  Slots
    // past the candidates, or without an item, load from the first subdomain that has one
    // (in bounds, as it covers the node) and add nothing; the sums keep the loop's order.
    int itm[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int a = c >> 1, b = c & 1;
      const int sub = (a < nyc && b < nxc) ? iy[a] * P.sub_x + ix[b] : -1;
      const int raw = sub_item[P.sub_item_off + (sub >= 0 ? sub : 0) * P.q];  // sub 0: in bounds
      itm[c] = sub >= 0 ? raw : -1;
    }
    int first = -1;
#pragma unroll
    for (int c = 3; c >= 0; --c)
      if (itm[c] >= 0) first = c;
    if (first >= 0) {
      const int safe = itm[first];
      const char* e0[4];
      int rs[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const TileItem it = items[itm[c] >= 0 ? itm[c] : safe];
        const int nx = it.cw * r - 1;
        const int lx = gx - (it.cx0 * r + 1), ly = gy - (it.cy0 * r + 1);
        e0[c] = store + it.off + ((int64_t)ly * nx + lx) * (int64_t)sizeof(double);
        rs[c] = it.rhs_stride;
      }
      double v[4][QM];
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int i = 0; i < QM; ++i)
          v[c][i] = i < P.q ? *reinterpret_cast<const double*>(e0[c] + (int64_t)i * rs[c]) : 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (itm[c] < 0) continue;
        const double phi = rx[c & 1] * ry[c >> 1];
#pragma unroll
        for (int i = 0; i < QM; ++i)
          if (i < P.q) acc[i] += phi * v[c][i];
        tot += phi;
      }
    }
  } else {
    // more covering subdomains (wider overlaps, narrow blocks) or the general division
    int ix[MLC_MAX_CAND], iy[MLC_MAX_CAND];
    double rx[MLC_MAX_CAND], ry[MLC_MAX_CAND];
    const int nxc = fast ? pou_axis_fast(P.n_c, P.sub_x, gx, m, P.overlap, P.pou, ix, rx)
                         : pou_axis(P.n_c, P.sub_x, gx, r, P.overlap, P.pou, ix, rx);
    const int nyc = fast ? pou_axis_fast(P.n_c, P.sub_y, gy, m, P.overlap, P.pou, iy, ry)
                         : pou_axis(P.n_c, P.sub_y, gy, r, P.overlap, P.pou, iy, ry);
    for (int a = 0; a < nyc; ++a) {
      for (int b = 0; b < nxc; ++b) {
        const int item = sub_item[P.sub_item_off + (iy[a] * P.sub_x + ix[b]) * P.q];
        if (item < 0) continue;
        const TileItem it = items[item];
        const int nx = it.cw * r - 1;
        const int lx = gx - (it.cx0 * r + 1), ly = gy - (it.cy0 * r + 1);
        const char* e0 = store + it.off + ((int64_t)ly * nx + lx) * (int64_t)sizeof(double);
        const double phi = rx[b] * ry[a];
#pragma unroll
        for (int i = 0; i < QM; ++i)
          if (i < P.q)
            acc[i] += phi * *reinterpret_cast<const double*>(e0 + (int64_t)i * it.rhs_stride);
        tot += phi;
      }
    }
  }
  // tot = 0 only on D_j block boundaries with overlap 0, where every e^j vanishes
#pragma unroll
  for (int i = 0; i < QM; ++i)
    if (i < P.q)
      P.ut[(int64_t)i * nn + idx] = P.ubar[(int64_t)i * nn + idx] + (tot > 0.0 ? acc[i] / tot : 0.0);
}

// Algorithm 4.1, step 3 (the border of (Eigen_Augment_Problem)): y_K = K u~ (into res),
// y_M = M u~ (into ubar), and per-block partial sums of alpha_ij = u~_i . y_K,j,
// beta_ij = u~_i . y_M,j and s_i = sum u~_i.
constexpr int RNV = 2 * MLC_MAX_Q * MLC_MAX_Q + MLC_MAX_Q;

// QM: a bound on q (1, 2, 4 or 8) that sizes the per-eigenpair registers.
template <int KIND, int QM>
__global__ __launch_bounds__(NTG) void k_rr_apply(const ProbDev* probs, int m) {
  __shared__ double red[(NTG / 64) * RNV];
  const ProbDev& P = probs[blockIdx.y];
  if (m > P.L) return;
  const int N = P.n_c << m;
  const int n1 = N + 1;
  const int64_t nn = (int64_t)n1 * n1;
  const int64_t nblk = (nn + NTG - 1) / NTG;
  if ((int64_t)blockIdx.x >= nblk) return;
  const int64_t idx = (int64_t)blockIdx.x * NTG + threadIdx.x;
  const int q = P.q;
  const bool inr = idx < nn;
  int gx = 0, gy = 0;
  if (inr) {
    gy = grid_row(idx, n1);
    gx = (int)(idx - (int64_t)gy * n1);
  }
  const bool dof = inr && is_dof(P.domain, N, gx, gy);
  const double h = P.side / N;
  const double mh = h * h * (1.0 / 12.0);
  Weights W;
  MassW Mw;
  if (dof) {
    W = edge_weights<KIND>(P, m, N, gx, gy);
    Mw = mass_weights<KIND>(P, m, N, gx, gy, mh);
  }
  double uv[QM], yk[QM], ym[QM];
  // every eigenpair's stencil values are loaded before the first store (a store between
  // them would keep the next loads from being issued early)
  double st[QM][7];
#pragma unroll
  for (int i = 0; i < QM; ++i)
    if (i < q && dof) {
      const double* u = P.ut + (int64_t)i * nn;
      st[i][0] = u[idx];
      st[i][1] = u[idx + 1];
      st[i][2] = u[idx - 1];
      st[i][3] = u[idx + n1];
      st[i][4] = u[idx - n1];
      st[i][5] = u[idx + n1 + 1];
      st[i][6] = u[idx - n1 - 1];
    }
#pragma unroll
  for (int i = 0; i < QM; ++i) {
    uv[i] = yk[i] = ym[i] = 0.0;
    if (i < q && dof) {
      const double c = st[i][0], e = st[i][1], w = st[i][2], n = st[i][3], s = st[i][4];
      const double ne = st[i][5], sw = st[i][6];
      uv[i] = c;
      double d;
      yk[i] = apply_k<KIND, double>(W, c, e, w, n, s, ne, sw, d);
      ym[i] = apply_mass<KIND>(Mw, mh, c, e, w, n, s, ne, sw);
    }
    if (i < q && inr) {
      P.res[(int64_t)i * nn + idx] = yk[i];
      P.ubar[(int64_t)i * nn + idx] = ym[i];
    }
  }
  // partial sums: every wave reduces each value across its lanes, one barrier, then the
  // waves' values are added in a fixed order
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
        red[wid * RNV + i * q + j] = a;
        red[wid * RNV + q * q + i * q + j] = c;
      }
    }
    const double s = wave_sum(uv[i]);
    if (lane == 0) red[wid * RNV + 2 * q * q + i] = s;
  }
  __syncthreads();
  for (int v = threadIdx.x; v < nv; v += NTG) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NTG / 64; ++w) s += red[w * RNV + v];
    out[v] = s;
  }
}

// Algorithm 4.1, step 3 (continued): one level of the transposed interpolation P^T (full
// weighting on the SW-NE mesh: centre 1, E/W/N/S/NE/SW 1/2) for the 2q border vectors,
// level l+1 -> l; blockIdx.z selects the vector, so the loads of all vectors are in flight
// together.
__global__ __launch_bounds__(NTG) void k_restrict(const ProbDev* probs, int l, int m) {
  const ProbDev& P = probs[blockIdx.y];
  if (m > P.L) return;
  const int q = P.q;
  const int v = blockIdx.z;
  if (v >= 2 * q) return;
  const int Nc = P.n_c << l;
  const int nc1 = Nc + 1;
  const int64_t nnc = (int64_t)nc1 * nc1;
  const int64_t idx = (int64_t)blockIdx.x * NTG + threadIdx.x;
  if (idx >= nnc) return;
  const int Iy = grid_row(idx, nc1), Ix = (int)(idx - (int64_t)Iy * nc1);
  const int nf1 = 2 * Nc + 1;
  const int64_t nnf = (int64_t)nf1 * nf1;
  const bool dof = is_dof(P.domain, Nc, Ix, Iy);
  double* outb = P.rchain + P.rchain_off[l];
  const double* f;
  if (l + 1 == m) {
    f = (v < q ? P.res + (int64_t)v * nnf : P.ubar + (int64_t)(v - q) * nnf);
  } else {
    f = P.rchain + P.rchain_off[l + 1] + (int64_t)v * nnf;
  }
  double val = 0.0;
  if (dof) {
    const int64_t c = (int64_t)(2 * Iy) * nf1 + 2 * Ix;
    val = f[c] + 0.5 * (f[c + 1] + f[c - 1] + f[c + nf1] + f[c - nf1] + f[c + nf1 + 1] +
                        f[c - nf1 - 1]);
  }
  outb[(int64_t)v * nnc + idx] = val;
}

// Algorithm 4.1, step 3 (the small eigenproblem, first half): f = V^T a, g = V^T b for the
// coarse eigenbasis V, one wave per column and border vector.
__global__ __launch_bounds__(NTG) void k_rr_project(const ProbDev* probs) {
  const ProbDev& P = probs[blockIdx.y];
  const int c = blockIdx.x * (NTG / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= P.nH) return;
  const int nH = P.nH, q = P.q;
  const int nc1 = P.c1;
  const double* a = P.rchain + P.rchain_off[0];
  const double* col = P.V + (int64_t)c * nH;
  const int v = blockIdx.z;  // border vector (one grid slice each)
  if (v >= 2 * q) return;
  const double* src = a + (int64_t)v * nc1 * nc1;
  double s = 0.0;
  for (int r = lane; r < nH; r += 64) s += col[r] * src[P.coarse_nodes[r]];
  s = wave_sum(s);
  if (lane == 0) P.fg[(int64_t)v * nH + c] = s;
}

// Algorithm 4.1, step 3 (the new eigenfunction, first half): coarse nodal coefficients
// c_H = V y_hat on the coarse grid, one wave per coarse node and eigenpair sweeping a row
// of V^T.
__global__ __launch_bounds__(NTG) void k_rr_combine(const ProbDev* probs) {
  const ProbDev& P = probs[blockIdx.y];
  const int nc1 = P.c1;
  const int node = blockIdx.x * (NTG / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (node >= nc1 * nc1) return;
  const int r = P.coarse_index[node];
  const int nH = P.nH;
  const int k = blockIdx.z;  // eigenpair (one grid slice each)
  if (k >= P.q) return;
  double s = 0.0;
  if (r >= 0) {
    const double* y = P.rr_y + (int64_t)k * nH;
    const double* row = P.VT + (int64_t)r * nH;
    for (int c = lane; c < nH; c += 64) s += row[c] * y[c];
    s = wave_sum(s);
  }
  if (lane == 0) P.cH_grid[(int64_t)k * nc1 * nc1 + node] = s;
}

// Algorithm 4.1, step 3 (the new eigenfunction): u_{k+1} = P_{0->m} c_H + sum_i t_i u~_i on
// level m.
__global__ __launch_bounds__(NTG) void k_assemble(const ProbDev* probs, int m, int dst) {
  const ProbDev& P = probs[blockIdx.y];
  if (m > P.L) return;
  const int k = blockIdx.z;  // eigenpair (one grid slice each)
  if (k >= P.q) return;
  const int N = P.n_c << m;
  const int n1 = N + 1;
  const int64_t nn = (int64_t)n1 * n1;
  const int64_t idx = (int64_t)blockIdx.x * NTG + threadIdx.x;
  if (idx >= nn) return;
  const int gy = grid_row(idx, n1), gx = (int)(idx - (int64_t)gy * n1);
  const bool dof = is_dof(P.domain, N, gx, gy);
  const int q = P.q;
  const int nc = P.n_c, nc1 = nc + 1;
  const int I = min(gx >> m, nc - 1), J = min(gy >> m, nc - 1);
  const int a = gx - (I << m), b = gy - (J << m);
  const double inv_r = 1.0 / (double)(1 << m);
  double val = 0.0;
  if (dof) {
    const double* c = P.cH_grid + (int64_t)k * nc1 * nc1;
    const double c00 = c[J * nc1 + I], c10 = c[J * nc1 + I + 1];
    const double c01 = c[(J + 1) * nc1 + I], c11 = c[(J + 1) * nc1 + I + 1];
    if (a >= b)
      val = c00 + (a * (c10 - c00) + b * (c11 - c10)) * inv_r;
    else
      val = c00 + (b * (c01 - c00) + a * (c11 - c01)) * inv_r;
    for (int i = 0; i < q; ++i) val += P.rr_t[k * q + i] * P.ut[(int64_t)i * nn + idx];
  }
  P.u[dst][(int64_t)k * nn + idx] = val;
}

// ---- setup kernels ----

// kappa on a coarser level: each coarse triangle takes the mean of its four children
// (exact integration of a(.,.) on the nested spaces).
__global__ __launch_bounds__(NTG) void k_coarsen_kappa(const double* lo_f, const double* up_f,
                                                       double* lo_c, double* up_c, int Nc) {
  const int idx = blockIdx.x * NTG + threadIdx.x;
  if (idx >= Nc * Nc) return;
  const int J = grid_row(idx, Nc), I = idx - J * Nc;
  const int Nf = 2 * Nc;
  const int a = (2 * J) * Nf + 2 * I;  // fine cell (2I, 2J)
  lo_c[idx] = 0.25 * (lo_f[a] + lo_f[a + 1] + up_f[a + 1] + lo_f[a + Nf + 1]);
  up_c[idx] = 0.25 * (up_f[a] + up_f[a + Nf] + lo_f[a + Nf] + up_f[a + Nf + 1]);
}

// Coefficient kind 3 on the finest level: the seven-point stiffness and mass of every
// node from the element matrices of the (up to) six triangles around it.  On a triangle
// with legs h along x and y, A and phi constant, a(phi_a, phi_b) = g_a . A g_b / 2 with
// g the gradients scaled by h, and b(phi_a, phi_b) = phi h^2 (1 + delta_ab) / 24.  Input:
// coef[c][t][J][I] (c: a11, a12, a22, phi; t: 0 below the SW-NE diagonal, 1 above).
// Output: the 7 planes described in ProbDev::st7 and the FP32 copy of the stiffness
// planes (stf).  h2 = h^2 on this level.
__global__ __launch_bounds__(NTG) void k_tensor_fine(const double* coef, double* st, float* stf,
                                                     int N, double h2) {
  const int n1 = N + 1;
  const int64_t pl = (int64_t)n1 * n1, cells = (int64_t)N * N;
  const int64_t idx = (int64_t)blockIdx.x * NTG + threadIdx.x;
  if (idx >= pl) return;
  const int gy = grid_row(idx, n1), gx = (int)(idx - (int64_t)gy * n1);
  // vertices (lattice offsets from the cell's SW corner) and scaled gradients
  const int vx[2][3] = {{0, 1, 1}, {0, 1, 0}}, vy[2][3] = {{0, 0, 1}, {0, 1, 1}};
  const double gxv[2][3] = {{-1.0, 1.0, 0.0}, {0.0, 1.0, -1.0}};
  const double gyv[2][3] = {{0.0, -1.0, 1.0}, {-1.0, 0.0, 1.0}};
  const int dx[4] = {0, 1, 0, 1}, dy[4] = {0, 0, 1, 1};
  double kv[4] = {0.0, 0.0, 0.0, 0.0}, mv[4] = {0.0, 0.0, 0.0, 0.0};
  for (int J = gy - 1; J <= gy; ++J) {
    for (int I = gx - 1; I <= gx; ++I) {
      if (I < 0 || J < 0 || I >= N || J >= N) continue;
      for (int t = 0; t < 2; ++t) {
        int a = -1;
        for (int k = 0; k < 3; ++k)
          if (I + vx[t][k] == gx && J + vy[t][k] == gy) a = k;
        if (a < 0) continue;
        const int64_t c = (int64_t)J * N + I;
        const double a11 = coef[(0 * 2 + t) * cells + c], a12 = coef[(1 * 2 + t) * cells + c];
        const double a22 = coef[(2 * 2 + t) * cells + c], phi = coef[(3 * 2 + t) * cells + c];
        for (int o = 0; o < 4; ++o) {
          int b = -1;
          for (int k = 0; k < 3; ++k)
            if (I + vx[t][k] == gx + dx[o] && J + vy[t][k] == gy + dy[o]) b = k;
          if (b < 0) continue;
          const double ag_x = a11 * gxv[t][b] + a12 * gyv[t][b];
          const double ag_y = a12 * gxv[t][b] + a22 * gyv[t][b];
          kv[o] += 0.5 * (gxv[t][a] * ag_x + gyv[t][a] * ag_y);
          mv[o] += phi * (a == b ? 2.0 : 1.0) / 24.0;
        }
      }
    }
  }
  // the diagonal kv[0] equals the sum of the weights (zero row sums) and is not stored
  for (int o = 1; o < 4; ++o) {
    st[(o - 1) * pl + idx] = -kv[o];  // stored as weights -K(i, j)
    stf[(o - 1) * pl + idx] = (float)(-kv[o]);
  }
  for (int o = 0; o < 4; ++o) st[(3 + o) * pl + idx] = mv[o] * h2;
}

// Coefficient kind 3 on a coarser level: the Galerkin product P^T A P of the seven-point
// stiffness and mass one level finer (exact integration on the nested spaces).  The
// coarse basis function of node I is 1 at fine node 2I and 1/2 at its six neighbours
// 2I +- (1,0), +-(0,1), +-(1,1); A_c(I, J) = sum over those fine nodes f of I and g of J
// of P(f,I) A_f(f,g) P(g,J).  Fine nodes off the grid are skipped: the hat functions of
// boundary nodes are cut at the boundary of the box, where no fine node lies beyond it
// (weights towards nodes off the grid are zero on every level).  The stiffness diagonal of
// a fine node is the sum of its weights to the neighbours on the grid (zero row sums
// hold for the cut hats of boundary nodes too).
__global__ __launch_bounds__(NTG) void k_galerkin7(const double* fine, double* coarse,
                                                   float* coarsef, int Nc) {
  const int nc1 = Nc + 1, Nf = 2 * Nc, nf1 = Nf + 1;
  const int64_t plc = (int64_t)nc1 * nc1, plf = (int64_t)nf1 * nf1;
  const int64_t idx = (int64_t)blockIdx.x * NTG + threadIdx.x;
  if (idx >= plc) return;
  const int Y = grid_row(idx, nc1), X = (int)(idx - (int64_t)Y * nc1);
  const int ox[7] = {0, 1, -1, 0, 0, 1, -1}, oy[7] = {0, 0, 0, 1, -1, 1, -1};
  const double ow[7] = {1.0, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5};
  const int dx[4] = {0, 1, 0, 1}, dy[4] = {0, 0, 1, 1};
  // matrix entry A_f(f, f + (ex, ey)) of operator `op` (0 stiffness, 1 mass) on the fine
  // grid; both nodes on the grid.  Stiffness planes: weights -K(i, i+E), -K(i, i+N),
  // -K(i, i+NE); mass planes: M(i,i), M(i,i+E), M(i,i+N), M(i,i+NE).
  auto entry = [&](int op, int fx, int fy, int ex, int ey) -> double {
    const int64_t f = (int64_t)fy * nf1 + fx;
    if (op == 0 && ex == 0 && ey == 0) {
      const double* K = fine;
      double d = K[f] + K[plf + f] + K[2 * plf + f];
      if (fx > 0) d += K[f - 1];
      if (fy > 0) d += K[plf + f - nf1];
      if (fx > 0 && fy > 0) d += K[2 * plf + f - nf1 - 1];
      return d;
    }
    const double sg = op == 0 ? -1.0 : 1.0;
    int k = 0;
    int64_t at = f;
    if (ex == 0 && ey == 0) k = 0;
    else if (ex == 1 && ey == 0) k = 1;
    else if (ex == 0 && ey == 1) k = 2;
    else if (ex == 1 && ey == 1) k = 3;
    else if (ex == -1 && ey == 0) { k = 1; at = f - 1; }
    else if (ex == 0 && ey == -1) { k = 2; at = f - nf1; }
    else if (ex == -1 && ey == -1) { k = 3; at = f - nf1 - 1; }
    else return 0.0;
    // stiffness: plane k-1 (k >= 1 here); mass: plane 3+k
    const int64_t plane = op == 0 ? k - 1 : 3 + k;
    return sg * fine[plane * plf + at];
  };
  for (int op = 0; op < 2; ++op) {
    for (int o = 0; o < 4; ++o) {
      double acc = 0.0;
      for (int a = 0; a < 7; ++a) {
        const int fx = 2 * X + ox[a], fy = 2 * Y + oy[a];
        if (fx < 0 || fy < 0 || fx > Nf || fy > Nf) continue;
        for (int b = 0; b < 7; ++b) {
          const int gx = 2 * (X + dx[o]) + ox[b], gy = 2 * (Y + dy[o]) + oy[b];
          if (gx < 0 || gy < 0 || gx > Nf || gy > Nf) continue;
          const int ex = gx - fx, ey = gy - fy;
          if (ex < -1 || ex > 1 || ey < -1 || ey > 1 || ex * ey < 0) continue;
          acc += ow[a] * ow[b] * entry(op, fx, fy, ex, ey);
        }
      }
      if (op == 0) {
        if (o == 0) continue;  // the diagonal is not stored
        coarse[(int64_t)(o - 1) * plc + idx] = -acc;
        coarsef[(int64_t)(o - 1) * plc + idx] = (float)(-acc);
      } else {
        coarse[(int64_t)(3 + o) * plc + idx] = acc;
      }
    }
  }
}

// Coarse stiffness K_H and consistent mass M_H (dense, column-major) on V_0H.
template <int KIND>
__global__ __launch_bounds__(NTG) void k_coarse_matrices(const ProbDev* probs) {
  const ProbDev& P = probs[blockIdx.y];
  const int r = blockIdx.x * NTG + threadIdx.x;
  if (r >= P.nH) return;
  const int nH = P.nH, N = P.n_c, n1 = N + 1;
  const int node = P.coarse_nodes[r];
  const int gy = node / n1, gx = node - gy * n1;
  const Weights W = edge_weights<KIND>(P, 0, N, gx, gy);
  const double H = P.side / N;
  const double mh = H * H / 12.0;
  const MassW Mw = mass_weights<KIND>(P, 0, N, gx, gy, mh);
  P.Kc[(int64_t)r * nH + r] = diag_of<KIND>(W);
  P.Mc[(int64_t)r * nH + r] = Mw.d;
  const int dx[6] = {1, -1, 0, 0, 1, -1}, dy[6] = {0, 0, 1, -1, 1, -1};
  const double kw[6] = {W.e, W.w, W.n, W.s, KIND == 3 ? W.ne : 0.0, KIND == 3 ? W.sw : 0.0};
  const double mw[6] = {Mw.e, Mw.w, Mw.n, Mw.s, Mw.ne, Mw.sw};
  for (int t = 0; t < 6; ++t) {
    const int c = P.coarse_index[(gy + dy[t]) * n1 + gx + dx[t]];
    if (c < 0) continue;
    P.Kc[(int64_t)c * nH + r] = -kw[t];
    P.Mc[(int64_t)c * nH + r] = mw[t];
  }
}

__global__ __launch_bounds__(NTG) void k_init_u0(const ProbDev* probs, int dst) {
  const ProbDev& P = probs[blockIdx.y];
  const int nc1 = P.c1;
  const int idx = blockIdx.x * NTG + threadIdx.x;
  if (idx >= nc1 * nc1) return;
  const int r = P.coarse_index[idx];
  for (int k = 0; k < P.q; ++k) {
    P.u[dst][(int64_t)k * nc1 * nc1 + idx] = r >= 0 ? P.V[(int64_t)k * P.nH + r] : 0.0;
    if (idx == 0) P.lam[dst * MLC_MAX_Q + k] = P.Lam[k];
  }
}

// Exact inverse of each subdomain's coarsest-grid operator K_H restricted to the coarse
// interior nodes of Omega_j (Gauss-Jordan, SPD so no pivoting: in LDS up to 64 nodes, in
// place in HBM up to 1024, O(n^3) at setup).  Nodes outside the domain get identity
// rows.  One workgroup per subdomain (first item of it).
template <int KIND>
__device__ __forceinline__ double tile_coarse_entry(const ProbDev& P, const TileItem& it, int nx,
                                                    int n, int e) {
  const int N = P.n_c;
  const int i = e / n, j = e - i * n;
  const int ix = i % nx, iy = i / nx;
  const int gx = it.cx0 + 1 + ix, gy = it.cy0 + 1 + iy;
  if (!is_dof(P.domain, N, gx, gy)) return (i == j) ? 1.0 : 0.0;
  const int jx = j % nx, jy = j / nx;
  const bool dj = is_dof(P.domain, N, it.cx0 + 1 + jx, it.cy0 + 1 + jy);
  const Weights W = edge_weights<KIND>(P, 0, N, gx, gy);
  if (i == j) return diag_of<KIND>(W);
  if (dj && jy == iy && jx == ix + 1) return -W.e;
  if (dj && jy == iy && jx == ix - 1) return -W.w;
  if (dj && jx == ix && jy == iy + 1) return -W.n;
  if (dj && jx == ix && jy == iy - 1) return -W.s;
  if constexpr (KIND == 3) {
    if (dj && jx == ix + 1 && jy == iy + 1) return -W.ne;
    if (dj && jx == ix - 1 && jy == iy - 1) return -W.sw;
  }
  return 0.0;
}

template <int KIND>
__global__ __launch_bounds__(NTG) void k_tile_inverse(const ProbDev* probs, const TileItem* items,
                                                       double* inv) {
  __shared__ double A[MLC_MAX_TILE_COARSE * MLC_MAX_TILE_COARSE];
  __shared__ double rowk[MLC_MAX_TILE_COARSE_ALL], colk[MLC_MAX_TILE_COARSE_ALL];
  constexpr int PER = MLC_MAX_TILE_COARSE * MLC_MAX_TILE_COARSE / NTG;
  const TileItem it = items[blockIdx.x];
  if (it.rhs != 0) return;
  const ProbDev& P = probs[it.prob];
  const int nx = it.cw - 1, ny = it.ch - 1, n = nx * ny;
  if (n > MLC_MAX_TILE_COARSE) {
    // Gauss-Jordan in place in HBM: pivot row and column of each step are first copied
    // to LDS, so every entry is updated from its own old value and the two copies
    double* G = inv + it.inv_off;
    for (int e = threadIdx.x; e < n * n; e += NTG) G[e] = tile_coarse_entry<KIND>(P, it, nx, n, e);
    for (int k = 0; k < n; ++k) {
      __syncthreads();
      for (int t = threadIdx.x; t < n; t += NTG) {
        rowk[t] = G[(int64_t)k * n + t];
        colk[t] = G[(int64_t)t * n + k];
      }
      __syncthreads();
      const double pk = 1.0 / rowk[k];
      for (int e = threadIdx.x; e < n * n; e += NTG) {
        const int i = e / n, j = e - i * n;
        double v;
        if (i == k && j == k)
          v = pk;
        else if (i == k)
          v = rowk[j] * pk;
        else if (j == k)
          v = -colk[i] * pk;
        else
          v = G[e] - colk[i] * rowk[j] * pk;
        G[e] = v;
      }
    }
    return;
  }
  for (int e = threadIdx.x; e < n * n; e += NTG) A[e] = tile_coarse_entry<KIND>(P, it, nx, n, e);
  double tmp[PER];
  for (int k = 0; k < n; ++k) {
    __syncthreads();
    const double pk = 1.0 / A[k * n + k];
    int c = 0;
    for (int e = threadIdx.x; e < n * n; e += NTG, ++c) {
      const int i = e / n, j = e - i * n;
      double v;
      if (i == k && j == k)
        v = pk;
      else if (i == k)
        v = A[k * n + j] * pk;
      else if (j == k)
        v = -A[i * n + k] * pk;
      else
        v = A[e] - A[i * n + k] * A[k * n + j] * pk;
      tmp[c] = v;
    }
    __syncthreads();
    c = 0;
    for (int e = threadIdx.x; e < n * n; e += NTG, ++c) A[e] = tmp[c];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += NTG) inv[it.inv_off + e] = A[e];
}

// Output sign (b(u, u) = 1 in Algorithm 4.1 step 3 fixes u only up to sign).  Per
// eigenvector: the nodal sum, the sum of magnitudes and the largest magnitude, each in two
// fixed-order stages (64 blocks, then one pass over their partials).  The sum decides when
// it exceeds 1e-8 of the magnitudes' sum; otherwise (an eigenvector odd under a symmetry
// of the problem, whose sum is rounding noise) the first node in grid order whose
// magnitude lies within a relative 1e-6 of the largest is made positive: the largest
// magnitudes of such a vector come in pairs of opposite sign that tie in exact
// arithmetic, and the relative band makes the choice stable under rounding.
// Partials: parts[(k * 4 + c) * nblk + block], c = 0 sum, 1 magnitudes, 2 largest
// magnitude, 3 first index within the band (as a double, exact below 2^53).
constexpr double kSignSumRtol = 1e-8;
constexpr double kSignMaxRtol = 1e-6;

__global__ __launch_bounds__(NTG) void k_sign_parts(const double* u, int64_t nn, int q,
                                                    double* parts, int nblk) {
  __shared__ double red[3][NTG / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < q; ++k) {
    double s = 0.0, a = 0.0, mx = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NTG + threadIdx.x; i < nn; i += (int64_t)nblk * NTG) {
      const double v = u[(int64_t)k * nn + i];
      s += v;
      a += fabs(v);
      mx = fmax(mx, fabs(v));
    }
    s = wave_sum(s);
    a = wave_sum(a);
    mx = read_lane_f64(group_reduce_last(mx, 64, 0.0, [](double x, double y) { return fmax(x, y); }), 63);
    __syncthreads();
    if (lane == 0) {
      red[0][wid] = s;
      red[1][wid] = a;
      red[2][wid] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double ts = 0.0, ta = 0.0, tm = 0.0;
      for (int w = 0; w < NTG / 64; ++w) {
        ts += red[0][w];
        ta += red[1][w];
        tm = fmax(tm, red[2][w]);
      }
      parts[(k * 4 + 0) * nblk + blockIdx.x] = ts;
      parts[(k * 4 + 1) * nblk + blockIdx.x] = ta;
      parts[(k * 4 + 2) * nblk + blockIdx.x] = tm;
    }
  }
}

__global__ __launch_bounds__(NTG) void k_sign_first(const double* u, int64_t nn, int q,
                                                    double* parts, int nblk) {
  __shared__ double red[NTG / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const double none = (double)nn;
  for (int k = 0; k < q; ++k) {
    double mx = 0.0;
    for (int b = 0; b < nblk; ++b) mx = fmax(mx, parts[(k * 4 + 2) * nblk + b]);
    const double thr = (1.0 - kSignMaxRtol) * mx;
    double first = none;  // each thread visits its nodes in ascending order
    for (int64_t i = (int64_t)blockIdx.x * NTG + threadIdx.x; i < nn; i += (int64_t)nblk * NTG)
      if (first == none && fabs(u[(int64_t)k * nn + i]) >= thr) first = (double)i;
    first = read_lane_f64(
        group_reduce_last(first, 64, none, [](double x, double y) { return fmin(x, y); }), 63);
    __syncthreads();
    if (lane == 0) red[wid] = first;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = none;
      for (int w = 0; w < NTG / 64; ++w) t = fmin(t, red[w]);
      parts[(k * 4 + 3) * nblk + blockIdx.x] = t;
    }
  }
}

__global__ __launch_bounds__(NTG) void k_copy_signed(const double* u, int64_t nn, int q,
                                                     const double* parts, int nblk, double* out) {
  const int64_t idx = (int64_t)blockIdx.x * NTG + threadIdx.x;
  if (idx >= nn) return;
  for (int k = 0; k < q; ++k) {
    double s = 0.0, a = 0.0, first = (double)nn;
    for (int b = 0; b < nblk; ++b) {
      s += parts[(k * 4 + 0) * nblk + b];
      a += parts[(k * 4 + 1) * nblk + b];
      first = fmin(first, parts[(k * 4 + 3) * nblk + b]);
    }
    bool flip;
    if (fabs(s) > kSignSumRtol * a)
      flip = s < 0.0;
    else
      flip = first < (double)nn && u[(int64_t)k * nn + (int64_t)first] < 0.0;
    out[(int64_t)k * nn + idx] = (flip ? -1.0 : 1.0) * u[(int64_t)k * nn + idx];
  }
}

__global__ __launch_bounds__(NTG) void k_set_state(const ProbDev* probs, int level, int dst,
                                                   const double* in) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << (level + P.order - 1);
  const int n1 = N + 1;
  const int64_t nn = (int64_t)n1 * n1;
  const int64_t idx = (int64_t)blockIdx.x * NTG + threadIdx.x;
  if (idx >= nn) return;
  const int gy = grid_row(idx, n1), gx = (int)(idx - (int64_t)gy * n1);
  const bool dof = is_dof(P.domain, N, gx, gy);
  for (int k = 0; k < P.q; ++k)
    P.u[dst][(int64_t)k * nn + idx] = dof ? in[(int64_t)k * nn + idx] : 0.0;
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + NTG - 1) / NTG); }

}  // namespace

hipError_t launch_prolong_residual(int kind, const ProbDev* probs, int nprob, int m, int src,
                                   int64_t max_nodes, int max_q, hipStream_t s) {
  dim3 g(nblocks(max_nodes), nprob, max_q);
  if (kind == 0)
    hipLaunchKernelGGL(k_prolong_residual<0>, g, dim3(NTG), 0, s, probs, m, src);
  else if (kind == 1)
    hipLaunchKernelGGL(k_prolong_residual<1>, g, dim3(NTG), 0, s, probs, m, src);
  else if (kind == 2)
    hipLaunchKernelGGL(k_prolong_residual<2>, g, dim3(NTG), 0, s, probs, m, src);
  else
    hipLaunchKernelGGL(k_prolong_residual<3>, g, dim3(NTG), 0, s, probs, m, src);
  return hipGetLastError();
}

hipError_t launch_pou_glue(const ProbDev* probs, int nprob, const TileItem* items,
                           const int32_t* sub_item, const char* store, int m, int64_t max_nodes,
                           int max_q, hipStream_t s) {
  const dim3 g(nblocks(max_nodes), nprob);
#define MLC_GLUE(QM) \
  hipLaunchKernelGGL(k_pou_glue<QM>, g, dim3(NTG), 0, s, probs, items, sub_item, store, m)
  if (max_q <= 1)
    MLC_GLUE(1);
  else if (max_q <= 2)
    MLC_GLUE(2);
  else if (max_q <= 4)
    MLC_GLUE(4);
  else
    MLC_GLUE(8);
#undef MLC_GLUE
  return hipGetLastError();
}

hipError_t launch_rr_apply(int kind, const ProbDev* probs, int nprob, int m, int64_t max_nodes,
                           int max_q, hipStream_t s) {
  const dim3 g(nblocks(max_nodes), nprob);
#define MLC_APPLY(K, QM) hipLaunchKernelGGL((k_rr_apply<K, QM>), g, dim3(NTG), 0, s, probs, m)
#define MLC_APPLY_Q(K)   \
  if (max_q <= 1)        \
    MLC_APPLY(K, 1);     \
  else if (max_q <= 2)   \
    MLC_APPLY(K, 2);     \
  else if (max_q <= 4)   \
    MLC_APPLY(K, 4);     \
  else                   \
    MLC_APPLY(K, 8)
  if (kind == 0) {
    MLC_APPLY_Q(0);
  } else if (kind == 1) {
    MLC_APPLY_Q(1);
  } else if (kind == 2) {
    MLC_APPLY_Q(2);
  } else {
    MLC_APPLY_Q(3);
  }
#undef MLC_APPLY_Q
#undef MLC_APPLY
  return hipGetLastError();
}

hipError_t launch_restrict(const ProbDev* probs, int nprob, int l, int m, int64_t max_nodes_l,
                           int max_q, hipStream_t s) {
  hipLaunchKernelGGL(k_restrict, dim3(nblocks(max_nodes_l), nprob, 2 * max_q), dim3(NTG), 0, s,
                     probs, l, m);
  return hipGetLastError();
}

hipError_t launch_rr_project(const ProbDev* probs, int nprob, int max_nH, int max_q,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_rr_project, dim3((max_nH + 3) / 4, nprob, 2 * max_q), dim3(NTG), 0, s,
                     probs);
  return hipGetLastError();
}

hipError_t launch_rr_combine(const ProbDev* probs, int nprob, int max_nc1sq, int max_q,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_rr_combine, dim3((max_nc1sq + NTG / 64 - 1) / (NTG / 64), nprob, max_q),
                     dim3(NTG), 0, s, probs);
  return hipGetLastError();
}

hipError_t launch_assemble(const ProbDev* probs, int nprob, int m, int dst, int64_t max_nodes,
                           int max_q, hipStream_t s) {
  hipLaunchKernelGGL(k_assemble, dim3(nblocks(max_nodes), nprob, max_q), dim3(NTG), 0, s, probs,
                     m, dst);
  return hipGetLastError();
}

hipError_t launch_coarsen_kappa(const double* lo_f, const double* up_f, double* lo_c,
                                double* up_c, int Nc, hipStream_t s) {
  hipLaunchKernelGGL(k_coarsen_kappa, dim3(nblocks((int64_t)Nc * Nc)), dim3(NTG), 0, s, lo_f,
                     up_f, lo_c, up_c, Nc);
  return hipGetLastError();
}

hipError_t launch_tensor_fine(const double* coef, double* st, float* stf, int N, double h2,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_tensor_fine, dim3(nblocks((int64_t)(N + 1) * (N + 1))), dim3(NTG), 0, s,
                     coef, st, stf, N, h2);
  return hipGetLastError();
}

hipError_t launch_galerkin7(const double* fine, double* coarse, float* coarsef, int Nc,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_galerkin7, dim3(nblocks((int64_t)(Nc + 1) * (Nc + 1))), dim3(NTG), 0, s,
                     fine, coarse, coarsef, Nc);
  return hipGetLastError();
}

hipError_t launch_coarse_matrices(int kind, const ProbDev* probs, int nprob, int max_nH,
                                  hipStream_t s) {
  dim3 g(nblocks(max_nH), nprob);
  if (kind == 0)
    hipLaunchKernelGGL(k_coarse_matrices<0>, g, dim3(NTG), 0, s, probs);
  else if (kind == 1)
    hipLaunchKernelGGL(k_coarse_matrices<1>, g, dim3(NTG), 0, s, probs);
  else if (kind == 2)
    hipLaunchKernelGGL(k_coarse_matrices<2>, g, dim3(NTG), 0, s, probs);
  else
    hipLaunchKernelGGL(k_coarse_matrices<3>, g, dim3(NTG), 0, s, probs);
  return hipGetLastError();
}

hipError_t launch_init_u0(const ProbDev* probs, int nprob, int dst, int max_nc1sq, hipStream_t s) {
  hipLaunchKernelGGL(k_init_u0, dim3(nblocks(max_nc1sq), nprob), dim3(NTG), 0, s, probs, dst);
  return hipGetLastError();
}

hipError_t launch_tile_inverse(int kind, const ProbDev* probs, const TileItem* items, int nitems,
                               double* inv, hipStream_t s) {
  if (kind == 0)
    hipLaunchKernelGGL(k_tile_inverse<0>, dim3(nitems), dim3(NTG), 0, s, probs, items, inv);
  else if (kind == 1)
    hipLaunchKernelGGL(k_tile_inverse<1>, dim3(nitems), dim3(NTG), 0, s, probs, items, inv);
  else if (kind == 2)
    hipLaunchKernelGGL(k_tile_inverse<2>, dim3(nitems), dim3(NTG), 0, s, probs, items, inv);
  else
    hipLaunchKernelGGL(k_tile_inverse<3>, dim3(nitems), dim3(NTG), 0, s, probs, items, inv);
  return hipGetLastError();
}

hipError_t launch_output_signed(const double* u, int64_t nn, int q, double* parts, double* out,
                                hipStream_t s) {
  const int nblk = 64;  // parts: 4 * q * nblk doubles
  hipLaunchKernelGGL(k_sign_parts, dim3(nblk), dim3(NTG), 0, s, u, nn, q, parts, nblk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sign_first, dim3(nblk), dim3(NTG), 0, s, u, nn, q, parts, nblk);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_copy_signed, dim3(nblocks(nn)), dim3(NTG), 0, s, u, nn, q, parts, nblk, out);
  return hipGetLastError();
}

hipError_t launch_set_state(const ProbDev* prob, int level, int dst, const double* in,
                            int64_t nn, hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(nblocks(nn)), dim3(NTG), 0, s, prob, level, dst, in);
  return hipGetLastError();
}
