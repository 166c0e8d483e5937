// Device building blocks of the batched local solves (Algorithm 4.1 step 1): tile
// level descriptors, the symmetric multigrid V-cycle and the preconditioned conjugate
// gradient loop, templated on the vector type of the tile buffers (double, or float for
// the mixed-precision solver).  Included by the FP64 and the mixed-precision kernels.
//
// Vectors of an item live in its slice of the workspace, row-major over the tile's
// interior nodes (no halo: outside the tile is the Dirichlet boundary, read as 0).
// Waves sweep rows, 64 consecutive nodes per wave, so every access is coalesced.
#pragma once
#include "mlc_launch.h"

namespace {

struct LevelDesc {
  int nx, ny, gx0, gy0, N, l;
  int64_t ob, oz, ot;  // element offsets of right-hand side, iterate, temporary
};

#define FOR_TILE(lv)                                                  \
  for (int iy = threadIdx.x >> 6; iy < (lv).ny; iy += NT / 64)       \
    for (int ix = threadIdx.x & 63; ix < (lv).nx; ix += 64)

template <int KIND, typename T>
__device__ __forceinline__ T stencil(const ProbDev& P, const LevelDesc& lv, const T* u, int ix,
                                     int iy, int64_t i, T& diag) {
  const Weights W = edge_weights<KIND>(P, lv.l, lv.N, lv.gx0 + ix, lv.gy0 + iy);
  const T c = u[i];
  const T e = (ix + 1 < lv.nx) ? u[i + 1] : T(0);
  const T w = (ix > 0) ? u[i - 1] : T(0);
  const T n = (iy + 1 < lv.ny) ? u[i + lv.nx] : T(0);
  const T s = (iy > 0) ? u[i - lv.nx] : T(0);
  const T we = T(W.e), ww = T(W.w), wn = T(W.n), ws = T(W.s);
  diag = we + ww + wn + ws;
  return diag * c - we * e - ww * w - wn * n - ws * s;
}

// z = omega D^-1 b (first sweep from a zero iterate)
template <int NT, int KIND, typename T>
__device__ void op_first(const ProbDev& P, const LevelDesc& lv, const T* b, T* z, T omega) {
  FOR_TILE(lv) {
    const int64_t i = (int64_t)iy * lv.nx + ix;
    T v = T(0);
    if (is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + iy)) {
      const Weights W = edge_weights<KIND>(P, lv.l, lv.N, lv.gx0 + ix, lv.gy0 + iy);
      v = omega * b[i] / T(W.e + W.w + W.n + W.s);
    }
    z[i] = v;
  }
}

// zo = zi + omega D^-1 (b - A zi)
template <int NT, int KIND, typename T>
__device__ void op_jacobi(const ProbDev& P, const LevelDesc& lv, const T* b, const T* zi, T* zo,
                          T omega) {
  FOR_TILE(lv) {
    const int64_t i = (int64_t)iy * lv.nx + ix;
    T v = T(0);
    if (is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + iy)) {
      T d;
      const T az = stencil<KIND, T>(P, lv, zi, ix, iy, i, d);
      v = zi[i] + omega * (b[i] - az) / d;
    }
    zo[i] = v;
  }
}

// ro = b - A z
template <int NT, int KIND, typename T>
__device__ void op_residual(const ProbDev& P, const LevelDesc& lv, const T* b, const T* z, T* ro) {
  FOR_TILE(lv) {
    const int64_t i = (int64_t)iy * lv.nx + ix;
    T v = T(0);
    if (is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + iy)) {
      T d;
      v = b[i] - stencil<KIND, T>(P, lv, z, ix, iy, i, d);
    }
    ro[i] = v;
  }
}

// bc = P^T rf: coarse node (cx, cy) sits on fine node (2cx+1, 2cy+1) of the tile.
template <int NT, typename T>
__device__ void op_restrict(const ProbDev& P, const LevelDesc& lf, const LevelDesc& lc,
                            const T* rf, T* bc) {
  const int nf = lf.nx;
  FOR_TILE(lc) {
    const int64_t i = (int64_t)iy * lc.nx + ix;
    T v = T(0);
    if (is_dof(P.domain, lc.N, lc.gx0 + ix, lc.gy0 + iy)) {
      const int64_t c = (int64_t)(2 * iy + 1) * nf + (2 * ix + 1);
      v = rf[c] + T(0.5) * (rf[c + 1] + rf[c - 1] + rf[c + nf] + rf[c - nf] + rf[c + nf + 1] +
                            rf[c - nf - 1]);
    }
    bc[i] = v;
  }
}

// zf += P zc (P1 interpolation on the SW-NE mesh; coarse nodes outside the tile are 0)
template <int NT, typename T>
__device__ void op_prolong_add(const ProbDev& P, const LevelDesc& lc, const LevelDesc& lf,
                               const T* zc, T* zf) {
  const int ncx = lc.nx, ncy = lc.ny;
  FOR_TILE(lf) {
    if (!is_dof(P.domain, lf.N, lf.gx0 + ix, lf.gy0 + iy)) continue;
    const int64_t i = (int64_t)iy * lf.nx + ix;
    auto at = [&](int cx, int cy) -> T {
      return (cx >= 0 && cy >= 0 && cx < ncx && cy < ncy) ? zc[(int64_t)cy * ncx + cx] : T(0);
    };
    T v;
    const bool ox = ix & 1, oy = iy & 1;  // odd tile index = even global index = coarse node
    if (ox && oy)
      v = at(ix >> 1, iy >> 1);
    else if (!ox && oy)
      v = T(0.5) * (at((ix >> 1) - 1, iy >> 1) + at(ix >> 1, iy >> 1));
    else if (ox && !oy)
      v = T(0.5) * (at(ix >> 1, (iy >> 1) - 1) + at(ix >> 1, iy >> 1));
    else
      v = T(0.5) * (at((ix >> 1) - 1, (iy >> 1) - 1) + at(ix >> 1, iy >> 1));
    zf[i] += v;
  }
}

// z = K_c^-1 b on the coarse-cell grid of the tile (dense inverse from setup)
template <int NT, typename T>
__device__ void op_coarse_solve(const LevelDesc& lc, const double* Kinv, const T* b, T* z) {
  const int n = lc.nx * lc.ny;
  for (int e = threadIdx.x; e < n; e += NT) {
    double s = 0.0;
    const double* row = Kinv + (int64_t)e * n;
    for (int j = 0; j < n; ++j) s += row[j] * (double)b[j];
    z[e] = T(s);
  }
}

// One symmetric V-cycle applied to the level-0 right-hand side at lev[0].ob; returns
// the buffer that holds the result.
template <int NT, int KIND, typename T>
__device__ T* vcycle(const ProbDev& P, const LevelDesc* lev, T* base, int m, const double* Kinv,
                     int nu, T omega) {
  for (int t = 0; t < m; ++t) {
    const LevelDesc& lv = lev[t];
    const T* b = base + lv.ob;
    T* za = base + lv.oz;
    T* zb = base + lv.ot;
    op_first<NT, KIND, T>(P, lv, b, za, omega);
    __syncthreads();
    for (int s = 1; s < nu; ++s) {
      op_jacobi<NT, KIND, T>(P, lv, b, za, zb, omega);
      __syncthreads();
      T* tmp = za;
      za = zb;
      zb = tmp;
    }
    op_residual<NT, KIND, T>(P, lv, b, za, zb);
    __syncthreads();
    op_restrict<NT, T>(P, lv, lev[t + 1], zb, base + lev[t + 1].ob);
    __syncthreads();
  }
  op_coarse_solve<NT, T>(lev[m], Kinv, base + lev[m].ob, base + lev[m].oz);
  __syncthreads();
  T* zc = base + lev[m].oz;
  for (int t = m - 1; t >= 0; --t) {
    const LevelDesc& lv = lev[t];
    const T* b = base + lv.ob;
    T* za = base + lv.oz;
    T* zb = base + lv.ot;
    if ((nu - 1) & 1) {
      T* tmp = za;
      za = zb;
      zb = tmp;
    }
    op_prolong_add<NT, T>(P, lev[t + 1], lv, zc, za);
    __syncthreads();
    for (int s = 0; s < nu; ++s) {
      op_jacobi<NT, KIND, T>(P, lv, b, za, zb, omega);
      __syncthreads();
      T* tmp = za;
      za = zb;
      zb = tmp;
    }
    zc = za;
  }
  return zc;
}

// Level descriptors of an item: t = 0 is the tile on level m, t = m its coarse-cell grid.
// Level-0 buffers: X, R(=rhs of the V-cycle), Z, Tmp, then extra vectors; coarser levels:
// B, Z, Tmp each.  Returns the element count of the item's storage.
__device__ inline int64_t fill_levels(const TileItem& it, const ProbDev& P, int m, int extra,
                               LevelDesc* lev) {
  int64_t off = 0;
  for (int t = 0; t <= m; ++t) {
    const int l = m - t;
    const int r = 1 << l;
    LevelDesc d;
    d.nx = it.cw * r - 1;
    d.ny = it.ch * r - 1;
    d.gx0 = it.cx0 * r + 1;
    d.gy0 = it.cy0 * r + 1;
    d.N = P.n_c << l;
    d.l = l;
    const int64_t S = (int64_t)d.nx * d.ny;
    if (t == 0) {
      d.ob = S;
      d.oz = 2 * S;
      d.ot = 3 * S;
      off = (4 + extra) * S;
    } else {
      d.ob = off;
      d.oz = off + S;
      d.ot = off + 2 * S;
      off += 3 * S;
    }
    lev[t] = d;
  }
  return off;
}

// Preconditioned conjugate gradients on K_j x = r with the V-cycle preconditioner, in
// the vector type T of the tile buffers (reductions in FP64).  On entry R (level-0
// right-hand side buffer) holds r and X is zero; bb = ||r||^2.  Iterates until
// ||r_k||^2 <= tol2 or max_it; returns the iteration count and the final ||r_k||^2 in rr.
template <int NT, int KIND, typename T>
__device__ int pcg_solve(const ProbDev& P, const LevelDesc* lev, T* base, int m, const double* Kinv,
                         double bb, double tol2, int max_it, int nu, double omega, double* red,
                         double& rr) {
  const LevelDesc& l0 = lev[0];
  const int64_t S0 = (int64_t)l0.nx * l0.ny;
  T* X = base;
  T* R = base + l0.ob;
  T* Pd = base + 4 * S0;
  T* Qd = base + 5 * S0;
  const T om = T(omega);
  int iters = 0;
  rr = bb;
  if (!(bb > 0.0)) return 0;
  double acc[2];
  T* Z = vcycle<NT, KIND, T>(P, lev, base, m, Kinv, nu, om);
  acc[0] = acc[1] = 0.0;
  FOR_TILE(l0) {
    const int64_t i = (int64_t)iy * l0.nx + ix;
    Pd[i] = Z[i];
    acc[0] += (double)R[i] * (double)Z[i];
  }
  block_sum<NT, 2>(acc, red);
  double rho = acc[0];
  while (iters < max_it) {
    ++iters;
    acc[0] = acc[1] = 0.0;
    FOR_TILE(l0) {
      const int64_t i = (int64_t)iy * l0.nx + ix;
      T q = T(0);
      if (is_dof(P.domain, l0.N, l0.gx0 + ix, l0.gy0 + iy)) {
        T d;
        q = stencil<KIND, T>(P, l0, Pd, ix, iy, i, d);
      }
      Qd[i] = q;
      acc[0] += (double)Pd[i] * (double)q;
    }
    block_sum<NT, 2>(acc, red);
    const T alpha = T(rho / acc[0]);
    acc[0] = acc[1] = 0.0;
    FOR_TILE(l0) {
      const int64_t i = (int64_t)iy * l0.nx + ix;
      X[i] += alpha * Pd[i];
      const T r = R[i] - alpha * Qd[i];
      R[i] = r;
      acc[0] += (double)r * (double)r;
    }
    block_sum<NT, 2>(acc, red);
    rr = acc[0];
    if (rr <= tol2) break;
    Z = vcycle<NT, KIND, T>(P, lev, base, m, Kinv, nu, om);
    acc[0] = acc[1] = 0.0;
    FOR_TILE(l0) {
      const int64_t i = (int64_t)iy * l0.nx + ix;
      acc[0] += (double)R[i] * (double)Z[i];
    }
    block_sum<NT, 2>(acc, red);
    const T beta = T(acc[0] / rho);
    rho = acc[0];
    FOR_TILE(l0) {
      const int64_t i = (int64_t)iy * l0.nx + ix;
      Pd[i] = Z[i] + beta * Pd[i];
    }
    __syncthreads();
  }
  return iters;
}

}  // namespace
