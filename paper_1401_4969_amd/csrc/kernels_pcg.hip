// Batched local solves of Algorithm 4.1 step 1, equation (Aux_Problem):
//   for every subdomain Omega_j and every eigenpair i, find e in V_0h(Omega_j) with
//   a(e, v) = lambda_i b(u_i, v) - a(u_i, v) for all v in V_0h(Omega_j),
// i.e. K_j e = r|_{T_j} with homogeneous Dirichlet data on the boundary of Omega_j.
//
// One workgroup owns one (subdomain, eigenpair) item and runs the whole preconditioned
// conjugate gradient to convergence with workgroup barriers only: the items are
// independent, so no grid-wide synchronisation is needed and the hardware dispatcher
// acts as the work queue (items are ordered largest first).  The preconditioner is a
// symmetric multigrid V-cycle over the nested grids of the tile (nu damped-Jacobi sweeps
// before and after each coarse correction, restriction P^T, interpolation P, Galerkin
// coarse operators = the same stencil with children-mean kappa, exact solve on the
// coarse-cell grid of Omega_j), so the work per item is O(tile size) (the multigrid remark
// after the work estimate of Section 5).
//
// Vectors of an item live in its slice of the workspace, row-major over the tile's
// interior nodes (no halo: outside the tile is the Dirichlet boundary, read as 0).
// Waves sweep rows, 64 consecutive nodes per wave, so every access is coalesced.
#include "mlc_launch.h"

namespace {

struct LevelDesc {
  int nx, ny, gx0, gy0, N, l;
  int64_t ob, oz, ot;  // element offsets of right-hand side, iterate, temporary
};

template <int NT>
struct Loop {
  static constexpr int TY = NT / 64;
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
__device__ int64_t fill_levels(const TileItem& it, const ProbDev& P, int m, int extra,
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

template <int NT, int KIND>
__global__ __launch_bounds__(NT) void k_local_pcg64(const ProbDev* probs, const TileItem* items,
                                                     char* store, const double* inv, int m,
                                                     ItemStat* stats, double rtol, int max_it,
                                                     int nu, double omega) {
  __shared__ LevelDesc lev[MLC_MAX_LEVELS + 1];
  __shared__ double red[2 * (NT / 64)];
  const TileItem it = items[blockIdx.x];
  const ProbDev& P = probs[it.prob];
  if (threadIdx.x == 0) fill_levels(it, P, m, 2, lev);
  __syncthreads();
  double* base = reinterpret_cast<double*>(store + it.off);
  const LevelDesc& l0 = lev[0];
  const int64_t S0 = (int64_t)l0.nx * l0.ny;
  double* X = base;
  double* R = base + l0.ob;
  double* Pd = base + 4 * S0;
  double* Qd = base + 5 * S0;
  const double* Kinv = inv + it.inv_off;
  const int n1 = l0.N + 1;
  const double* bglob = P.res + (int64_t)it.rhs * n1 * n1;

  double acc[2] = {0.0, 0.0};
  FOR_TILE(l0) {
    const int64_t i = (int64_t)iy * l0.nx + ix;
    const double v = bglob[(int64_t)(l0.gy0 + iy) * n1 + (l0.gx0 + ix)];
    R[i] = v;
    X[i] = 0.0;
    acc[0] += v * v;
  }
  block_sum<NT, 2>(acc, red);
  const double bb = acc[0];
  int iters = 0;
  double rr = bb;
  if (bb > 0.0) {
    const double tol2 = rtol * rtol * bb;
    double* Z = vcycle<NT, KIND, double>(P, lev, base, m, Kinv, nu, omega);
    acc[0] = acc[1] = 0.0;
    FOR_TILE(l0) {
      const int64_t i = (int64_t)iy * l0.nx + ix;
      Pd[i] = Z[i];
      acc[0] += R[i] * Z[i];
    }
    block_sum<NT, 2>(acc, red);
    double rho = acc[0];
    while (iters < max_it) {
      ++iters;
      acc[0] = acc[1] = 0.0;
      FOR_TILE(l0) {
        const int64_t i = (int64_t)iy * l0.nx + ix;
        double q = 0.0;
        if (is_dof(P.domain, l0.N, l0.gx0 + ix, l0.gy0 + iy)) {
          double d;
          q = stencil<KIND, double>(P, l0, Pd, ix, iy, i, d);
        }
        Qd[i] = q;
        acc[0] += Pd[i] * q;
      }
      block_sum<NT, 2>(acc, red);
      const double alpha = rho / acc[0];
      acc[0] = acc[1] = 0.0;
      FOR_TILE(l0) {
        const int64_t i = (int64_t)iy * l0.nx + ix;
        X[i] += alpha * Pd[i];
        const double r = R[i] - alpha * Qd[i];
        R[i] = r;
        acc[0] += r * r;
      }
      block_sum<NT, 2>(acc, red);
      rr = acc[0];
      if (rr <= tol2) break;
      Z = vcycle<NT, KIND, double>(P, lev, base, m, Kinv, nu, omega);
      acc[0] = acc[1] = 0.0;
      FOR_TILE(l0) {
        const int64_t i = (int64_t)iy * l0.nx + ix;
        acc[0] += R[i] * Z[i];
      }
      block_sum<NT, 2>(acc, red);
      const double beta = acc[0] / rho;
      rho = acc[0];
      FOR_TILE(l0) {
        const int64_t i = (int64_t)iy * l0.nx + ix;
        Pd[i] = Z[i] + beta * Pd[i];
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    ItemStat s;
    s.iters = iters;
    s.refine = 0;
    s.relres = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    stats[blockIdx.x] = s;
  }
}

}  // namespace

// Storage (bytes) one item needs at level m in the FP64 path.
int64_t item_bytes_fp64(int cw, int ch, int m) {
  int64_t total = 0;
  for (int t = 0; t <= m; ++t) {
    const int r = 1 << (m - t);
    const int64_t S = (int64_t)(cw * r - 1) * (ch * r - 1);
    total += (t == 0 ? 6 : 3) * S;
  }
  return total * (int64_t)sizeof(double);
}

hipError_t launch_local_pcg(int kind, int nt, const ProbDev* probs, const TileItem* items,
                            int nitems, char* store, const double* inv, int m, ItemStat* stats,
                            double rtol, int max_it, int nu, double omega, int64_t, hipStream_t s) {
#define MLC_PCG(NTV, KV)                                                                        \
  hipLaunchKernelGGL((k_local_pcg64<NTV, KV>), dim3(nitems), dim3(NTV), 0, s, probs, items,      \
                     store, inv, m, stats, rtol, max_it, nu, omega)
#define MLC_PCG_NT(NTV)    \
  if (kind == 0)           \
    MLC_PCG(NTV, 0);       \
  else if (kind == 1)      \
    MLC_PCG(NTV, 1);       \
  else                     \
    MLC_PCG(NTV, 2);
  if (nt == 256) {
    MLC_PCG_NT(256)
  } else if (nt == 512) {
    MLC_PCG_NT(512)
  } else {
    MLC_PCG_NT(1024)
  }
#undef MLC_PCG_NT
#undef MLC_PCG
  return hipGetLastError();
}

int64_t pcg_lds_bytes(const TileItem*, int, int, int) { return 0; }
