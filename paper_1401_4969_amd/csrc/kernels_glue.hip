// Algorithm 4.1 step 2 as the paper states it (gluing MLC_GLUE_INTERFACE): u~ = u~^j on
// G_j, and on G_{m+1} = Omega minus the closed G_j the solution of
//   a(u~, v) = lambda_k b(u_k, v) for all v in V_0h(G_{m+1}),
// with u~ = u~^j on the boundary of each G_j and 0 on the boundary of Omega (equation
// (G_m+1_Problem)).  G_j is D_j shrunk by half a coarse cell on every side, so the closed
// G_j are disjoint and lie inside the tiles.  In correction form (u~ = I u + e): e = e^j
// on each closed G_j, and on the remaining dofs S ("skeleton") K_SS e_S = r_S - K_SG e_G.
//
// The skeleton is one connected region of the whole grid, so it is solved by a global
// preconditioned CG (Jacobi) over full-grid vectors that vanish off S: one thread per
// node, a few launches per iteration for all q right-hand sides at once (blockIdx.y),
// scalars kept in device memory (no host round trip per iteration), block partial sums
// reduced in a fixed order (deterministic).  A right-hand side that has converged is
// frozen by a flag its reduction sets; the host polls the flags every 16 iterations.
//
// Per right-hand side i: vectors E, W, Z, P (two, used alternately), Q at vec + i*6*nodes;
// block partials at parts + i*2*nblk; scalars at scal + i*SKEL_NS: rho, alpha, beta,
// ||w||^2, ||w_0||^2, done, tol^2, iterations.
#include "mlc_launch.h"

namespace {

constexpr int NTS = 256;
constexpr int SKEL_NS = 8;  // scalars per right-hand side

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
                                                   int m, double* vec) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1, r = 1 << m;
  const int64_t nn = (int64_t)n1 * n1;
  const int i_rhs = blockIdx.y;
  double* E = vec + (int64_t)i_rhs * 6 * nn;
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

// w = r - K e on S (0 elsewhere), z = D^-1 w, p = z; partial sums (w.z, w.w).
template <int KIND>
__global__ __launch_bounds__(NTS) void k_skel_init(const ProbDev* probs, int m, double* vec,
                                                   double* parts_all) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1, r = 1 << m;
  const int64_t nn = (int64_t)n1 * n1;
  const int i_rhs = blockIdx.y;
  const double* E = vec + (int64_t)i_rhs * 6 * nn;
  double* Wv = vec + ((int64_t)i_rhs * 6 + 1) * nn;
  double* Z = vec + ((int64_t)i_rhs * 6 + 2) * nn;
  double* Pv = vec + ((int64_t)i_rhs * 6 + 3) * nn;
  double* parts = parts_all + (int64_t)i_rhs * 2 * gridDim.x;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  double wz = 0.0, ww = 0.0;
  if (idx < nn) {
    const int gy = (int)(idx / n1), gx = (int)(idx - (int64_t)gy * n1);
    double w = 0.0, z = 0.0;
    if (skel_dof(P, N, r, gx, gy)) {
      double d;
      w = P.res[(int64_t)i_rhs * nn + idx] - apply_masked<KIND>(P, m, N, n1, gx, gy, idx, E, d);
      z = w / d;
      wz = w * z;
      ww = w * w;
    }
    Wv[idx] = w;
    Z[idx] = z;
    Pv[idx] = z;
  }
  block_partials(wz, ww, parts);
}

// p_new = z + beta p_old on S (formed on the fly at the stencil points; 0 off S), stored
// in Pn; q = A p_new on S; partial sums (p.q, 0).  first: beta = 0, p_old unread.
template <int KIND>
__global__ __launch_bounds__(NTS) void k_skel_dir(const ProbDev* probs, int m, double* vec,
                                                  int po, const double* scal_all, int first,
                                                  double* parts_all) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1, r = 1 << m;
  const int64_t nn = (int64_t)n1 * n1;
  const int i_rhs = blockIdx.y;
  const double* scal = scal_all + i_rhs * SKEL_NS;
  if (scal[5] != 0.0) return;  // converged: frozen (uniform over the workgroup)
  double* base = vec + (int64_t)i_rhs * 6 * nn;
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

// e += alpha p, w -= alpha q, z = D^-1 w on S; partial sums (w.z, w.w).
template <int KIND>
__global__ __launch_bounds__(NTS) void k_skel_upd(const ProbDev* probs, int m, double* vec,
                                                  int pn, const double* scal_all,
                                                  double* parts_all) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1, r = 1 << m;
  const int64_t nn = (int64_t)n1 * n1;
  const int i_rhs = blockIdx.y;
  const double* scal = scal_all + i_rhs * SKEL_NS;
  if (scal[5] != 0.0) return;  // converged: frozen
  double* base = vec + (int64_t)i_rhs * 6 * nn;
  double* E = base;
  double* Wv = base + nn;
  double* Z = base + 2 * nn;
  const double* Pv = base + (3 + pn) * nn;
  const double* Q = base + 5 * nn;
  double* parts = parts_all + (int64_t)i_rhs * 2 * gridDim.x;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  const double alpha = scal[1];
  double wz = 0.0, ww = 0.0;
  if (idx < nn) {
    const int gy = (int)(idx / n1), gx = (int)(idx - (int64_t)gy * n1);
    if (skel_dof(P, N, r, gx, gy)) {
      const Weights W = edge_weights<KIND>(P, m, N, gx, gy);
      E[idx] += alpha * Pv[idx];
      const double w = Wv[idx] - alpha * Q[idx];
      const double z = w / diag_of<KIND>(W);
      Wv[idx] = w;
      Z[idx] = z;
      wz = w * z;
      ww = w * w;
    }
  }
  block_partials(wz, ww, parts);
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
                                                     const double* vec) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1;
  const int64_t nn = (int64_t)n1 * n1;
  const int i_rhs = blockIdx.y;
  const double* E = vec + (int64_t)i_rhs * 6 * nn;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  if (idx >= nn) return;
  const int gy = (int)(idx / n1), gx = (int)(idx - (int64_t)gy * n1);
  const int64_t o = (int64_t)i_rhs * nn + idx;
  P.ut[o] = is_dof(P.domain, N, gx, gy) ? P.ubar[o] + E[idx] : 0.0;
}

}  // namespace

hipError_t run_interface_gluing(int kind, const ProbDev* dprob, const TileItem* items,
                                const int32_t* sub_item, const char* store, int m, int q,
                                int64_t nodes, double rtol, int max_it, double* vec,
                                double* parts, double* scal, hipStream_t s, int* iters_out,
                                double* relres_out) {
  const unsigned nblk = (unsigned)((nodes + NTS - 1) / NTS);
  const dim3 g(nblk, (unsigned)q);
  hipLaunchKernelGGL(k_skel_fill, g, dim3(NTS), 0, s, dprob, items, sub_item, store, m, vec);
#define MLC_SKEL(K, ...)                                                                  \
  do {                                                                                    \
    if (kind == 0)                                                                        \
      hipLaunchKernelGGL(K<0>, g, dim3(NTS), 0, s, __VA_ARGS__);                          \
    else if (kind == 1)                                                                   \
      hipLaunchKernelGGL(K<1>, g, dim3(NTS), 0, s, __VA_ARGS__);                          \
    else if (kind == 2)                                                                   \
      hipLaunchKernelGGL(K<2>, g, dim3(NTS), 0, s, __VA_ARGS__);                          \
    else                                                                                  \
      hipLaunchKernelGGL(K<3>, g, dim3(NTS), 0, s, __VA_ARGS__);                          \
  } while (0)
  MLC_SKEL(k_skel_init, dprob, m, vec, parts);
  hipLaunchKernelGGL(k_skel_reduce, dim3(q), dim3(1024), 0, s, parts, (int)nblk, 0, rtol, scal);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double h[SKEL_NS * MLC_MAX_Q];
  int it = 0;
  while (it < max_it) {
    // sixteen iterations between polls of the convergence flags
    for (int k = 0; k < 16 && it < max_it; ++k, ++it) {
      const int po = it & 1;  // the two direction buffers alternate
      MLC_SKEL(k_skel_dir, dprob, m, vec, po, scal, it == 0 ? 1 : 0, parts);
      hipLaunchKernelGGL(k_skel_reduce, dim3(q), dim3(1024), 0, s, parts, (int)nblk, 1, rtol, scal);
      MLC_SKEL(k_skel_upd, dprob, m, vec, 1 - po, scal, parts);
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
  hipLaunchKernelGGL(k_skel_finish, g, dim3(NTS), 0, s, dprob, m, vec);
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
