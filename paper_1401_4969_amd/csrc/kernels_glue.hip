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
// node, a few launches per iteration, scalars kept in device memory (no host round trip
// per iteration), block partial sums reduced in a fixed order (deterministic).
#include "mlc_launch.h"

namespace {

constexpr int NTS = 256;

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
                                                   int m, int i_rhs, double* E) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1, r = 1 << m;
  const int64_t idx = (int64_t)blockIdx.x * NTS + threadIdx.x;
  if (idx >= (int64_t)n1 * n1) return;
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
__global__ __launch_bounds__(NTS) void k_skel_init(const ProbDev* probs, int m, int i_rhs,
                                                   const double* E, double* Wv, double* Z,
                                                   double* Pv, double* parts) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1, r = 1 << m;
  const int64_t nn = (int64_t)n1 * n1;
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
__global__ __launch_bounds__(NTS) void k_skel_dir(const ProbDev* probs, int m, const double* Z,
                                                  const double* Po, double* Pn, double* Q,
                                                  const double* scal, int first,
                                                  double* parts) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1, r = 1 << m;
  const int64_t nn = (int64_t)n1 * n1;
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
__global__ __launch_bounds__(NTS) void k_skel_upd(const ProbDev* probs, int m, double* E,
                                                  double* Wv, double* Z, const double* Pv,
                                                  const double* Q, const double* scal,
                                                  double* parts) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1, r = 1 << m;
  const int64_t nn = (int64_t)n1 * n1;
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

// Fixed-order sum of the block partials, then the CG scalars in scal:
//   stage 0 (after init):  scal[0] = rho = w.z, scal[3] = ||w||^2, scal[4] = ||w_0||^2
//   stage 1 (after dir):   scal[1] = alpha = rho / p.q
//   stage 2 (after upd):   scal[2] = beta = (w.z) / rho, scal[0] = w.z, scal[3] = ||w||^2
__global__ __launch_bounds__(1024) void k_skel_reduce(const double* parts, int nblk, int stage,
                                                      double* scal) {
  __shared__ double red[2 * 16];
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
    } else if (stage == 1) {
      scal[1] = sa != 0.0 ? scal[0] / sa : 0.0;
    } else {
      scal[2] = scal[0] != 0.0 ? sa / scal[0] : 0.0;
      scal[0] = sa;
      scal[3] = sb;
    }
  }
}

// u~ = I u + e for right-hand side i (0 off the domain).
__global__ __launch_bounds__(NTS) void k_skel_finish(const ProbDev* probs, int m, int i_rhs,
                                                     const double* E) {
  const ProbDev& P = probs[0];
  const int N = P.n_c << m, n1 = N + 1;
  const int64_t nn = (int64_t)n1 * n1;
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
  double* E = vec;
  double* Wv = vec + nodes;
  double* Z = vec + 2 * nodes;
  double* Pa = vec + 3 * nodes;
  double* Pb = vec + 4 * nodes;
  double* Q = vec + 5 * nodes;
  int it_max = 0;
  double rel_max = 0.0;
  for (int i = 0; i < q; ++i) {
    hipLaunchKernelGGL(k_skel_fill, dim3(nblk), dim3(NTS), 0, s, dprob, items, sub_item, store,
                       m, i, E);
    if (kind == 0)
      hipLaunchKernelGGL(k_skel_init<0>, dim3(nblk), dim3(NTS), 0, s, dprob, m, i, E, Wv, Z, Pa, parts);
    else if (kind == 1)
      hipLaunchKernelGGL(k_skel_init<1>, dim3(nblk), dim3(NTS), 0, s, dprob, m, i, E, Wv, Z, Pa, parts);
    else if (kind == 2)
      hipLaunchKernelGGL(k_skel_init<2>, dim3(nblk), dim3(NTS), 0, s, dprob, m, i, E, Wv, Z, Pa, parts);
    else
      hipLaunchKernelGGL(k_skel_init<3>, dim3(nblk), dim3(NTS), 0, s, dprob, m, i, E, Wv, Z, Pa, parts);
    hipLaunchKernelGGL(k_skel_reduce, dim3(1), dim3(1024), 0, s, parts, (int)nblk, 0, scal);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double h[5];
    if ((e = hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    const double rr0 = h[4];
    double rr = rr0;
    int it = 0;
    double* Po = Pa;
    double* Pn = Pb;
    if (rr0 > 0.0) {
      const double tol2 = rtol * rtol * rr0;
      while (it < max_it) {
        // eight iterations between convergence checks
        for (int k = 0; k < 8 && it < max_it; ++k, ++it) {
          const int first = it == 0 ? 1 : 0;
          if (kind == 0)
            hipLaunchKernelGGL(k_skel_dir<0>, dim3(nblk), dim3(NTS), 0, s, dprob, m, Z, Po, Pn, Q, scal, first, parts);
          else if (kind == 1)
            hipLaunchKernelGGL(k_skel_dir<1>, dim3(nblk), dim3(NTS), 0, s, dprob, m, Z, Po, Pn, Q, scal, first, parts);
          else if (kind == 2)
            hipLaunchKernelGGL(k_skel_dir<2>, dim3(nblk), dim3(NTS), 0, s, dprob, m, Z, Po, Pn, Q, scal, first, parts);
          else
            hipLaunchKernelGGL(k_skel_dir<3>, dim3(nblk), dim3(NTS), 0, s, dprob, m, Z, Po, Pn, Q, scal, first, parts);
          hipLaunchKernelGGL(k_skel_reduce, dim3(1), dim3(1024), 0, s, parts, (int)nblk, 1, scal);
          if (kind == 0)
            hipLaunchKernelGGL(k_skel_upd<0>, dim3(nblk), dim3(NTS), 0, s, dprob, m, E, Wv, Z, Pn, Q, scal, parts);
          else if (kind == 1)
            hipLaunchKernelGGL(k_skel_upd<1>, dim3(nblk), dim3(NTS), 0, s, dprob, m, E, Wv, Z, Pn, Q, scal, parts);
          else if (kind == 2)
            hipLaunchKernelGGL(k_skel_upd<2>, dim3(nblk), dim3(NTS), 0, s, dprob, m, E, Wv, Z, Pn, Q, scal, parts);
          else
            hipLaunchKernelGGL(k_skel_upd<3>, dim3(nblk), dim3(NTS), 0, s, dprob, m, E, Wv, Z, Pn, Q, scal, parts);
          hipLaunchKernelGGL(k_skel_reduce, dim3(1), dim3(1024), 0, s, parts, (int)nblk, 2, scal);
          double* t = Po;
          Po = Pn;
          Pn = t;
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, s)) != hipSuccess)
          return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        rr = h[3];
        if (rr <= tol2) break;
      }
    }
    hipLaunchKernelGGL(k_skel_finish, dim3(nblk), dim3(NTS), 0, s, dprob, m, i, E);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    it_max = it > it_max ? it : it_max;
    const double rel = rr0 > 0.0 ? sqrt(rr / rr0) : 0.0;
    rel_max = rel > rel_max ? rel : rel_max;
  }
  *iters_out = it_max;
  *relres_out = rel_max;
  return hipSuccess;
}
