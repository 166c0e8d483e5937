// Batched local solves of Algorithm 4.1 step 1, equation (Aux_Problem), in FP64:
//   for every subdomain Omega_j and every eigenpair i, find e in V_0h(Omega_j) with
//   a(e, v) = lambda_i b(u_i, v) - a(u_i, v) for all v in V_0h(Omega_j),
// i.e. K_j e = r|_{T_j} with homogeneous Dirichlet data on the boundary of Omega_j.
//
// One workgroup owns one (subdomain, eigenpair) item and runs the whole preconditioned
// conjugate gradient to convergence with workgroup barriers only: the items are
// independent, so no grid-wide synchronisation is needed and the hardware dispatcher
// acts as the work queue (items are ordered largest first).  The preconditioner is a
// symmetric multigrid V-cycle over the nested grids of the tile (nu Jacobi sweeps, with
// the two Chebyshev weights for nu = 2, before and after each coarse correction, restriction P^T, interpolation P, Galerkin
// coarse operators = the same stencil with children-mean kappa, exact solve on the
// coarse-cell grid of Omega_j), so the work per item is O(tile size) (the multigrid remark
// after the work estimate of Section 5).
#include "pcg_ops.h"

namespace {

template <int NT, int KIND>
__global__ __launch_bounds__(NT) void k_local_pcg64(const ProbDev* probs, const TileItem* items,
                                                     char* store, const double* inv, int m,
                                                     ItemStat* stats, double rtol, int max_it,
                                                     int nu, double omega, double omega2,
                                                     int rhs_in_tile,
                                                     int ring_cap, int ring_cap2, int ring_cap2n) {
  __shared__ double red[2 * (NT / 64)];
  extern __shared__ double ring_lds[];  // banded smoothing rings (dynamic size)
  const TileItem it = items[blockIdx.x];
  const ProbDev& P = probs[it.prob];
  const Levels lev(it, P, m, 2);
  double* base = reinterpret_cast<double*>(store + it.off);
  const LevelDesc l0 = lev[0];
  double* X = base;
  double* R = base + l0.ob;
  const int n1 = l0.N + 1;
  const double* bglob = P.res + (int64_t)it.rhs * n1 * n1;
  double acc[2] = {0.0, 0.0};
  FOR_TILE(l0) {
    const unsigned i = (unsigned)(iy * l0.nx + ix);
    // right-hand side: the global residual window, or (adjoint solves) already in R; x is
    // cleared only where the first update reads it
    const double v = rhs_in_tile ? R[i] : bglob[(int64_t)(l0.gy0 + iy) * n1 + (l0.gx0 + ix)];
    R[i] = v;
    if constexpr (!SKIP_X0<double, KIND>) X[i] = 0.0;
    acc[0] += v * v;
  }
  block_sum<NT, 2>(acc, red);
  const double bb = acc[0];
  double rr = bb;
  // banded passes when this tile's rows fit the rings (a per-item decision, so the
  // arithmetic of an item does not depend on the other items of the launch)
  // band rows per wave: two where this tile's rows fit the taller rings, else one; tiles
  // too wide for the taller rings beside the LDS V-cycle tail but narrow enough without
  // it (ring_cap2 < nx <= ring_cap2n) give the tail up for them
  const bool tall_no_tail = l0.nx > ring_cap2 && l0.nx <= ring_cap2n;
  const int rows = (l0.nx <= ring_cap2 || tall_no_tail) ? 2 : (l0.nx <= ring_cap ? 1 : 0);
  double* ring = rows ? ring_lds : nullptr;
  // the LDS V-cycle tail, after the rings, with 1024-thread workgroups (one per CU: the
  // extra LDS costs no concurrency there)
  double* tail = (rows && NT == 1024 && !tall_no_tail)
                     ? ring_lds + ring_elems(NT / 64, ring_cap, ring_cap2)
                     : nullptr;
  const int iters = pcg_solve<NT, KIND, double, 2>(P, lev, base, m, inv + it.inv_off, bb,
                                                rtol * rtol * bb, max_it, nu, omega, omega2, red, ring,
                                                rows, tail, rr);
  if (threadIdx.x == 0) {
    ItemStat s;
    s.iters = iters;
    s.refine = 0;
    s.relres = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    stats[blockIdx.x] = s;
    if (!rhs_in_tile)  // forward solves: the step's largest relative residual
      atomicMax(reinterpret_cast<unsigned long long*>(P.conv + m),
                (unsigned long long)__double_as_longlong(s.relres));
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

int ring_capacity(int nt, int nu, int max_tile_nx, int elem_bytes, bool with_tail, size_t* lds,
                  int* cap2) {
  static int limit = -1;
  if (limit < 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      v = 0;
    limit = v;
  }
  *lds = 0;
  *cap2 = 0;
  if (nu != 2) return 0;
  // three rings of B + 2 rows (B = nt/64 rows per band step, or twice that) and the LDS
  // V-cycle tail; keep room for the reduction buffer and the compiler's own LDS.  The
  // caps depend on the device only, unless every tile is narrower.
  const int nw = nt / 64;
  const long row1 = 3L * (nw + 2) * elem_bytes, row2 = 3L * (2 * nw + 2) * elem_bytes;
  const long tail = with_tail ? (long)TAIL_ELEMS * elem_bytes : 0L;
  const long room = limit - 4096L - tail;
  const long fit1 = room / row1, fit2 = room / row2;
  const int cap1 = (int)(fit1 < max_tile_nx ? fit1 : max_tile_nx);
  if (cap1 < 1) return 0;
  *cap2 = (int)(fit2 < max_tile_nx ? fit2 : max_tile_nx);
  *lds = (size_t)ring_elems(nw, cap1, *cap2) * elem_bytes + tail;
  return cap1;
}

int ring_layout(int nt, int nu, int max_tile_nx, int elem_bytes, size_t* lds, int* cap2,
                int* cap2n) {
  const bool tail = nt == 1024;
  const int cap = ring_capacity(nt, nu, max_tile_nx, elem_bytes, tail, lds, cap2);
  *cap2n = 0;
  if (tail && cap > 0 && *cap2 < max_tile_nx) {
    size_t lds_n = 0;
    int c2n = 0;
    ring_capacity(nt, nu, max_tile_nx, elem_bytes, false, &lds_n, &c2n);
    if (c2n > *cap2) {
      *cap2n = c2n;
      *lds = std::max(*lds, lds_n);
    }
  }
  return cap;
}

hipError_t launch_local_pcg(int kind, int nt, const ProbDev* probs, const TileItem* items,
                            int nitems, char* store, const double* inv, int m, ItemStat* stats,
                            double rtol, int max_it, int nu, double omega, double omega2,
                            int64_t rhs_in_tile,
                            int max_tile_nx, hipStream_t s) {
  // the ring is sized for the workgroup size actually launched
  const int ntv = nt == 256 ? 256 : (nt == 512 ? 512 : 1024);
  size_t lds = 0;
  int cap2 = 0, cap2n = 0;
  const int cap = ring_layout(ntv, nu, max_tile_nx, 8, &lds, &cap2, &cap2n);
  // a constant coefficient keeps one band row with the tail: its one-row passes prefetch
  // the next band's rows (config 3's 191-wide tiles: 6% slower on two rows without tail)
  if (kind == 0) cap2n = 0;
#define MLC_PCG(NTV, KV)                                                                        \
  hipLaunchKernelGGL((k_local_pcg64<NTV, KV>), dim3(nitems), dim3(NTV), lds, s, probs, items,    \
                     store, inv, m, stats, rtol, max_it, nu, omega, omega2, (int)rhs_in_tile,   \
                     cap, cap2, cap2n)
#define MLC_PCG_NT(NTV)    \
  if (kind == 0)           \
    MLC_PCG(NTV, 0);       \
  else if (kind == 1)      \
    MLC_PCG(NTV, 1);       \
  else if (kind == 2)      \
    MLC_PCG(NTV, 2);       \
  else                     \
    MLC_PCG(NTV, 3);
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
