// Mixed-precision local solves of Algorithm 4.1 step 1 (equation (Aux_Problem)):
// FP32 preconditioned conjugate gradients with the FP32 V-cycle, wrapped in FP64
// iterative refinement.  The correction e and the residual b - K e stay in FP64:
//   e = 0; repeat { r = b - K e (FP64 stencil); stop when ||r|| <= rtol ||b||;
//                   solve K d = r in FP32 to inner_rtol; e += d (FP64) }.
// Only the inner iterations run in FP32, so they stream half the bytes of the FP64
// solver; the accuracy of e is that of the FP64 residual.
#include "pcg_ops.h"

namespace {

// One band row per wave: taller bands' registers would crowd out the prefetching passes.
constexpr int MIXED_MAX_ROWS = 1;

// e += d (e = d on the first refinement: e is not cleared beforehand, nor read then) and
// the FP64 residual r = b - K e of the updated correction in one banded pass:
// the workgroup walks the tile in bands of NW rows with an LDS ring of NW + 2 FP64 rows
// of e (rows -1 and ny zero, the Dirichlet values).  At step k wave w forms row
// k NW + w - 1 of e + d (stored), and after a barrier the residual of the row above it
// from the ring, stored in FP32 as the next inner solve's right-hand side with that
// solve's iterate cleared; acc receives this thread's share of ||r||^2.  A ring row is
// overwritten only after the barrier that follows its last reader.  Rows of at most
// RING_CHUNKS * 64 nodes.
template <int NT, int KIND>
__device__ void refine_banded(const ProbDev& P, const LevelDesc& l0, double* E, float* X,
                              float* R, const double* bglob, int n1, bool first, double* ring,
                              double* acc) {
  constexpr int NW = NT / 64, RING = NW + 2, CM = RING_CHUNKS;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nx = l0.nx, ny = l0.ny, nch = (nx + 63) >> 6;
  auto row = [&](int y) -> double* { return ring + ((y + 1) % RING) * nx; };
  for (int k = 0; k * NW - 2 < ny; ++k) {
    const int ya = k * NW + w - 1, yb = ya - 1;
    const bool inA = ya >= 0 && ya < ny, inB = yb >= 0 && yb < ny;
    double ev[CM], bv[CM];
    float xv[CM];
#pragma unroll
    for (int c = 0; c < CM; ++c) {
      if (c < nch) {
        const int ix = lane + 64 * c;
        const unsigned i = (inA && ix < nx) ? (unsigned)(ya * nx + ix) : 0u;
        ev[c] = first ? 0.0 : E[i];  // e_0 = 0 is not read
        xv[c] = X[i];
        // b of the row the second stage takes (a node of the tile's first row otherwise)
        const int bx = ix < nx ? ix : nx - 1, by = inB ? yb : 0;
        bv[c] = bglob[(int64_t)(l0.gy0 + by) * n1 + (l0.gx0 + bx)];
      }
    }
    if (ya >= -1 && ya <= ny) {
      double* dst = row(ya);
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        const int ix = lane + 64 * c;
        if (c < nch && ix < nx) {
          double v = 0.0;
          if (inA) {
            v = ev[c] + (double)xv[c];
            E[(unsigned)(ya * nx + ix)] = v;
          }
          dst[ix] = v;
        }
      }
    }
    __syncthreads();
    if (inB) {
      const double* rs = row(yb - 1);
      const double* rc = row(yb);
      const double* rn = row(yb + 1);
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        const int ix = lane + 64 * c;
        if (c < nch && ix < nx) {
          double r = 0.0;
          if (is_dof(P.domain, l0.N, l0.gx0 + ix, l0.gy0 + yb)) {
            double d;
            r = bv[c] - apply_rows<KIND, double>(P, l0, rs, rc, rn, ix, yb, d);
          }
          const unsigned i = (unsigned)(yb * nx + ix);
          R[i] = (float)r;
          X[i] = 0.0f;
          *acc += r * r;
        }
      }
    }
    __syncthreads();
  }
}

template <int NT, int KIND>
__global__ __launch_bounds__(NT) void k_local_mixed(const ProbDev* probs, const TileItem* items,
                                                    char* store, const double* inv, int m,
                                                    ItemStat* stats, double rtol, int max_it,
                                                    int max_refine, double inner_rtol, int nu,
                                                    double omega, double omega2, int ring_cap,
                                                    int ring_cap2) {
  __shared__ double red[2 * (NT / 64)];
  extern __shared__ float ring_lds_f[];  // banded smoothing rings (dynamic size)
  const TileItem it = items[blockIdx.x];
  const ProbDev& P = probs[it.prob];
  const Levels lev(it, P, m, 2);
  const LevelDesc l0 = lev[0];
  const int64_t S0 = (int64_t)l0.nx * l0.ny;
  double* E = reinterpret_cast<double*>(store + it.off);      // FP64 correction, read by the gluing
  float* base = reinterpret_cast<float*>(store + it.off + 8 * S0);
  float* X = base;
  float* R = base + l0.ob;
  const double* Kinv = inv + it.inv_off;
  const int n1 = l0.N + 1;
  const double* bglob = P.res + (int64_t)it.rhs * n1 * n1;
  auto bat = [&](int ix, int iy) -> double {
    return bglob[(int64_t)(l0.gy0 + iy) * n1 + (l0.gx0 + ix)];
  };
  double acc[2] = {0.0, 0.0};
  FOR_TILE(l0) {
    const unsigned i = (unsigned)(iy * l0.nx + ix);
    const double v = bat(ix, iy);
    R[i] = (float)v;  // e is written by the first refinement, without being read
    X[i] = 0.0f;
    acc[0] += v * v;
  }
  block_sum<NT, 2>(acc, red);
  const double bb = acc[0];
  double rr = bb;
  int total = 0, refine = 0;
  const int rows = l0.nx <= ring_cap ? 1 : 0;  // banded passes where the rings fit (per item)
  float* ring = rows ? ring_lds_f : nullptr;
  // the LDS V-cycle tail with 1024-thread workgroups (one per CU), as in the FP64 solver
  float* tail = (rows && NT == 1024) ? ring_lds_f + ring_elems(NT / 64, ring_cap, 0) : nullptr;
  // at least one refinement, which writes e (with a zero right-hand side it adds x = 0)
  do {
    ++refine;
    double rr_inner;
    total += pcg_solve<NT, KIND, float, MIXED_MAX_ROWS>(P, lev, base, m, Kinv, rr, inner_rtol * inner_rtol * rr,
                                        max_it, nu, omega, omega2, red, ring, rows, tail,
                                        rr_inner);
    acc[0] = acc[1] = 0.0;
    if (rows && l0.nx <= 64 * RING_CHUNKS) {
      // the ring space (three FP32 rings) holds the one FP64 ring of this pass
      refine_banded<NT, KIND>(P, l0, E, X, R, bglob, n1, refine == 1,
                              reinterpret_cast<double*>(ring_lds_f), &acc[0]);
      block_sum<NT, 2>(acc, red);
      rr = acc[0];
      continue;
    }
    FOR_TILE(l0) {
      const unsigned i = (unsigned)(iy * l0.nx + ix);
      E[i] = (refine == 1 ? 0.0 : E[i]) + (double)X[i];
    }
    __syncthreads();
    // FP64 residual of the accumulated correction, handed to the next FP32 solve
    FOR_TILE(l0) {
      const unsigned i = (unsigned)(iy * l0.nx + ix);
      double r = 0.0;
      if (is_dof(P.domain, l0.N, l0.gx0 + ix, l0.gy0 + iy)) {
        double d;
        r = bat(ix, iy) - stencil<KIND, double>(P, l0, E, ix, iy, i, d);
      }
      R[i] = (float)r;
      X[i] = 0.0f;
      acc[0] += r * r;
    }
    block_sum<NT, 2>(acc, red);
    rr = acc[0];
  } while (rr > rtol * rtol * bb && refine < max_refine);
  if (threadIdx.x == 0) {
    ItemStat s;
    s.iters = total;
    s.refine = refine;
    s.relres = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    stats[blockIdx.x] = s;
    atomicMax(reinterpret_cast<unsigned long long*>(P.conv + m),
              (unsigned long long)__double_as_longlong(s.relres));
  }
}

}  // namespace

// Storage (bytes) of one item at level m: the FP64 correction, then the FP32 tile buffers
// (X, R, Z, Tmp, P, Q on the tile level and B, Z, Tmp on every coarser level).
int64_t item_bytes_mixed(int cw, int ch, int m) {
  int64_t fl = 0, S0 = 0;
  for (int t = 0; t <= m; ++t) {
    const int r = 1 << (m - t);
    const int64_t S = (int64_t)(cw * r - 1) * (ch * r - 1);
    if (t == 0) S0 = S;
    fl += (t == 0 ? 6 : 3) * S;
  }
  return 8 * S0 + ((4 * fl + 7) / 8) * 8;
}

hipError_t launch_local_mixed(int kind, int nt, const ProbDev* probs, const TileItem* items,
                              int nitems, char* store, const double* inv, int m, ItemStat* stats,
                              double rtol, int max_it, int max_refine, double inner_rtol, int nu,
                              double omega, double omega2, int max_tile_nx, hipStream_t s) {
  // the ring is sized for the workgroup size actually launched
  const int ntv = nt == 256 ? 256 : (nt == 512 ? 512 : 1024);
  size_t lds = 0;
  int cap2 = 0;
  const int cap = ring_capacity(ntv, nu, max_tile_nx, 4, ntv == 1024, &lds, &cap2);
  cap2 = 0;  // one band row per wave here
  lds = cap > 0 ? (size_t)ring_elems(ntv / 64, cap, 0) * 4 + (ntv == 1024 ? (size_t)TAIL_ELEMS * 4 : 0) : 0;
#define MLC_MIX(NTV, KV)                                                                     \
  hipLaunchKernelGGL((k_local_mixed<NTV, KV>), dim3(nitems), dim3(NTV), lds, s, probs, items, \
                     store, inv, m, stats, rtol, max_it, max_refine, inner_rtol, nu, omega,   \
                     omega2, cap, cap2)
#define MLC_MIX_NT(NTV) \
  if (kind == 0)        \
    MLC_MIX(NTV, 0);    \
  else if (kind == 1)   \
    MLC_MIX(NTV, 1);    \
  else if (kind == 2)   \
    MLC_MIX(NTV, 2);    \
  else                  \
    MLC_MIX(NTV, 3);
  if (nt == 256) {
    MLC_MIX_NT(256)
  } else if (nt == 512) {
    MLC_MIX_NT(512)
  } else {
    MLC_MIX_NT(1024)
  }
#undef MLC_MIX_NT
#undef MLC_MIX
  return hipGetLastError();
}
