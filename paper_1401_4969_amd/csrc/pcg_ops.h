// Device building blocks of the batched local solves (Algorithm 4.1 step 1): tile
// level descriptors, the symmetric multigrid V-cycle and the preconditioned conjugate
// gradient loop, templated on the vector type of the tile buffers (double, or float for
// the mixed-precision solver).  Included by the FP64 and the mixed-precision kernels.
//
// Vectors of an item live in its slice of the workspace, row-major over the tile's
// interior nodes (no halo: outside the tile is the Dirichlet boundary, read as 0).
// Waves sweep rows, 64 consecutive nodes per wave, so every access is coalesced.
//
// The tile vectors do not fit in cache (hundreds of items are live at once), so every
// pass streams from HBM; passes are merged where that removes a whole vector read or
// write without a second copy of any vector:
//   - the first two Jacobi sweeps from a zero iterate are one pass over b;
//   - r.z is accumulated in the last post-smoothing sweep on the tile level;
//   - the direction update p = z + beta p and A p are one pass (A p is not stored:
//     the x/r update applies the stencil to p again).
#pragma once
#include "mlc_launch.h"

namespace {

struct LevelDesc {
  int nx, ny, gx0, gy0, N, l;
  int64_t ob, oz, ot;  // element offsets of right-hand side, iterate, temporary
};

// Tile indices are 32-bit (the finest grid has at most 32768 cells per side, so a tile
// has fewer than 2^30 nodes): with a uniform vector base the loads take a scalar base
// and a 32-bit vector offset instead of a 64-bit address per lane.
#define FOR_TILE(lv)                                                  \
  for (int iy = threadIdx.x >> 6; iy < (lv).ny; iy += NT / 64)       \
    for (int ix = threadIdx.x & 63; ix < (lv).nx; ix += 64)

// Every load of a sweep is issued unconditionally, from an index clamped into the tile
// (the node itself stands in for a neighbour off the tile), and the value is then
// selected: a load behind a branch would be waited for inside that branch, so a stencil
// would cost several memory round trips instead of one.
template <int KIND, typename T>
__device__ __forceinline__ T stencil(const ProbDev& P, const LevelDesc& lv, const T* u, int ix,
                                     int iy, unsigned i, T& diag) {
  const Weights W = edge_weights<KIND, T>(P, lv.l, lv.N, lv.gx0 + ix, lv.gy0 + iy);
  const bool he = ix + 1 < lv.nx, hw = ix > 0, hn = iy + 1 < lv.ny, hs = iy > 0;
  const T c = u[i];
  const T e0 = u[he ? i + 1 : i];
  const T w0 = u[hw ? i - 1 : i];
  const T n0 = u[hn ? i + lv.nx : i];
  const T s0 = u[hs ? i - lv.nx : i];
  const T e = he ? e0 : T(0), w = hw ? w0 : T(0), n = hn ? n0 : T(0), s = hs ? s0 : T(0);
  T ne = T(0), sw = T(0);
  if constexpr (KIND == 3) {  // the hypotenuse neighbours
    const bool hne = he && hn, hsw = hw && hs;
    const T ne0 = u[hne ? i + lv.nx + 1 : i];
    const T sw0 = u[hsw ? i - lv.nx - 1 : i];
    ne = hne ? ne0 : T(0);
    sw = hsw ? sw0 : T(0);
  }
  return apply_k<KIND, T>(W, c, e, w, n, s, ne, sw, diag);
}

// z = omega D^-1 b (first sweep from a zero iterate)
template <int NT, int KIND, typename T>
__device__ void op_first(const ProbDev& P, const LevelDesc& lv, const T* b, T* z, T omega) {
  FOR_TILE(lv) {
    const unsigned i = (unsigned)(iy * lv.nx + ix);
    T v = T(0);
    if (is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + iy)) {
      const Weights W = edge_weights<KIND, T>(P, lv.l, lv.N, lv.gx0 + ix, lv.gy0 + iy);
      v = omega * b[i] / T(diag_of<KIND>(W));
    }
    z[i] = v;
  }
}

// z = two damped-Jacobi sweeps from a zero iterate in one pass:
//   z1 = omega D^-1 b,  z = z1 + omega D^-1 (b - A z1),
// with z1 formed on the fly at the node and its four neighbours (zero off the tile and
// on nodes outside the domain, where b is zero and the diagonal need not exist).
template <int KIND, typename T>
__device__ __forceinline__ double diag_at(const ProbDev& P, const LevelDesc& lv, int ix, int iy) {
  const Weights W = edge_weights<KIND, T>(P, lv.l, lv.N, lv.gx0 + ix, lv.gy0 + iy);
  return diag_of<KIND>(W);
}

template <int NT, int KIND, typename T>
__device__ void op_first2(const ProbDev& P, const LevelDesc& lv, const T* b, T* z, T omega,
                          T omega2) {
  FOR_TILE(lv) {
    const unsigned i = (unsigned)(iy * lv.nx + ix);
    // first-sweep value at tile node (jx, jy) = index j, zero when `in` is false
    auto z1 = [&](bool in, int jx, int jy, unsigned j) -> T {
      const T bj = b[in ? j : i];
      const T dj = T(diag_at<KIND, T>(P, lv, in ? jx : ix, in ? jy : iy));
      const bool ok = in && is_dof(P.domain, lv.N, lv.gx0 + jx, lv.gy0 + jy);
      return ok ? omega * bj / dj : T(0);
    };
    const Weights W = edge_weights<KIND, T>(P, lv.l, lv.N, lv.gx0 + ix, lv.gy0 + iy);
    const T we = T(W.e), ww = T(W.w), wn = T(W.n), ws = T(W.s);
    T d;
    if constexpr (KIND == 3)
      d = we + ww + wn + ws + T(W.ne) + T(W.sw);
    else
      d = we + ww + wn + ws;
    const T bc = b[i];
    const T zc = omega * bc / d;
    const T ze = z1(ix + 1 < lv.nx, ix + 1, iy, i + 1);
    const T zw = z1(ix > 0, ix - 1, iy, i - 1);
    const T zn = z1(iy + 1 < lv.ny, ix, iy + 1, i + lv.nx);
    const T zs = z1(iy > 0, ix, iy - 1, i - lv.nx);
    T zne = T(0), zsw = T(0);
    if constexpr (KIND == 3) {
      zne = z1(ix + 1 < lv.nx && iy + 1 < lv.ny, ix + 1, iy + 1, i + lv.nx + 1);
      zsw = z1(ix > 0 && iy > 0, ix - 1, iy - 1, i - lv.nx - 1);
    }
    T dd;
    const T az = apply_k<KIND, T>(W, zc, ze, zw, zn, zs, zne, zsw, dd);
    const T v = zc + omega2 * (bc - az) / d;
    z[i] = is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + iy) ? v : T(0);
  }
}

// zo = zi + omega D^-1 (b - A zi); with DOT, also acc += b . zo
template <int NT, int KIND, typename T, bool DOT = false>
__device__ void op_jacobi(const ProbDev& P, const LevelDesc& lv, const T* b, const T* zi, T* zo,
                          T omega, double* acc = nullptr) {
  FOR_TILE(lv) {
    const unsigned i = (unsigned)(iy * lv.nx + ix);
    T v = T(0);
    if (is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + iy)) {
      T d;
      const T az = stencil<KIND, T>(P, lv, zi, ix, iy, i, d);
      const T bi = b[i];
      v = zi[i] + omega * (bi - az) / d;
      if (DOT) *acc += (double)bi * (double)v;
    }
    zo[i] = v;
  }
}

// ro = b - A z
template <int NT, int KIND, typename T>
__device__ void op_residual(const ProbDev& P, const LevelDesc& lv, const T* b, const T* z, T* ro) {
  FOR_TILE(lv) {
    const unsigned i = (unsigned)(iy * lv.nx + ix);
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
    const unsigned i = (unsigned)(iy * lc.nx + ix);
    T v = T(0);
    if (is_dof(P.domain, lc.N, lc.gx0 + ix, lc.gy0 + iy)) {
      const unsigned c = (unsigned)((2 * iy + 1) * nf + (2 * ix + 1));
      v = rf[c] + T(0.5) * (rf[c + 1] + rf[c - 1] + rf[c + nf] + rf[c - nf] + rf[c + nf + 1] +
                            rf[c - nf - 1]);
    }
    bc[i] = v;
  }
}

// zf += P zc (P1 interpolation on the SW-NE mesh; coarse nodes outside the tile are 0).
// Odd tile indices are even global indices, i.e. coarse nodes.  Every fine node takes
// half the sum of two coarse values: the same node twice (odd, odd), the W-E pair (even,
// odd), the S-N pair (odd, even) or the SW-NE pair (even, even).
template <int NT, typename T>
__device__ void op_prolong_add(const ProbDev& P, const LevelDesc& lc, const LevelDesc& lf,
                               const T* zc, T* zf) {
  const int ncx = lc.nx, ncy = lc.ny;
  auto at = [&](int cx, int cy) -> T {
    const bool in = cx >= 0 && cy >= 0 && cx < ncx && cy < ncy;
    const T v = zc[in ? (unsigned)(cy * ncx + cx) : 0u];
    return in ? v : T(0);
  };
  FOR_TILE(lf) {
    const unsigned i = (unsigned)(iy * lf.nx + ix);
    const int cx = ix >> 1, cy = iy >> 1;
    const int ax = cx - ((ix & 1) ^ 1), ay = cy - ((iy & 1) ^ 1);
    const T v = T(0.5) * (at(ax, ay) + at(cx, cy));
    const T old = zf[i];
    zf[i] = is_dof(P.domain, lf.N, lf.gx0 + ix, lf.gy0 + iy) ? old + v : old;
  }
}

// One damped-Jacobi update at tile node (ix, y) from three consecutive rows held in LDS
// (rows -1 and ny are stored as zeros, the Dirichlet values).
template <int KIND, typename T>
__device__ __forceinline__ T apply_rows(const ProbDev& P, const LevelDesc& lv, const T* rs,
                                        const T* rc, const T* rn, int ix, int y, T& d) {
  const Weights W = edge_weights<KIND, T>(P, lv.l, lv.N, lv.gx0 + ix, lv.gy0 + y);
  const bool he = ix + 1 < lv.nx, hw = ix > 0;
  const T c = rc[ix];
  const T e0 = rc[he ? ix + 1 : ix], w0 = rc[hw ? ix - 1 : ix];
  const T e = he ? e0 : T(0), w = hw ? w0 : T(0), n = rn[ix], s = rs[ix];
  T ne = T(0), sw = T(0);
  if constexpr (KIND == 3) {  // hypotenuse neighbours: the rows above and below hold zeros
    const T ne0 = rn[he ? ix + 1 : ix], sw0 = rs[hw ? ix - 1 : ix];  // off the tile
    ne = he ? ne0 : T(0);
    sw = hw ? sw0 : T(0);
  }
  return apply_k<KIND, T>(W, c, e, w, n, s, ne, sw, d);
}

template <int KIND, typename T>
__device__ __forceinline__ T jacobi_rows(const ProbDev& P, const LevelDesc& lv, const T* rs,
                                         const T* rc, const T* rn, T bi, int ix, int y, T omega) {
  T d;
  const T az = apply_rows<KIND, T>(P, lv, rs, rc, rn, ix, y, d);
  return rc[ix] + omega * (bi - az) / d;
}

// Pre-smoothing, residual and restriction of a V-cycle level with nu = 2 as one pass:
//   z = J(J(0)) (two damped-Jacobi sweeps from zero), r = b - A z, bc = P^T r.
// The workgroup walks the tile in bands of B = NW R rows (wave w owns rows w + NW r of a
// band) with three LDS rings of B + 2 rows (first sweep, second sweep, residual): at
// step k the first sweep is formed on rows k B - 1 .. k B + B - 2 (stage A), the second
// sweep one row below, also written to za (B), the residual two rows below (C), and the
// B/2 coarse rows cy = k B/2 - 2 .. are restricted from residual rows 2cy .. 2cy+2 (D).
// b is read once from HBM (the later stages hit cache); z and bc are written once,
// instead of the 6 passes of separate sweeps.  A ring row is overwritten only after the
// barrier that follows its last reader.  Taller bands (R = 2) halve the barrier
// intervals where the rings fit.
// CMP > 0 (rows of at most 64 CMP nodes): the right-hand side rows of the next band
// step's first stage are loaded into registers at the end of this step's first stage, so
// their memory latency overlaps the three later stages instead of opening the next step;
// the second and third stages' rows (cache hits) are loaded one stage ahead, at the start
// of the step and of the second stage, so each waits behind the stage before it and its
// barrier rather than after it.  (Used with a constant coefficient, in FP64 and FP32: with
// variable coefficients the extra registers measured slower.)
template <int NT, int KIND, typename T, int R, int CMP = 0>
__device__ void op_pre_fused(const ProbDev& P, const LevelDesc& lv, const LevelDesc& lc,
                             const T* b, T* za, T* bc, T omega, T omega2, T* ring) {
  constexpr int NW = NT / 64, BH = NW * R, RING = BH + 2;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nx = lv.nx, ny = lv.ny, ncx = lc.nx, ncy = lc.ny;
  T* r1 = ring;
  T* r2 = ring + RING * nx;
  T* rr = ring + 2 * RING * nx;
  auto row = [&](T* r, int y) -> T* { return r + ((y + 1) % RING) * nx; };
  constexpr int CP = CMP > 0 ? CMP : 1;
  T nb[R][CP];  // first-stage right-hand side of the coming band step (CMP > 0)
  auto load_a = [&](int kk) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int ya = kk * BH + w + NW * q - 1;
      const bool inside = ya >= 0 && ya < ny;
#pragma unroll
      for (int c = 0; c < CP; ++c) {
        const int ix = lane + 64 * c;
        nb[q][c] = b[(inside && ix < nx) ? (unsigned)(ya * nx + ix) : 0u];
      }
    }
  };
  // rows y = kk BH + w + NW q - off of b into regs (zero outside the tile)
  auto load_rows = [&](T (&regs)[R][CP], int kk, int off) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int y = kk * BH + w + NW * q - off;
      const bool inside = y >= 0 && y < ny;
#pragma unroll
      for (int c = 0; c < CP; ++c) {
        const int ix = lane + 64 * c;
        regs[q][c] = b[(inside && ix < nx) ? (unsigned)(y * nx + ix) : 0u];
      }
    }
  };
  T bb2[R][CP], bc3[R][CP];  // stage B and C right-hand sides (CMP > 0)
  if constexpr (CMP > 0) load_a(0);
  for (int k = 0; k * BH - 3 < ny || k * (BH / 2) - 2 < ncy; ++k) {
    if constexpr (CMP > 0) load_rows(bb2, k, 2);  // stage B's right-hand side, a stage ahead
    if constexpr (CMP > 0) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int ya = k * BH + w + NW * q - 1;
        if (ya >= -1 && ya <= ny) {
          T* dst = row(r1, ya);
          const bool inside = ya >= 0 && ya < ny;
#pragma unroll
          for (int c = 0; c < CP; ++c) {
            const int ix = lane + 64 * c;
            if (ix < nx) {
              T v = T(0);
              if (inside) {
                const T d = T(diag_at<KIND, T>(P, lv, ix, ya));
                v = is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + ya) ? omega * nb[q][c] / d : T(0);
              }
              dst[ix] = v;
            }
          }
        }
      }
      load_a(k + 1);
    } else {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int ya = k * BH + w + NW * q - 1;
        if (ya >= -1 && ya <= ny) {
          T* dst = row(r1, ya);
          const bool inside = ya >= 0 && ya < ny;
          for (int ix = lane; ix < nx; ix += 64) {
            T v = T(0);
            if (inside) {
              const T bi = b[(unsigned)(ya * nx + ix)];
              const T d = T(diag_at<KIND, T>(P, lv, ix, ya));
              v = is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + ya) ? omega * bi / d : T(0);
            }
            dst[ix] = v;
          }
        }
      }
    }
    __syncthreads();
    if constexpr (CMP > 0) load_rows(bc3, k, 3);  // stage C's right-hand side, one stage ahead
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int yb = k * BH + w + NW * q - 2;
      if (yb >= -1 && yb <= ny) {
        T* dst = row(r2, yb);
        if (yb >= 0 && yb < ny) {
          const T* rs = row(r1, yb - 1);
          const T* rc = row(r1, yb);
          const T* rn = row(r1, yb + 1);
          if constexpr (CMP > 0) {
#pragma unroll
            for (int c = 0; c < CP; ++c) {
              const int ix = lane + 64 * c;
              if (ix < nx) {
                const unsigned i = (unsigned)(yb * nx + ix);
                T v = jacobi_rows<KIND, T>(P, lv, rs, rc, rn, bb2[q][c], ix, yb, omega2);
                v = is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + yb) ? v : T(0);
                dst[ix] = v;
                za[i] = v;
              }
            }
          } else {
            for (int ix = lane; ix < nx; ix += 64) {
              const unsigned i = (unsigned)(yb * nx + ix);
              T v = jacobi_rows<KIND, T>(P, lv, rs, rc, rn, b[i], ix, yb, omega2);
              v = is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + yb) ? v : T(0);
              dst[ix] = v;
              za[i] = v;
            }
          }
        } else {
          for (int ix = lane; ix < nx; ix += 64) dst[ix] = T(0);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int yc = k * BH + w + NW * q - 3;
      if (yc >= -1 && yc <= ny) {
        T* dst = row(rr, yc);
        if (yc >= 0 && yc < ny) {
          const T* rs = row(r2, yc - 1);
          const T* rc = row(r2, yc);
          const T* rn = row(r2, yc + 1);
          if constexpr (CMP > 0) {
#pragma unroll
            for (int c = 0; c < CP; ++c) {
              const int ix = lane + 64 * c;
              if (ix < nx) {
                T d;
                const T v = bc3[q][c] - apply_rows<KIND, T>(P, lv, rs, rc, rn, ix, yc, d);
                dst[ix] = is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + yc) ? v : T(0);
              }
            }
          } else {
            for (int ix = lane; ix < nx; ix += 64) {
              T d;
              const T v =
                  b[(unsigned)(yc * nx + ix)] - apply_rows<KIND, T>(P, lv, rs, rc, rn, ix, yc, d);
              dst[ix] = is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + yc) ? v : T(0);
            }
          }
        } else {
          for (int ix = lane; ix < nx; ix += 64) dst[ix] = T(0);
        }
      }
    }
    __syncthreads();
    for (int j = w; j < BH / 2; j += NW) {
      const int y = k * BH - 2 + 2 * j;  // even: the top fine row 2cy + 2 of coarse row cy
      const int cy = (y - 2) / 2;
      if (cy >= 0 && cy < ncy) {
        const T* rs = row(rr, y - 2);
        const T* rc = row(rr, y - 1);
        const T* rn = row(rr, y);
        for (int cx = lane; cx < ncx; cx += 64) {
          const int x = 2 * cx + 1;
          const T v = rc[x] + T(0.5) * (rc[x + 1] + rc[x - 1] + rn[x] + rs[x] + rn[x + 1] + rs[x - 1]);
          bc[(unsigned)(cy * ncx + cx)] = is_dof(P.domain, lc.N, lc.gx0 + cx, lc.gy0 + cy) ? v : T(0);
        }
      }
    }
  }
}

// Post-smoothing of a V-cycle level with nu = 2 as one pass over the tile:
//   za <- J(J(za + P zc)),   J(z) = z + omega D^-1 (b - A z).
// Same banded walk with two LDS rings of B + 2 rows (the prolonged iterate, the first
// sweep): at step k rows k B - 1 .. of za + P zc are formed (stage A), the first sweep
// one row below (B) and the second sweep two rows below (C, written into za in place: no
// later stage reads za at or below that row).  za is read and written once and b read
// once from HBM, instead of the 8 passes of a separate interpolation and two sweeps.
// CMP > 0 (rows of at most 64 CMP nodes): the right-hand side rows of the second stage are
// loaded into registers before the first stage and those of the third at the start of the
// second, so their memory latencies overlap the stage before; the iterate rows of the
// next step's first stage are loaded at the end of this step, and the coarse rows it
// interpolates from are staged in LDS during this step.
template <int NT, int KIND, typename T, bool DOT, int R, int CMP = 0>
__device__ void op_post_fused(const ProbDev& P, const LevelDesc& lc, const LevelDesc& lv,
                              const T* zc, const T* b, T* za, T omega, T omega2, T* ring,
                              double* acc) {
  constexpr int NW = NT / 64, BH = NW * R, RING = BH + 2;
  constexpr int CP = CMP > 0 ? CMP : 1;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nx = lv.nx, ny = lv.ny;
  T* ringA = ring;
  T* ringB = ring + RING * nx;
  auto row = [&](T* r, int y) -> T* { return r + ((y + 1) % RING) * nx; };
  const int ncx = lc.nx, ncy = lc.ny;
  auto at = [&](int cx, int cy) -> T {
    const bool in = cx >= 0 && cy >= 0 && cx < ncx && cy < ncy;
    const T v = zc[in ? (unsigned)(cy * ncx + cx) : 0u];
    return in ? v : T(0);
  };
  T nz[R][CP];  // first-stage iterate rows of the coming step (CMP > 0)
  auto load_z = [&](int kk) {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int ya = kk * BH + w + NW * q - 1;
      const bool inside = ya >= 0 && ya < ny;
#pragma unroll
      for (int c = 0; c < CP; ++c) {
        const int ix = lane + 64 * c;
        nz[q][c] = za[(inside && ix < nx) ? (unsigned)(ya * nx + ix) : 0u];
      }
    }
  };
  // (CMP > 0) the coarse rows of a step's first stage, staged in LDS one step ahead in the
  // third ring's space (unused by this pass), two buffers: the loads of step kk + 1 are
  // issued at the start of step kk and written at the end of its second stage, before a
  // barrier, so the first stage reads them from LDS instead of waiting on memory
  constexpr int CBN = (NT / 64) * R / 2 + 3;  // coarse rows a step's first stage touches (max)
  constexpr int CBV = (CBN * 128 + NT - 1) / NT;  // staged values per thread, rows <= 128
  T* cbuf = ring + 2 * RING * nx;
  const int cbs = CBN * ncx;  // one buffer
  auto cb_row0 = [&](int kk) { return ((kk * BH - 1) >> 1) - 1; };
  T cv[CBV];
  auto cb_load = [&](int kk) {
    const int c0 = cb_row0(kk);
#pragma unroll
    for (int u = 0; u < CBV; ++u) {
      const int e = threadIdx.x + NT * u;
      const int j = e / ncx, cx = e - j * ncx;
      const int cy = c0 + j;
      const bool in = e < cbs && cy >= 0 && cy < ncy;
      const T v = zc[in ? (unsigned)(cy * ncx + cx) : 0u];
      cv[u] = in ? v : T(0);
    }
  };
  auto cb_store = [&](int kk) {
    T* dst = cbuf + (kk & 1) * cbs;
#pragma unroll
    for (int u = 0; u < CBV; ++u) {
      const int e = threadIdx.x + NT * u;
      if (e < cbs) dst[e] = cv[u];
    }
  };
  if constexpr (CMP > 0) {
    load_z(0);
    cb_load(0);
    cb_store(0);
    __syncthreads();
  }
  for (int k = 0; k * BH - 3 < ny; ++k) {
    if constexpr (CMP > 0) cb_load(k + 1);
    T bb[R][CP];  // second-stage right-hand side (CMP > 0)
    if constexpr (CMP > 0) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int yb = k * BH + w + NW * q - 2;
        const bool inside = yb >= 0 && yb < ny;
#pragma unroll
        for (int c = 0; c < CP; ++c) {
          const int ix = lane + 64 * c;
          bb[q][c] = b[(inside && ix < nx) ? (unsigned)(yb * nx + ix) : 0u];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int ya = k * BH + w + NW * q - 1;
      if (ya >= -1 && ya <= ny) {
        T* dst = row(ringA, ya);
        const bool inside = ya >= 0 && ya < ny;
        if constexpr (CMP > 0) {
#pragma unroll
          for (int c = 0; c < CP; ++c) {
            const int ix = lane + 64 * c;
            if (ix < nx) {
              T v = T(0);
              if (inside) {
                const int cx = ix >> 1, cy = ya >> 1;
                const int ax = cx - ((ix & 1) ^ 1), ay = cy - ((ya & 1) ^ 1);
                const T* cb = cbuf + (k & 1) * cbs;
                const int c0 = cb_row0(k);
                const T za_ = (ax >= 0 && ax < ncx) ? cb[(ay - c0) * ncx + ax] : T(0);
                const T zc_ = (cx >= 0 && cx < ncx) ? cb[(cy - c0) * ncx + cx] : T(0);
                const T pz = T(0.5) * (za_ + zc_);
                const T old = nz[q][c];
                v = is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + ya) ? old + pz : old;
              }
              dst[ix] = v;
            }
          }
        } else {
          for (int ix = lane; ix < nx; ix += 64) {
            T v = T(0);
            if (inside) {
              const unsigned i = (unsigned)(ya * nx + ix);
              const int cx = ix >> 1, cy = ya >> 1;
              const int ax = cx - ((ix & 1) ^ 1), ay = cy - ((ya & 1) ^ 1);
              const T pz = T(0.5) * (at(ax, ay) + at(cx, cy));
              const T old = za[i];
              v = is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + ya) ? old + pz : old;
            }
            dst[ix] = v;
          }
        }
      }
    }
    __syncthreads();
    T bb3[R][CP];  // stage C's right-hand side, loaded a stage ahead (CMP > 0)
    if constexpr (CMP > 0) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int yc = k * BH + w + NW * q - 3;
        const bool inside = yc >= 0 && yc < ny;
#pragma unroll
        for (int c = 0; c < CP; ++c) {
          const int ix = lane + 64 * c;
          bb3[q][c] = b[(inside && ix < nx) ? (unsigned)(yc * nx + ix) : 0u];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int yb = k * BH + w + NW * q - 2;
      if (yb >= -1 && yb <= ny) {
        T* dst = row(ringB, yb);
        if (yb >= 0 && yb < ny) {
          const T* rs = row(ringA, yb - 1);
          const T* rc = row(ringA, yb);
          const T* rn = row(ringA, yb + 1);
          if constexpr (CMP > 0) {
#pragma unroll
            for (int c = 0; c < CP; ++c) {
              const int ix = lane + 64 * c;
              if (ix < nx) {
                const T v = jacobi_rows<KIND, T>(P, lv, rs, rc, rn, bb[q][c], ix, yb, omega);
                dst[ix] = is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + yb) ? v : T(0);
              }
            }
          } else {
            for (int ix = lane; ix < nx; ix += 64) {
              const T v = jacobi_rows<KIND, T>(P, lv, rs, rc, rn, b[(unsigned)(yb * nx + ix)],
                                               ix, yb, omega);
              dst[ix] = is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + yb) ? v : T(0);
            }
          }
        } else {
          for (int ix = lane; ix < nx; ix += 64) dst[ix] = T(0);
        }
      }
    }
    if constexpr (CMP > 0) cb_store(k + 1);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int yc = k * BH + w + NW * q - 3;
      if (yc >= 0 && yc < ny) {
        const T* rs = row(ringB, yc - 1);
        const T* rc = row(ringB, yc);
        const T* rn = row(ringB, yc + 1);
        if constexpr (CMP > 0) {
#pragma unroll
          for (int c = 0; c < CP; ++c) {
            const int ix = lane + 64 * c;
            if (ix < nx) {
              const unsigned i = (unsigned)(yc * nx + ix);
              const T bi = bb3[q][c];
              const T v = jacobi_rows<KIND, T>(P, lv, rs, rc, rn, bi, ix, yc, omega2);
              const bool dof = is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + yc);
              za[i] = dof ? v : T(0);
              if (DOT && dof) *acc += (double)bi * (double)v;
            }
          }
          continue;
        }
        for (int ix = lane; ix < nx; ix += 64) {
          const unsigned i = (unsigned)(yc * nx + ix);
          const T bi = b[i];
          const T v = jacobi_rows<KIND, T>(P, lv, rs, rc, rn, bi, ix, yc, omega2);
          const bool dof = is_dof(P.domain, lv.N, lv.gx0 + ix, lv.gy0 + yc);
          za[i] = dof ? v : T(0);
          if (DOT && dof) *acc += (double)bi * (double)v;
        }
      }
    }
    // the next step's first-stage rows lie above every row this step writes
    if constexpr (CMP > 0) load_z(k + 1);
  }
}

// Rows of at most RING_CHUNKS chunks of 64 nodes are held in registers by the prefetching
// forms of the banded passes and the banded CG passes.
constexpr int RING_CHUNKS = 4;

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

// Level descriptors of an item: t = 0 is the tile on level m, t = m its coarse-cell grid.
// Level-0 buffers: X, R(=rhs of the V-cycle), Z, Tmp, then `extra` vectors; coarser
// levels: B, Z, Tmp each.  Descriptors are computed on demand from the item; every
// input is uniform over the workgroup, so they stay in scalar registers (a table in LDS
// would put every field, and every address formed from it, in vector registers).
struct Levels {
  int cw, ch, cx0, cy0, n_c, m, extra;
  __device__ __forceinline__ Levels(const TileItem& it, const ProbDev& P, int m_, int extra_)
      : cw(it.cw), ch(it.ch), cx0(it.cx0), cy0(it.cy0), n_c(P.n_c), m(m_), extra(extra_) {}
  __device__ __forceinline__ int64_t size(int t) const {
    const int r = 1 << (m - t);
    return (int64_t)(cw * r - 1) * (ch * r - 1);
  }
  __device__ __forceinline__ LevelDesc operator[](int t) const {
    const int l = m - t;
    const int r = 1 << l;
    LevelDesc d;
    d.nx = cw * r - 1;
    d.ny = ch * r - 1;
    d.gx0 = cx0 * r + 1;
    d.gy0 = cy0 * r + 1;
    d.N = n_c << l;
    d.l = l;
    const int64_t S = (int64_t)d.nx * d.ny;
    if (t == 0) {
      d.ob = S;
      d.oz = 2 * S;
      d.ot = 3 * S;
    } else {
      int64_t off = (4 + extra) * size(0);
      for (int u = 1; u < t; ++u) off += 3 * size(u);
      d.ob = off;
      d.oz = off + S;
      d.ot = off + 2 * S;
    }
    return d;
  }
};

// The coarse end of the V-cycle runs in LDS: from the first level whose grid is at most
// TAIL_N x TAIL_N, every sweep, restriction, interpolation and the coarse solve work on
// LDS copies (three vectors per level, at most TAIL_ELEMS elements in all), so those
// small levels cost LDS latency instead of an HBM round trip per barrier interval.
constexpr int TAIL_N = 31;
constexpr int TAIL_ELEMS = 3 * 1280;  // >= 3 (31^2 + 15^2 + 7^2 + 3^2 + 1^2)

__device__ __forceinline__ bool tail_level(const LevelDesc& lv) {
  return lv.nx <= TAIL_N && lv.ny <= TAIL_N;
}

// Levels t0 .. m of one V-cycle in LDS (sm, TAIL_ELEMS elements): b of level t0 is read
// from the item's global buffer, the correction z of level t0 is written back to it
// (base + lev[t0].oz).  With t0 = 0 the last post-smoothing sweep also adds this
// thread's share of b.z to *rz.
template <int NT, int KIND, typename T>
__device__ void vcycle_tail(const ProbDev& P, const Levels& lev, int t0, int m,
                            const double* Kinv, int nu, T omega, T omega2, T* base, T* sm,
                            double* rz) {
  auto loff = [&](int t) -> int {
    int o = 0;
    for (int u = t0; u < t; ++u) o += 3 * (int)lev.size(u);
    return o;
  };
  {
    const LevelDesc lv = lev[t0];
    const T* gb = base + lv.ob;
    FOR_TILE(lv) {
      const unsigned i = (unsigned)(iy * lv.nx + ix);
      sm[i] = gb[i];
    }
    __syncthreads();
  }
  for (int t = t0; t < m; ++t) {
    const LevelDesc lv = lev[t];
    const int S = (int)lev.size(t);
    T* b = sm + loff(t);
    T* za = b + S;
    T* zb = za + S;
    if (nu >= 2)
      op_first2<NT, KIND, T>(P, lv, b, za, omega, omega2);
    else
      op_first<NT, KIND, T>(P, lv, b, za, omega);
    __syncthreads();
    for (int s = 2; s < nu; ++s) {
      op_jacobi<NT, KIND, T>(P, lv, b, za, zb, omega2);
      __syncthreads();
      T* tmp = za;
      za = zb;
      zb = tmp;
    }
    op_residual<NT, KIND, T>(P, lv, b, za, zb);
    __syncthreads();
    op_restrict<NT, T>(P, lv, lev[t + 1], zb, sm + loff(t + 1));
    __syncthreads();
  }
  T* zc = sm + loff(m) + (int)lev.size(m);
  op_coarse_solve<NT, T>(lev[m], Kinv, sm + loff(m), zc);
  __syncthreads();
  for (int t = m - 1; t >= t0; --t) {
    const LevelDesc lv = lev[t];
    const int S = (int)lev.size(t);
    T* b = sm + loff(t);
    T* za = b + S;
    T* zb = za + S;
    const int singles = nu >= 2 ? nu - 2 : 0;
    if (singles & 1) {
      T* tmp = za;
      za = zb;
      zb = tmp;
    }
    op_prolong_add<NT, T>(P, lev[t + 1], lv, zc, za);
    __syncthreads();
    for (int s = 0; s < nu; ++s) {
      const T w = s == 0 ? omega : omega2;
      if (t == 0 && s == nu - 1)
        op_jacobi<NT, KIND, T, true>(P, lv, b, za, zb, w, rz);
      else
        op_jacobi<NT, KIND, T>(P, lv, b, za, zb, w);
      __syncthreads();
      T* tmp = za;
      za = zb;
      zb = tmp;
    }
    zc = za;
  }
  {
    const LevelDesc lv = lev[t0];
    T* gz = base + lv.oz;
    FOR_TILE(lv) {
      const unsigned i = (unsigned)(iy * lv.nx + ix);
      gz[i] = zc[i];
    }
  }
}

// One symmetric V-cycle applied to the level-0 right-hand side at lev[0].ob; returns
// the buffer that holds the result z and adds this thread's share of b.z to *rz.  With
// nu = 2 and three LDS rings sized for the tile level (ring_rows = rows per wave per
// band step, 1 or 2; 0: no rings), the pre-smoothing with residual and restriction and
// the post-smoothing of every level run as one banded pass each.
template <int NT, int KIND, typename T, int MAXR>
__device__ T* vcycle(const ProbDev& P, const Levels& lev, T* base, int m, const double* Kinv,
                     int nu, T omega, T omega2, double* rz, T* ring, int ring_rows, T* tail) {
  int tl = m + 1;  // first level handled in LDS (none when m + 1)
  if (tail != nullptr) {
    for (int t = 0; t < m; ++t)
      if (tail_level(lev[t])) {
        tl = t;
        break;
      }
  }
  for (int t = 0; t < m && t < tl; ++t) {
    const LevelDesc lv = lev[t];
    const T* b = base + lv.ob;
    T* za = base + lv.oz;
    T* zb = base + lv.ot;
    if (ring_rows > 0 && nu == 2) {
      T* bc = base + lev[t + 1].ob;
      // a constant coefficient: the next band's first-stage rows are prefetched (the
      // variable coefficients' weight loads leave no registers for it)
      constexpr bool PFC = KIND == 0;
      if (MAXR >= 2 && ring_rows == 2) {
        if (PFC && lv.nx <= 128)
          op_pre_fused<NT, KIND, T, MAXR, PFC ? 2 : 0>(P, lv, lev[t + 1], b, za, bc, omega, omega2, ring);
        else
          op_pre_fused<NT, KIND, T, MAXR>(P, lv, lev[t + 1], b, za, bc, omega, omega2, ring);
      } else if (PFC && lv.nx <= 128)
        op_pre_fused<NT, KIND, T, 1, PFC ? 2 : 0>(P, lv, lev[t + 1], b, za, bc, omega, omega2, ring);
      else if (PFC && lv.nx <= 256)
        op_pre_fused<NT, KIND, T, 1, PFC ? 4 : 0>(P, lv, lev[t + 1], b, za, bc, omega, omega2, ring);
      else
        op_pre_fused<NT, KIND, T, 1>(P, lv, lev[t + 1], b, za, bc, omega, omega2, ring);
      __syncthreads();
      continue;
    }
    if (nu >= 2)
      op_first2<NT, KIND, T>(P, lv, b, za, omega, omega2);
    else
      op_first<NT, KIND, T>(P, lv, b, za, omega);
    __syncthreads();
    for (int s = 2; s < nu; ++s) {
      op_jacobi<NT, KIND, T>(P, lv, b, za, zb, omega2);
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
  T* zc;
  if (tl <= m) {
    vcycle_tail<NT, KIND, T>(P, lev, tl, m, Kinv, nu, omega, omega2, base, tail, rz);
    __syncthreads();
    zc = base + lev[tl].oz;
  } else {
    op_coarse_solve<NT, T>(lev[m], Kinv, base + lev[m].ob, base + lev[m].oz);
    __syncthreads();
    zc = base + lev[m].oz;
  }
  for (int t = (tl <= m ? tl : m) - 1; t >= 0; --t) {
    const LevelDesc lv = lev[t];
    const T* b = base + lv.ob;
    T* za = base + lv.oz;
    T* zb = base + lv.ot;
    // the pre-smoothed iterate is in za when an even number of single sweeps followed
    // the first pass (two sweeps for nu >= 2, one for nu = 1)
    const int singles = nu >= 2 ? nu - 2 : 0;
    if (singles & 1) {
      T* tmp = za;
      za = zb;
      zb = tmp;
    }
    if (ring_rows > 0 && nu == 2) {
      const LevelDesc lc = lev[t + 1];
      constexpr bool PFC = KIND == 0;
      constexpr int C2 = PFC ? 2 : 0, C4 = PFC ? 4 : 0;
      if (MAXR >= 2 && ring_rows == 2) {
        if (PFC && lv.nx <= 128) {
          if (t == 0)
            op_post_fused<NT, KIND, T, true, MAXR, C2>(P, lc, lv, zc, b, za, omega, omega2, ring, rz);
          else
            op_post_fused<NT, KIND, T, false, MAXR, C2>(P, lc, lv, zc, b, za, omega, omega2, ring,
                                                        nullptr);
        } else if (t == 0)
          op_post_fused<NT, KIND, T, true, MAXR>(P, lc, lv, zc, b, za, omega, omega2, ring, rz);
        else
          op_post_fused<NT, KIND, T, false, MAXR>(P, lc, lv, zc, b, za, omega, omega2, ring, nullptr);
      } else if (PFC && lv.nx <= 256) {
        if (t == 0)
          op_post_fused<NT, KIND, T, true, 1, C4>(P, lc, lv, zc, b, za, omega, omega2, ring, rz);
        else
          op_post_fused<NT, KIND, T, false, 1, C4>(P, lc, lv, zc, b, za, omega, omega2, ring, nullptr);
      } else {
        if (t == 0)
          op_post_fused<NT, KIND, T, true, 1>(P, lc, lv, zc, b, za, omega, omega2, ring, rz);
        else
          op_post_fused<NT, KIND, T, false, 1>(P, lc, lv, zc, b, za, omega, omega2, ring, nullptr);
      }
      __syncthreads();
      zc = za;
      continue;
    }
    op_prolong_add<NT, T>(P, lev[t + 1], lv, zc, za);
    __syncthreads();
    for (int s = 0; s < nu; ++s) {
      const T w = s == 0 ? omega : omega2;
      if (t == 0 && s == nu - 1)
        op_jacobi<NT, KIND, T, true>(P, lv, b, za, zb, w, rz);
      else
        op_jacobi<NT, KIND, T>(P, lv, b, za, zb, w);
      __syncthreads();
      T* tmp = za;
      za = zb;
      zb = tmp;
    }
    zc = za;
  }
  return zc;
}

// FP64 solves with a constant or a tensor coefficient do not clear x before the first
// update, which writes x_1 = alpha p without reading x; the others keep reading a cleared
// x (the same change made config 3 mixed 4% slower in FP32 and config 5's fine-cell
// coefficient 2.5% slower in FP64).
template <typename T, int KIND>
constexpr bool SKIP_X0 = sizeof(T) == 8 && (KIND == 0 || KIND == 3);

// x += alpha p, r -= alpha A p and this thread's share of ||r||^2 over the tile, software
// pipelined: each wave walks its row chunks (rows w, w + NW, ..., 64 nodes per chunk) and
// issues the loads of the next chunk (p at the five stencil points, x, r) before it
// computes and stores the current one, so two memory round trips are in flight.
template <int NT, int KIND, typename T>
__device__ void pass_xr(const ProbDev& P, const LevelDesc& l0, T* X, T* R, const T* Pn, T alpha,
                        bool first, double* acc) {
  constexpr int NW = NT / 64;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nx = l0.nx, ny = l0.ny, nxc = (nx + 63) >> 6;
  struct Ld {
    T c, e, w, n, s, x, r;
  };
  auto load = [&](int iy, int ix, Ld& L) {
    const int jx = ix < nx ? ix : nx - 1;  // lanes past the row end read a valid node
    const unsigned i = (unsigned)(iy * nx + jx);
    const bool he = jx + 1 < nx, hw = jx > 0, hn = iy + 1 < ny, hs = iy > 0;
    L.c = Pn[i];
    L.e = Pn[he ? i + 1 : i];
    L.w = Pn[hw ? i - 1 : i];
    L.n = Pn[hn ? i + nx : i];
    L.s = Pn[hs ? i - nx : i];
    L.x = (SKIP_X0<T, KIND> && first) ? T(0) : X[i];  // x_0 = 0 is not read
    L.r = R[i];
  };
  int iy = w, cix = 0;
  Ld cur, nxt;
  if (iy < ny) load(iy, lane, cur);
  while (iy < ny) {
    int niy = iy, ncx = cix + 1;
    if (ncx == nxc) {
      ncx = 0;
      niy += NW;
    }
    if (niy < ny) load(niy, lane + 64 * ncx, nxt);
    const int ix = lane + 64 * cix;
    if (ix < nx) {
      const unsigned i = (unsigned)(iy * nx + ix);
      T q = T(0);
      if (is_dof(P.domain, l0.N, l0.gx0 + ix, l0.gy0 + iy)) {
        const Weights W = edge_weights<KIND, T>(P, l0.l, l0.N, l0.gx0 + ix, l0.gy0 + iy);
        const T we = T(W.e), ww = T(W.w), wn = T(W.n), ws = T(W.s);
        const T e = ix + 1 < nx ? cur.e : T(0), wv = ix > 0 ? cur.w : T(0);
        const T n = iy + 1 < ny ? cur.n : T(0), sv = iy > 0 ? cur.s : T(0);
        q = (we + ww + wn + ws) * cur.c - we * e - ww * wv - wn * n - ws * sv;
      }
      X[i] = cur.x + alpha * cur.c;
      const T r = cur.r - alpha * q;
      R[i] = r;
      *acc += (double)r * (double)r;
    }
    cur = nxt;
    iy = niy;
    cix = ncx;
  }
}

// p_new = z + beta p_old (beta = 0 and p_old unread on the first iteration), stored, and
// this thread's share of p_new . A p_new with A p_new formed from p_new at the node and
// its neighbours; software pipelined like pass_xr (z and p_old at the five stencil points
// of the next chunk are loaded before the current chunk is computed).
template <int NT, int KIND, typename T>
__device__ void pass_dir(const ProbDev& P, const LevelDesc& l0, const T* Z, const T* Po, T* Pn,
                         T beta, bool first, double* acc) {
  constexpr int NW = NT / 64;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nx = l0.nx, ny = l0.ny, nxc = (nx + 63) >> 6;
  const T bet = first ? T(0) : beta;
  const T* Pold = first ? Z : Po;  // any valid vector: its values are multiplied by 0
  struct Ld {
    T z[5], p[5];  // centre, e, w, n, s
  };
  auto load = [&](int iy, int ix, Ld& L) {
    const int jx = ix < nx ? ix : nx - 1;
    const unsigned i = (unsigned)(iy * nx + jx);
    const bool he = jx + 1 < nx, hw = jx > 0, hn = iy + 1 < ny, hs = iy > 0;
    const unsigned j[5] = {i, he ? i + 1 : i, hw ? i - 1 : i, hn ? i + nx : i, hs ? i - nx : i};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      L.z[k] = Z[j[k]];
      L.p[k] = Pold[j[k]];
    }
  };
  int iy = w, cix = 0;
  Ld cur, nxt;
  if (iy < ny) load(iy, lane, cur);
  while (iy < ny) {
    int niy = iy, ncx = cix + 1;
    if (ncx == nxc) {
      ncx = 0;
      niy += NW;
    }
    if (niy < ny) load(niy, lane + 64 * ncx, nxt);
    const int ix = lane + 64 * cix;
    if (ix < nx) {
      const unsigned i = (unsigned)(iy * nx + ix);
      T v[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) v[k] = cur.z[k] + bet * cur.p[k];
      if (is_dof(P.domain, l0.N, l0.gx0 + ix, l0.gy0 + iy)) {
        const Weights W = edge_weights<KIND, T>(P, l0.l, l0.N, l0.gx0 + ix, l0.gy0 + iy);
        const T we = T(W.e), ww = T(W.w), wn = T(W.n), ws = T(W.s);
        const T e = ix + 1 < nx ? v[1] : T(0), wv = ix > 0 ? v[2] : T(0);
        const T n = iy + 1 < ny ? v[3] : T(0), sv = iy > 0 ? v[4] : T(0);
        const T q = (we + ww + wn + ws) * v[0] - we * e - ww * wv - wn * n - ws * sv;
        *acc += (double)v[0] * (double)q;
      }
      Pn[i] = v[0];
    }
    cur = nxt;
    iy = niy;
    cix = ncx;
  }
}

// p_new = z + beta p_old (stored) and this thread's share of p_new . A p_new, banded:
// the workgroup walks the tile in bands of NW rows with one LDS ring of NW + 2 rows.  At
// step k wave w forms row k NW + w - 1 of p_new from z and p_old (two loads per node, the
// row's chunks issued together) into HBM and the ring, and after a barrier applies A to
// the row above it (k NW + w - 2) from the ring, so A p_new takes no global gathers.
// Rows -1 and ny of the ring hold zeros (the Dirichlet values); a ring row is overwritten
// only after the barrier that follows its last reader.  Rows of at most RING_CHUNKS * 64
// nodes.
template <int NT, int KIND, typename T>
__device__ void pass_dir_banded(const ProbDev& P, const LevelDesc& l0, const T* Z, const T* Po,
                                T* Pn, T beta, bool first, T* ring, double* acc) {
  constexpr int NW = NT / 64, RING = NW + 2, CM = RING_CHUNKS;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nx = l0.nx, ny = l0.ny, nch = (nx + 63) >> 6;
  const T bet = first ? T(0) : beta;
  const T* Pold = first ? Z : Po;  // any valid vector: its values are multiplied by 0
  auto row = [&](int y) -> T* { return ring + ((y + 1) % RING) * nx; };
  for (int k = 0; k * NW - 2 < ny; ++k) {
    const int ya = k * NW + w - 1, yb = ya - 1;
    if (ya >= -1 && ya <= ny) {
      const bool inA = ya >= 0 && ya < ny;
      T zv[CM], pv[CM];
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        if (c < nch) {
          const int ix = lane + 64 * c;
          const unsigned i = (inA && ix < nx) ? (unsigned)(ya * nx + ix) : 0u;
          zv[c] = Z[i];
          pv[c] = Pold[i];
        }
      }
      T* dst = row(ya);
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        const int ix = lane + 64 * c;
        if (c < nch && ix < nx) {
          T v = T(0);
          if (inA) {
            v = zv[c] + bet * pv[c];
            Pn[(unsigned)(ya * nx + ix)] = v;
          }
          dst[ix] = v;
        }
      }
    }
    __syncthreads();
    if (yb >= 0 && yb < ny) {
      const T* rs = row(yb - 1);
      const T* rc = row(yb);
      const T* rn = row(yb + 1);
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        const int ix = lane + 64 * c;
        if (c < nch && ix < nx && is_dof(P.domain, l0.N, l0.gx0 + ix, l0.gy0 + yb)) {
          T d;
          const T q = apply_rows<KIND, T>(P, l0, rs, rc, rn, ix, yb, d);
          *acc += (double)rc[ix] * (double)q;
        }
      }
    }
    __syncthreads();
  }
}

// x += alpha p, r -= alpha A p and this thread's share of ||r||^2, banded like
// pass_dir_banded: at step k wave w stages row k NW + w - 1 of p in the ring and loads x
// and r of the row above it, and after a barrier updates that row with A p from the ring
// (three loads per node instead of seven).  Rows of at most RING_CHUNKS * 64 nodes.
template <int NT, int KIND, typename T>
__device__ void pass_xr_banded(const ProbDev& P, const LevelDesc& l0, T* X, T* R, const T* Pn,
                               T alpha, bool first, T* ring, double* acc) {
  constexpr int NW = NT / 64, RING = NW + 2, CM = RING_CHUNKS;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nx = l0.nx, ny = l0.ny, nch = (nx + 63) >> 6;
  auto row = [&](int y) -> T* { return ring + ((y + 1) % RING) * nx; };
  for (int k = 0; k * NW - 2 < ny; ++k) {
    const int ya = k * NW + w - 1, yb = ya - 1;
    const bool inA = ya >= 0 && ya < ny, inB = yb >= 0 && yb < ny;
    T pv[CM], xv[CM], rv[CM];
#pragma unroll
    for (int c = 0; c < CM; ++c) {
      if (c < nch) {
        const int ix = lane + 64 * c;
        const int jx = ix < nx ? ix : nx - 1;
        pv[c] = Pn[inA ? (unsigned)(ya * nx + jx) : 0u];
        const unsigned ib = inB ? (unsigned)(yb * nx + jx) : 0u;
        xv[c] = (SKIP_X0<T, KIND> && first) ? T(0) : X[ib];  // x_0 = 0 is not read
        rv[c] = R[ib];
      }
    }
    if (ya >= -1 && ya <= ny) {
      T* dst = row(ya);
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        const int ix = lane + 64 * c;
        if (c < nch && ix < nx) dst[ix] = inA ? pv[c] : T(0);
      }
    }
    __syncthreads();
    if (inB) {
      const T* rs = row(yb - 1);
      const T* rc = row(yb);
      const T* rn = row(yb + 1);
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        const int ix = lane + 64 * c;
        if (c < nch && ix < nx) {
          T q = T(0);
          if (is_dof(P.domain, l0.N, l0.gx0 + ix, l0.gy0 + yb)) {
            T d;
            q = apply_rows<KIND, T>(P, l0, rs, rc, rn, ix, yb, d);
          }
          const unsigned i = (unsigned)(yb * nx + ix);
          X[i] = xv[c] + alpha * rc[ix];
          const T r = rv[c] - alpha * q;
          R[i] = r;
          *acc += (double)r * (double)r;
        }
      }
    }
    __syncthreads();
  }
}

// The same two passes without pipelining: one chunk at a time.  With a variable
// coefficient the edge-weight loads need the registers the pipelining would take.
template <int NT, int KIND, typename T>
__device__ void pass_dir_plain(const ProbDev& P, const LevelDesc& l0, const T* Z, const T* Po,
                               T* Pn, T beta, bool first, double* acc) {
  const T bet = first ? T(0) : beta;
  const T* Pold = first ? Z : Po;  // any valid vector: its values are multiplied by 0
  auto pv = [&](unsigned j) -> T { return Z[j] + bet * Pold[j]; };
  FOR_TILE(l0) {
    const unsigned i = (unsigned)(iy * l0.nx + ix);
    const bool he = ix + 1 < l0.nx, hw = ix > 0, hn = iy + 1 < l0.ny, hs = iy > 0;
    const T pc = pv(i);
    const T e0 = pv(he ? i + 1 : i), w0 = pv(hw ? i - 1 : i);
    const T n0 = pv(hn ? i + l0.nx : i), s0 = pv(hs ? i - l0.nx : i);
    const T e = he ? e0 : T(0), w = hw ? w0 : T(0), n = hn ? n0 : T(0), s = hs ? s0 : T(0);
    T ne = T(0), sw = T(0);
    if constexpr (KIND == 3) {
      const bool hne = he && hn, hsw = hw && hs;
      const T ne0 = pv(hne ? i + l0.nx + 1 : i), sw0 = pv(hsw ? i - l0.nx - 1 : i);
      ne = hne ? ne0 : T(0);
      sw = hsw ? sw0 : T(0);
    }
    const Weights W = edge_weights<KIND, T>(P, l0.l, l0.N, l0.gx0 + ix, l0.gy0 + iy);
    T d;
    const T q = apply_k<KIND, T>(W, pc, e, w, n, s, ne, sw, d);
    if (is_dof(P.domain, l0.N, l0.gx0 + ix, l0.gy0 + iy)) *acc += (double)pc * (double)q;
    Pn[i] = pc;
  }
}

template <int NT, int KIND, typename T>
__device__ void pass_xr_plain(const ProbDev& P, const LevelDesc& l0, T* X, T* R, const T* Pn,
                              T alpha, bool first, double* acc) {
  FOR_TILE(l0) {
    const unsigned i = (unsigned)(iy * l0.nx + ix);
    T q = T(0);
    if (is_dof(P.domain, l0.N, l0.gx0 + ix, l0.gy0 + iy)) {
      T d;
      q = stencil<KIND, T>(P, l0, Pn, ix, iy, i, d);
    }
    X[i] = ((SKIP_X0<T, KIND> && first) ? T(0) : X[i]) + alpha * Pn[i];  // x_0 = 0 is not read
    const T r = R[i] - alpha * q;
    R[i] = r;
    *acc += (double)r * (double)r;
  }
}

// Preconditioned conjugate gradients on K_j x = r with the V-cycle preconditioner, in
// the vector type T of the tile buffers (reductions in FP64).  On entry R (level-0
// right-hand side buffer) holds r; where SKIP_X0 holds X need not be set: the first
// update writes x_1 = alpha p without reading it (with r = 0 the iteration runs once with
// p = 0 and alpha = 0, so x_1 = 0); elsewhere X is zero.  bb = ||r||^2.  Iterates until
// ||r_k||^2 <= tol2 or max_it; returns the iteration count and the final ||r_k||^2 in rr.
// MAXR: the most band rows per wave the caller's rings may ask for (1 or 2).
// The search direction alternates between two buffers (the new one is formed from the
// old one and the preconditioned residual while neighbours still read the old one).
template <int NT, int KIND, typename T, int MAXR>
__device__ int pcg_solve(const ProbDev& P, const Levels& lev, T* base, int m, const double* Kinv,
                         double bb, double tol2, int max_it, int nu, double omega,
                         double omega2, double* red,
                         T* ring, int ring_rows, T* tail, double& rr) {
  const LevelDesc l0 = lev[0];
  const int64_t S0 = (int64_t)l0.nx * l0.ny;
  T* X = base;
  T* R = base + l0.ob;
  T* Po = base + 4 * S0;
  T* Pn = base + 5 * S0;
  const T om = T(omega), om2 = T(omega2);
  int iters = 0;
  rr = bb;
  if constexpr (!SKIP_X0<T, KIND>) {
    if (!(bb > 0.0)) return 0;
  }
  double acc[2];
  // One call site for the V-cycle (it is inlined, and a second copy would cost
  // registers): the first pass through the loop only preconditions r_0.
  const T* Z = nullptr;
  double rho = 0.0;
  T beta = T(0);
  bool first = true;
  for (;;) {
    if (Z != nullptr) {
      if (iters >= max_it) break;
      ++iters;
      // p_new = z + beta p_old and p_new . A p_new, with A p_new formed from p_new at the
      // node and its neighbours
      acc[0] = acc[1] = 0.0;
      if (ring != nullptr && l0.nx <= 64 * RING_CHUNKS)
        pass_dir_banded<NT, KIND, T>(P, l0, Z, Po, Pn, beta, first, ring, &acc[0]);
      else if constexpr (KIND == 0)
        pass_dir<NT, KIND, T>(P, l0, Z, Po, Pn, beta, first, &acc[0]);
      else
        pass_dir_plain<NT, KIND, T>(P, l0, Z, Po, Pn, beta, first, &acc[0]);
      block_sum<NT, 2>(acc, red);
      // (FP64) a zero right-hand side gives p = 0: alpha = 0 writes x_1 = 0, r stays 0
      const T alpha = SKIP_X0<T, KIND> ? (acc[0] > 0.0 ? T(rho / acc[0]) : T(0)) : T(rho / acc[0]);
      // x += alpha p, r -= alpha A p, ||r||^2
      acc[0] = acc[1] = 0.0;
      if (ring != nullptr && l0.nx <= 64 * RING_CHUNKS)
        pass_xr_banded<NT, KIND, T>(P, l0, X, R, Pn, alpha, first, ring, &acc[0]);
      else if constexpr (KIND == 0)
        pass_xr<NT, KIND, T>(P, l0, X, R, Pn, alpha, first, &acc[0]);
      else
        pass_xr_plain<NT, KIND, T>(P, l0, X, R, Pn, alpha, first, &acc[0]);
      block_sum<NT, 2>(acc, red);
      rr = acc[0];
      if (rr <= tol2) break;
    }
    acc[0] = acc[1] = 0.0;
    const bool init = Z == nullptr;
    Z = vcycle<NT, KIND, T, MAXR>(P, lev, base, m, Kinv, nu, om, om2, &acc[0], ring, ring_rows,
                                  tail);
    block_sum<NT, 2>(acc, red);
    if (init) {
      rho = acc[0];
      continue;
    }
    beta = T(acc[0] / rho);
    rho = acc[0];
    first = false;
    T* tmp = Po;
    Po = Pn;
    Pn = tmp;
  }
  return iters;
}

}  // namespace
