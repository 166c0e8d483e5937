// Device-side data structures and helpers shared by the HIP kernels of libmlc.
//
// Geometry: a level-l grid of the bounding box has N_l = n_c * 2^l cells per side and
// (N_l+1)^2 nodes, node (gx, gy) at index gy*(N_l+1)+gx.  Square cell (I, J) is cut by
// its SW-NE diagonal into a lower triangle (SW, SE, NE) and an upper one (SW, NE, NW).
// With P1 elements and a scalar coefficient only the two legs of each triangle couple,
// so the stiffness is a five-point stencil whose edge weights average the kappa of the
// two triangles on each side of the edge; the mass is (h^2/12)[6; E, W, N, S, NE, SW].
// With a full tensor A (Example 6.2) the hypotenuse couples too and the mass carries the
// weight phi: both are seven-point stencils, stored per level (coefficient kind 3).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MLC_MAX_LEVELS 10
#define MLC_MAX_Q 8
#define MLC_MAX_TILE_COARSE 64      // coarse tile grids up to this size are inverted in LDS
#define MLC_MAX_TILE_COARSE_ALL 1024  // larger ones (up to this) in HBM
#define MLC_MAX_CAND 8
#define MLC_JACOBI_MAX_NH 400       // coarse spaces up to this size are decomposed on the device
// The device eigensolver pads the order to an even number of Jacobi blocks of 16, and its
// scratch per problem is L (n x n) and three n2 x n2 matrices.
__host__ __device__ constexpr int eig_padded(int n) {
  int nb = (n + 15) / 16;
  nb += nb & 1;
  return nb * 16;
}
__host__ __device__ inline int64_t eig_scratch_doubles(int n) {
  const int64_t n2 = eig_padded(n);
  return (int64_t)n * n + 3 * n2 * n2;
}

// Per-problem device record.  Pointers are into the caller's workspace.
struct ProbDev {
  int32_t domain, n_c, L, q, coef_kind, sub_x, sub_y, overlap;
  // element degree (1 or 2).  A level-l grid vector holds the element's nodes: the mesh
  // nodes for P1, the vertices and edge midpoints for P2, i.e. the nodes of the grid with
  // n_c 2^(l + order - 1) intervals per side.  Lg = L + order - 1 is that grid's level at
  // the finest mesh; c1 = n_c * order + 1 nodes per side on the coarse mesh.
  int32_t order, Lg, c1;
  int32_t nH;                 // coarse interior nodes (dofs of V_0H)
  int32_t nparts;             // blocks of the fine-level reductions at the finest level
  double side;                // bounding-box side length
  const double* kH;           // coef kinds 0/1: n_c*n_c per coarse cell
  const double* kLR[MLC_MAX_LEVELS + 1];  // coef kind 2: per level, N_l*N_l lower-triangle kappa
  const double* kUL[MLC_MAX_LEVELS + 1];  //                            upper-triangle kappa
  // coef kind 3: per level, 7 planes of (N_l+1)^2 values: the stiffness weights
  // -K(i, i+E), -K(i, i+N), -K(i, i+NE), then the mass M(i,i), M(i,i+E), M(i,i+N),
  // M(i,i+NE).  The stiffness diagonal is the sum of the six weights of a node (every row
  // of the Galerkin stiffness sums to zero: a(phi_i, 1) = 0), so it is not stored.
  const double* st7[MLC_MAX_LEVELS + 1];
  const float* st7f[MLC_MAX_LEVELS + 1];  // the three stiffness planes in FP32 (mixed solver)
  const int32_t* bx;          // sub_x+1 block boundaries in coarse cells
  const int32_t* by;          // sub_y+1
  int32_t sub_item_off;       // offset of this problem's (sub_x*sub_y)*q block in a step's
                              // subdomain -> item table (-1 entries: dropped or inactive)
  int32_t pou;                // gluing weights: 0 ramp, 1 indicator of the closed D_j
  const int32_t* coarse_nodes;  // nH: grid index (on (n_c+1)^2) of coarse dof r
  const int32_t* coarse_index;  // (n_c+1)^2: dof index or -1
  double* u[2];               // eigenvectors, q*(N_L+1)^2 each (ping-pong)
  double* lam;                // [2][MLC_MAX_Q]
  double* ubar;               // q*(N_L+1)^2: I u_k, later M u~
  double* res;                // q*(N_L+1)^2: Aux_Problem right-hand side, later K u~
  double* ut;                 // q*(N_L+1)^2: glued u~
  double* rchain;             // restriction chain
  int64_t rchain_off[MLC_MAX_LEVELS + 1];
  double* V;                  // nH*nH column-major, M_H-orthonormal coarse eigenvectors
  double* Lam;                // nH ascending coarse eigenvalues
  double* Kc;                 // nH*nH coarse stiffness (setup scratch, overwritten by V)
  double* Mc;                 // nH*nH coarse mass (setup scratch, then V^T)
  double* VT;                 // nH*nH row-major V^T (aliases Mc after setup)
  double* fg;                 // 2*q*nH: f = V^T a, g = V^T b
  double* partials;           // nparts*(2q^2+q)
  double* rr_y;               // q*nH coarse eigen-coordinates of the new eigenvectors
  double* rr_t;               // q*q coefficients of u~
  double* rr_ab;              // alpha = u~^T K u~, beta = u~^T M u~ (q = 1: 2 values)
  double* cH_grid;            // q*(n_c+1)^2 coarse nodal coefficients
  double* sum_parts;          // output sign partial sums
  // per level step s: the largest final relative residual of the step's local solves,
  // [MLC_MAX_LEVELS + 1] doubles shared by every problem of a batch (non-negative doubles
  // order as their bit patterns, so the solves raise it with an integer atomic maximum);
  // cleared by the step's first kernel
  double* conv;
  // setup: scratch of the device eigensolver (n_H^2 + 2 (n_H + 1)^2 doubles), NULL when the
  // coarse space goes to rocSOLVER; its status (0 = success)
  double* eig_ws;
  int32_t* info;
};

// One local solve: subdomain Omega_j of problem prob, right-hand side rhs.
struct TileItem {
  // rhs_stride: bytes from this item's storage to that of the next right-hand side of the
  // same subdomain (the q items of a subdomain are consecutive and equally sized)
  int32_t prob, sub, rhs, rhs_stride;
  int32_t cx0, cy0, cw, ch;   // Omega_j in coarse cells
  int64_t off;                // byte offset of the item's storage
  int64_t inv_off;            // double offset of the subdomain's coarsest-grid inverse
};

struct ItemStat {
  int32_t iters, refine;
  double relres;
};

// Row of entry idx of a row-major array with n columns, floor(idx / n), for
// 0 <= idx < n^2 <= 2^31: a float reciprocal estimate (error below 2^-20 of a quotient
// under 2^16) corrected by one step either way.  A 64-bit integer division costs about a
// hundred vector instructions, which the one-thread-per-node grid kernels would otherwise
// spend on every node.
__device__ __forceinline__ int grid_row(int64_t idx, int n) {
  const unsigned u = (unsigned)idx, un = (unsigned)n;
  unsigned q = (unsigned)((float)u * __builtin_amdgcn_rcpf((float)n));
  if (q * un > u)
    --q;
  else if ((q + 1u) * un <= u)
    ++q;
  return (int)q;
}

__device__ __forceinline__ bool is_dof(int domain, int N, int gx, int gy) {
  if (gx <= 0 || gy <= 0 || gx >= N || gy >= N) return false;
  if (domain == 1 && gx >= (N >> 1) && gy <= (N >> 1)) return false;
  return true;
}

// Edge weights around node (gx, gy) on a level with N cells, level index l (coarse = 0):
// minus the stiffness couplings to the four leg neighbours, and with coefficient kind 3
// also to the NE and SW neighbours (for kinds 0-2 ne and sw are not set).  The diagonal
// is the sum of the weights.
struct Weights {
  double e, w, n, s, ne, sw;
};

// Coefficient arrays are reached through pointers held in ProbDev; the cast to the
// global address space lets the compiler emit global (not flat) loads for them.
typedef __attribute__((address_space(1))) const double gconst_double;

typedef __attribute__((address_space(1))) const float gconst_float;

// T selects the stored precision of the kind-3 stiffness (FP32 planes for float solves).
template <int KIND, typename T = double>
__device__ __forceinline__ Weights edge_weights(const ProbDev& P, int l, int N, int gx, int gy) {
  Weights W;
  if constexpr (KIND == 3) {
    const int n1 = N + 1;
    const int64_t pl = (int64_t)n1 * n1;
    const int64_t c = (int64_t)gy * n1 + gx;
    if constexpr (sizeof(T) == 4) {
      const gconst_float* st = (const gconst_float*)P.st7f[l];
      W.e = st[c];
      W.w = st[c - 1];
      W.n = st[pl + c];
      W.s = st[pl + c - n1];
      W.ne = st[2 * pl + c];
      W.sw = st[2 * pl + c - n1 - 1];
    } else {
      const gconst_double* st = (const gconst_double*)P.st7[l];
      W.e = st[c];
      W.w = st[c - 1];
      W.n = st[pl + c];
      W.s = st[pl + c - n1];
      W.ne = st[2 * pl + c];
      W.sw = st[2 * pl + c - n1 - 1];
    }
  } else if (KIND == 0) {
    W.e = W.w = W.n = W.s = 1.0;
  } else if (KIND == 1) {
    const int nc = P.n_c;
    const gconst_double* k = (const gconst_double*)P.kH;
    const int cx = gx >> l, cxm = (gx - 1) >> l;
    const int cy = gy >> l, cym = (gy - 1) >> l;
    const double k00 = k[cy * nc + cx];      // cell (gx, gy)
    const double k10 = k[cy * nc + cxm];     // cell (gx-1, gy)
    const double k01 = k[cym * nc + cx];     // cell (gx, gy-1)
    const double k11 = k[cym * nc + cxm];    // cell (gx-1, gy-1)
    W.e = 0.5 * (k00 + k01);
    W.w = 0.5 * (k10 + k11);
    W.n = 0.5 * (k00 + k10);
    W.s = 0.5 * (k01 + k11);
  } else {
    const gconst_double* lo = (const gconst_double*)P.kLR[l];
    const gconst_double* up = (const gconst_double*)P.kUL[l];
    const int c = gy * N + gx;
    // horizontal edge (gx,gy)-(gx+1,gy): lower triangle of cell (gx,gy), upper of (gx,gy-1)
    W.e = 0.5 * (lo[c] + up[c - N]);
    W.w = 0.5 * (lo[c - 1] + up[c - N - 1]);
    // vertical edge (gx,gy)-(gx,gy+1): upper triangle of cell (gx,gy), lower of (gx-1,gy)
    W.n = 0.5 * (up[c] + lo[c - 1]);
    W.s = 0.5 * (up[c - N] + lo[c - N - 1]);
  }
  return W;
}

// Stiffness diagonal from the weights.
template <int KIND>
__device__ __forceinline__ double diag_of(const Weights& W) {
  if constexpr (KIND == 3)
    return W.e + W.w + W.n + W.s + W.ne + W.sw;
  else
    return W.e + W.w + W.n + W.s;
}

// K u at a node from u at the node and its six neighbours (five-point for kinds 0-2,
// where ne and sw are not used); d receives the diagonal.
template <int KIND, typename T>
__device__ __forceinline__ T apply_k(const Weights& W, T c, T e, T w, T n, T s, T ne, T sw, T& d) {
  const T we = T(W.e), ww = T(W.w), wn = T(W.n), ws = T(W.s);
  if constexpr (KIND == 3) {
    const T wne = T(W.ne), wsw = T(W.sw);
    d = we + ww + wn + ws + wne + wsw;
    return d * c - we * e - ww * w - wn * n - ws * s - wne * ne - wsw * sw;
  } else {
    d = we + ww + wn + ws;
    return d * c - we * e - ww * w - wn * n - ws * s;
  }
}

// Mass couplings of node (gx, gy) on level l: the diagonal and the six neighbours
// (kind 3 reads the stored weighted mass; kinds 0-2 have the constant h^2/12 pattern).
struct MassW {
  double d, e, w, n, s, ne, sw;
};

template <int KIND>
__device__ __forceinline__ MassW mass_weights(const ProbDev& P, int l, int N, int gx, int gy,
                                              double mh) {
  MassW M;
  if constexpr (KIND == 3) {
    const int n1 = N + 1;
    const int64_t pl = (int64_t)n1 * n1;
    const gconst_double* m = (const gconst_double*)P.st7[l] + 3 * pl;
    const int64_t i = (int64_t)gy * n1 + gx;
    M.d = m[i];
    M.e = m[pl + i];
    M.w = m[pl + i - 1];
    M.n = m[2 * pl + i];
    M.s = m[2 * pl + i - n1];
    M.ne = m[3 * pl + i];
    M.sw = m[3 * pl + i - n1 - 1];
  } else {
    M.d = 6.0 * mh;
    M.e = M.w = M.n = M.s = M.ne = M.sw = mh;
  }
  return M;
}

// M u at a node: the consistent mass (h^2/12)[6; E, W, N, S, NE, SW] for kinds 0-2
// (mh = h^2/12), the stored weighted mass for kind 3.
template <int KIND>
__device__ __forceinline__ double apply_mass(const MassW& M, double mh, double c, double e,
                                             double w, double n, double s, double ne, double sw) {
  if constexpr (KIND == 3)
    return M.d * c + M.e * e + M.w * w + M.n * n + M.s * s + M.ne * ne + M.sw * sw;
  else
    return mh * (6.0 * c + e + w + n + s + ne + sw);
}

// D_j block boundaries along one axis: floor(b * nc / nb) coarse cells (nb blocks over nc
// cells, each block at least one cell wide), and the block holding coarse cell c.
__device__ __forceinline__ int block_bound(int b, int nc, int nb) { return (b * nc) / nb; }
__device__ __forceinline__ int block_of_cell(int c, int nc, int nb) {
  return ((c + 1) * nb - 1) / nc;
}

// Blocks along one axis whose Omega range (D_j grown by `ov` coarse cells) holds fine
// grid index g strictly inside, i.e. whose tiles cover the node, with the factor rho of
// phi_j along that axis: the ramp (1 on D_j, linear to 0 across the overlap; exact
// dyadic arithmetic) or the indicator of the closed D_j range.  r = fine cells per
// coarse cell, nc coarse cells, nb blocks.  Blocks are at least one coarse cell wide, so
// only the block of g's coarse cell and ov + 1 blocks on each side can qualify; they are
// visited in ascending order.  Returns the number of candidates (at most MLC_MAX_CAND).
__device__ __forceinline__ int pou_axis(int nc, int nb, int g, int r, int ov, int pou,
                                        int (&id)[MLC_MAX_CAND], double (&rho)[MLC_MAX_CAND]) {
  const int d = ov * r;
  const int b0 = block_of_cell(min(g / r, nc - 1), nc, nb);
  const int blo = max(0, b0 - ov - 1), bhi = min(nb - 1, b0 + ov + 1);
  int n = 0;
  for (int b = blo; b <= bhi && n < MLC_MAX_CAND; ++b) {
    const int lo = block_bound(b, nc, nb) * r, hi = block_bound(b + 1, nc, nb) * r;
    const int v = min(g - lo + d, hi + d - g);
    if (v > 0) {
      id[n] = b;
      rho[n] = pou == 0 ? (double)min(v, d) / (double)d : (g >= lo && g <= hi ? 1.0 : 0.0);
      ++n;
    }
  }
  return n;
}

// ---------------------------------------------------------------------------------
// Workgroup reductions (fixed order: across a wave's lanes by DPP moves, then the waves in
// index order)
// ---------------------------------------------------------------------------------
// A value every lane holds equally, moved to a scalar register.
__device__ __forceinline__ double uniform_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One cross-lane move of a double by DPP (a register read from another lane of the same
// row of 16 lanes, or a row broadcast), applied to both 32-bit halves; lanes without a
// source lane, or in rows not selected by ROW_MASK, receive `old`.  Needs every lane of
// the wave active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v, double old) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned long long o = (unsigned long long)__double_as_longlong(old);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)o, (int)(unsigned)b,
                                                            CTRL, ROW_MASK, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(
      (int)(unsigned)(o >> 32), (int)(unsigned)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Reduction over aligned groups of gs lanes (gs a power of two, 1..64) with the operation
// op and its identity id; the result is complete in the last lane of each group.  Steps:
// neighbour pairs and quads (quad permutations), shifts by 4 and 8 inside rows of 16, then
// row 0 into row 1 and row 2 into row 3 (broadcast of lane 15), rows 0-1 into rows 2-3
// (broadcast of lane 31).
template <typename Op>
__device__ __forceinline__ double group_reduce_last(double v, int gs, double id, Op op) {
  if (gs > 1) v = op(v, dpp_f64<0xb1, 0xf>(v, id));   // quad_perm [1,0,3,2]
  if (gs > 2) v = op(v, dpp_f64<0x4e, 0xf>(v, id));   // quad_perm [2,3,0,1]
  if (gs > 4) v = op(v, dpp_f64<0x114, 0xf>(v, id));  // row_shr 4
  if (gs > 8) v = op(v, dpp_f64<0x118, 0xf>(v, id));  // row_shr 8
  if (gs > 16) v = op(v, dpp_f64<0x142, 0xa>(v, id)); // row_bcast 15 into rows 1 and 3
  if (gs > 32) v = op(v, dpp_f64<0x143, 0xc>(v, id)); // row_bcast 31 into rows 2 and 3
  return v;
}

__device__ __forceinline__ double group_sum_last(double v, int gs) {
  return group_reduce_last(v, gs, 0.0, [](double a, double b) { return a + b; });
}

__device__ __forceinline__ double read_lane_f64(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes of a wave (every lane active), the same value in every lane.
__device__ __forceinline__ double wave_sum(double v) {
  return read_lane_f64(group_sum_last(v, 64), 63);
}

template <int NT, int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* lds) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[k * NW + wid] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += lds[k * NW + w];
    v[k] = uniform_f64(s);  // every lane summed the same values in the same order
  }
}

// Kernel launchers (defined in the .hip files).
struct LaunchCfg {
  hipStream_t stream;
};
