// P2 elements on the SW-NE right-triangle meshes (Section 2.1 with k = 2; Example 6.1 runs
// P1 and P2): device helpers shared by the P2 kernels.
//
// A P2 function is fixed by its values at the vertices and edge midpoints of the mesh.
// On a mesh of N cells per side these are the nodes of the grid with 2N intervals per side
// (the "half grid"): node (x, y) is a vertex when x and y are even, the midpoint of a
// horizontal edge when only x is odd, of a vertical edge when only y is odd, and of a
// cell's SW-NE diagonal when both are odd (class = (x & 1) | (y & 1) << 1).
//
// Cell (I, J) spans half-grid [2I, 2I+2] x [2J, 2J+2] and holds two triangles, each with
// local nodes v0, v1, v2, e01, e12, e20 (vertices, then the midpoints of v0v1, v1v2, v2v0):
//   lower (up = 0): v0 = SW, v1 = SE, v2 = NE;   upper (up = 1): v0 = SW, v1 = NE, v2 = NW.
// With barycentric coordinates l_a and G_ab = |T| grad l_a . grad l_b, the P2 shape
// functions l_a (2 l_a - 1) and 4 l_a l_b give the element stiffness
//   K(a, a) = G_aa,  K(a, b) = -G_ab / 3 (vertices),  K(a, e_ab) = 4 G_ab / 3,
//   K(a, opposite edge) = 0,  K(e_ab, e_ab) = 8 (G_aa + G_ab + G_bb) / 3,
//   K(e_ab, e_ac) = 8 G_bc / 3,
// and the element mass |T| / 180 times: 6 on vertex diagonals, -1 between vertices, -4
// between a vertex and the opposite edge, 0 between a vertex and its own edges, 32 on edge
// diagonals, 16 between edges.  On these right triangles (legs h, |T| = h^2 / 2),
// G = [[1/2, -1/2, 0], [-1/2, 1, -1/2], [0, -1/2, 1/2]] for the lower triangle and
// [[1/2, 0, -1/2], [0, 1/2, -1/2], [-1/2, -1/2, 1]] for the upper one, independent of h:
// the tables below hold 6 K (stiffness, kappa = 1) and 360 M / h^2 (mass).  Every row of
// K sums to zero (the shape functions sum to one).
#pragma once
#include "mlc_device.h"

namespace p2 {

// Local node positions (half-grid offsets from the cell's SW corner).
__host__ __device__ constexpr int node_dx(int up, int b) {
  return up == 0 ? (b == 0 ? 0 : b == 1 ? 2 : b == 2 ? 2 : b == 3 ? 1 : b == 4 ? 2 : 1)
                 : (b == 0 ? 0 : b == 1 ? 2 : b == 2 ? 0 : b == 3 ? 1 : b == 4 ? 1 : 0);
}
__host__ __device__ constexpr int node_dy(int up, int b) {
  return up == 0 ? (b == 0 ? 0 : b == 1 ? 0 : b == 2 ? 2 : b == 3 ? 0 : b == 4 ? 1 : 1)
                 : (b == 0 ? 0 : b == 1 ? 2 : b == 2 ? 2 : b == 3 ? 1 : b == 4 ? 2 : 1);
}

// 6 K of the lower (up = 0) and upper (up = 1) triangle.
__host__ __device__ constexpr int k6(int up, int a, int b) {
  constexpr int lo[6][6] = {{3, 1, 0, -4, 0, 0},   {1, 6, 1, -4, -4, 0}, {0, 1, 3, 0, -4, 0},
                            {-4, -4, 0, 16, 0, -8}, {0, -4, -4, 0, 16, -8}, {0, 0, 0, -8, -8, 16}};
  constexpr int hi[6][6] = {{3, 0, 1, 0, 0, -4},   {0, 3, 1, 0, -4, 0},  {1, 1, 6, 0, -4, -4},
                            {0, 0, 0, 16, -8, -8}, {0, -4, -4, -8, 16, 0}, {-4, 0, -4, -8, 0, 16}};
  return up == 0 ? lo[a][b] : hi[a][b];
}

// 360 M / h^2 (the same for both triangles).
__host__ __device__ constexpr int m360(int a, int b) {
  constexpr int m[6][6] = {{6, -1, -1, 0, -4, 0},  {-1, 6, -1, 0, 0, -4}, {-1, -1, 6, -4, 0, 0},
                           {0, 0, -4, 32, 16, 16}, {-4, 0, 0, 16, 32, 16}, {0, -4, 0, 16, 16, 32}};
  return m[a][b];
}

// The triangles holding a node of each class, relative to the cell (x >> 1, y >> 1): cell
// offset (di, dj), triangle (up) and the node's local index (loc).
//   vertex: SW of the lower and upper triangle of (0, 0), SE of the lower of (-1, 0), NE
//           of the lower and the upper of (-1, -1), NW of the upper of (0, -1);
//   horizontal midpoint: e01 of the lower of (0, 0), e12 of the upper of (0, -1);
//   vertical midpoint: e20 of the upper of (0, 0), e12 of the lower of (-1, 0);
//   diagonal midpoint: e20 of the lower and e01 of the upper of (0, 0).
__host__ __device__ constexpr int ntri(int cls) { return cls == 0 ? 6 : 2; }
__host__ __device__ constexpr int tri_field(int cls, int t, int f) {
  // f: 0 di, 1 dj, 2 up, 3 loc
  constexpr int v[6][4] = {{0, 0, 0, 0}, {0, 0, 1, 0}, {-1, 0, 0, 1},
                           {-1, -1, 0, 2}, {-1, -1, 1, 1}, {0, -1, 1, 2}};
  constexpr int x[2][4] = {{0, 0, 0, 3}, {0, -1, 1, 4}};
  constexpr int y[2][4] = {{0, 0, 1, 5}, {-1, 0, 0, 4}};
  constexpr int d[2][4] = {{0, 0, 0, 5}, {0, 0, 1, 3}};
  return cls == 0 ? v[t][f] : cls == 1 ? x[t][f] : cls == 2 ? y[t][f] : d[t][f];
}

template <int CLS, int T, int F>
struct TriF {
  static constexpr int v = tri_field(CLS, T, F);
};

// Offset of local node B of triangle T (of class CLS) from the node itself.
template <int CLS, int T, int B>
struct NodeOff {
  static constexpr int up = TriF<CLS, T, 2>::v;
  static constexpr int dx = 2 * TriF<CLS, T, 0>::v + node_dx(up, B) - (CLS & 1);
  static constexpr int dy = 2 * TriF<CLS, T, 1>::v + node_dy(up, B) - (CLS >> 1);
};

template <bool MASS, int UP, int A, int B>
struct Coef {
  static constexpr int v = MASS ? m360(A, B) : k6(UP, A, B);
};

// Row of triangle T of a class-CLS node: sum_b coef(loc, b) u(node + offset_b).
template <int CLS, int T, bool MASS, typename U>
__device__ __forceinline__ double tri_row(const U& u) {
  constexpr int up = TriF<CLS, T, 2>::v, loc = TriF<CLS, T, 3>::v;
  double s = 0.0;
  if constexpr (Coef<MASS, up, loc, 0>::v != 0)
    s += (double)Coef<MASS, up, loc, 0>::v * u(NodeOff<CLS, T, 0>::dx, NodeOff<CLS, T, 0>::dy);
  if constexpr (Coef<MASS, up, loc, 1>::v != 0)
    s += (double)Coef<MASS, up, loc, 1>::v * u(NodeOff<CLS, T, 1>::dx, NodeOff<CLS, T, 1>::dy);
  if constexpr (Coef<MASS, up, loc, 2>::v != 0)
    s += (double)Coef<MASS, up, loc, 2>::v * u(NodeOff<CLS, T, 2>::dx, NodeOff<CLS, T, 2>::dy);
  if constexpr (Coef<MASS, up, loc, 3>::v != 0)
    s += (double)Coef<MASS, up, loc, 3>::v * u(NodeOff<CLS, T, 3>::dx, NodeOff<CLS, T, 3>::dy);
  if constexpr (Coef<MASS, up, loc, 4>::v != 0)
    s += (double)Coef<MASS, up, loc, 4>::v * u(NodeOff<CLS, T, 4>::dx, NodeOff<CLS, T, 4>::dy);
  if constexpr (Coef<MASS, up, loc, 5>::v != 0)
    s += (double)Coef<MASS, up, loc, 5>::v * u(NodeOff<CLS, T, 5>::dx, NodeOff<CLS, T, 5>::dy);
  return s;
}

// sum over the node's triangles of w(cell offset) times their rows (in the table units).
template <int CLS, int T, bool MASS, typename W, typename U>
__device__ __forceinline__ double tri_sum(const W& w, const U& u) {
  if constexpr (T >= ntri(CLS)) {
    return 0.0;
  } else {
    const double r = tri_row<CLS, T, MASS>(u);
    const double t = MASS ? r : w(TriF<CLS, T, 0>::v, TriF<CLS, T, 1>::v) * r;
    return t + tri_sum<CLS, T + 1, MASS>(w, u);
  }
}

template <bool MASS, typename W, typename U>
__device__ __forceinline__ double row(int cls, const W& w, const U& u) {
  switch (cls) {
    case 0: return tri_sum<0, 0, MASS>(w, u);
    case 1: return tri_sum<1, 0, MASS>(w, u);
    case 2: return tri_sum<2, 0, MASS>(w, u);
    default: return tri_sum<3, 0, MASS>(w, u);
  }
}

// K u at half-grid node (x, y) of P2 mesh level lm (n_c 2^lm cells per side): the
// coefficient is 1 (kind 0) or constant per coarse cell (kind 1).  u(dx, dy) returns the
// value at the node offset by (dx, dy) (0 off the tile or outside the domain).
template <int KIND, typename U>
__device__ __forceinline__ double apply_k(const ProbDev& P, int lm, int x, int y, const U& u) {
  const int cls = (x & 1) | ((y & 1) << 1);
  const int a = x >> 1, b = y >> 1;
  auto w = [&](int di, int dj) -> double {
    if constexpr (KIND == 0) {
      return 1.0;
    } else {
      const gconst_double* k = (const gconst_double*)P.kH;
      return k[((b + dj) >> lm) * P.n_c + ((a + di) >> lm)];
    }
  };
  return row<false>(cls, w, u) * (1.0 / 6.0);
}

// M u at half-grid node (x, y), with h2 = (mesh size)^2 of the level.
template <typename U>
__device__ __forceinline__ double apply_m(int x, int y, double h2, const U& u) {
  const int cls = (x & 1) | ((y & 1) << 1);
  auto w = [](int, int) -> double { return 1.0; };
  return row<true>(cls, w, u) * (h2 * (1.0 / 360.0));
}

// Diagonal of K at a node (the coefficient of u at the node itself).
template <int KIND>
__device__ __forceinline__ double diag_k(const ProbDev& P, int lm, int x, int y) {
  return apply_k<KIND>(P, lm, x, y, [](int dx, int dy) -> double {
    return (dx == 0 && dy == 0) ? 1.0 : 0.0;
  });
}

// The six P2 shape functions at barycentric coordinates (l0, l1, l2).
__device__ __forceinline__ void shape(double l0, double l1, double l2, double (&f)[6]) {
  f[0] = l0 * (2.0 * l0 - 1.0);
  f[1] = l1 * (2.0 * l1 - 1.0);
  f[2] = l2 * (2.0 * l2 - 1.0);
  f[3] = 4.0 * l0 * l1;
  f[4] = 4.0 * l1 * l2;
  f[5] = 4.0 * l2 * l0;
}

// Where a point of a finer half grid lies in the cells of a coarse mesh (nc cells per side):
// the point (x, y) in units of 1/R of a coarse cell; cell (I, J), the triangle (points on
// the diagonal count as lower) and the barycentric coordinates, all exact dyadic values.
struct Loc {
  int I, J, up;
  double l0, l1, l2;
};
__device__ __forceinline__ Loc locate(int x, int y, int R, int shift, int nc) {
  Loc L;
  L.I = min(x >> shift, nc - 1);
  L.J = min(y >> shift, nc - 1);
  const int p = x - (L.I << shift), q = y - (L.J << shift);
  const double inv = 1.0 / (double)R;
  L.up = p < q ? 1 : 0;
  if (!L.up) {  // lower: v0 = SW, v1 = SE, v2 = NE
    L.l0 = (double)(R - p) * inv;
    L.l1 = (double)(p - q) * inv;
    L.l2 = (double)q * inv;
  } else {      // upper: v0 = SW, v1 = NE, v2 = NW
    L.l0 = (double)(R - q) * inv;
    L.l1 = (double)p * inv;
    L.l2 = (double)(q - p) * inv;
  }
  return L;
}

// Half-grid index offsets (on the coarse half grid) of local node b of the cell's triangle.
__device__ __forceinline__ int node_dx_rt(int up, int b) {
  const int lo = 0x121220;  // nibbles b = 0..5: 0 2 2 1 2 1 (lower)
  const int hi = 0x011020;  //                   0 2 0 1 1 0 (upper)
  return ((up ? hi : lo) >> (4 * b)) & 0xf;
}
__device__ __forceinline__ int node_dy_rt(int up, int b) {
  const int lo = 0x110200;  // 0 0 2 0 1 1
  const int hi = 0x121220;  // 0 2 2 1 2 1
  return ((up ? hi : lo) >> (4 * b)) & 0xf;
}

}  // namespace p2
