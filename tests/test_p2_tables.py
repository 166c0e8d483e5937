"""The P2 stencils and interpolation of the GPU path, checked on the host against the
oracle: the device helpers of p2_ops.h (element tables, the triangles around each node
class, point location and shape functions) are compiled for the CPU with g++ (stub
definitions stand in for the HIP header), a driver applies them as the kernels do, and
the matrices it prints must equal the oracle's P2 assembly and interpolation."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W
from oracle import fem_p2
from oracle.fem import triangle_kappa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1401_4969_amd", "csrc")

STUB = r"""
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdint>
#define __device__
#define __host__
#define __forceinline__ inline
using std::min;
typedef const double gconst_double;
struct ProbDev { int n_c; const double* kH; };
"""

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "p2_ops.h"
// argv: n (mesh cells per side), kind, side; stdin: n_c*n_c kappa values when kind = 1
int main(int argc, char** argv) {
  const int n = atoi(argv[1]), kind = atoi(argv[2]), nc = atoi(argv[3]);
  const double side = atof(argv[4]);
  std::vector<double> kap(nc * nc, 1.0);
  if (kind == 1) for (auto& v : kap) if (scanf("%lf", &v) != 1) return 2;
  ProbDev P{nc, kap.data()};
  int lm = 0;
  while ((nc << lm) < n) ++lm;
  const int g = 2 * n, n1 = g + 1;
  const double h = side / n;
  // K and M rows of every node at least one half step inside the grid (their triangles
  // all lie in the box), against the unit vector of every node within two half steps
  for (int y = 1; y < g; ++y)
    for (int x = 1; x < g; ++x)
      for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
          const int jx = x + dx, jy = y + dy;
          if (jx < 0 || jy < 0 || jx > g || jy > g) continue;
          auto e = [&](int ox, int oy) -> double { return (ox == dx && oy == dy) ? 1.0 : 0.0; };
          const double k = kind == 0 ? p2::apply_k<0>(P, lm, x, y, e) : p2::apply_k<1>(P, lm, x, y, e);
          const double m = p2::apply_m(x, y, h * h, e);
          if (k != 0.0 || m != 0.0)
            printf("A %d %d %.17g %.17g\n", y * n1 + x, jy * n1 + jx, k, m);
        }
  // interpolation from the mesh of n/2 cells: fine node -> six coarse nodes and weights
  const int nh = n / 2, c1 = 2 * nh + 1;
  for (int y = 0; y <= g; ++y)
    for (int x = 0; x <= g; ++x) {
      const p2::Loc L = p2::locate(x, y, 4, 2, nh);
      double f[6];
      p2::shape(L.l0, L.l1, L.l2, f);
      for (int b = 0; b < 6; ++b)
        if (f[b] != 0.0)
          printf("P %d %d %.17g\n", y * n1 + x,
                 (2 * L.J + p2::node_dy_rt(L.up, b)) * c1 + 2 * L.I + p2::node_dx_rt(L.up, b), f[b]);
    }
  return 0;
}
"""


def _run(tmp_path, n, kind, nc, side, kap=None):
    (tmp_path / "mlc_device.h").write_text(STUB)
    shutil.copy(os.path.join(CSRC, "p2_ops.h"), tmp_path / "p2_ops.h")
    (tmp_path / "drv.cpp").write_text(DRIVER)
    exe = tmp_path / "drv"
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", str(tmp_path), "-o", str(exe),
                    str(tmp_path / "drv.cpp")], check=True)
    inp = "" if kap is None else " ".join(repr(float(v)) for v in np.asarray(kap).ravel())
    out = subprocess.run([str(exe), str(n), str(kind), str(nc), repr(side)], input=inp,
                         capture_output=True, text=True, timeout=120, check=True).stdout
    A, Pm = {}, {}
    for line in out.splitlines():
        t = line.split()
        if t[0] == "A":
            A[(int(t[1]), int(t[2]))] = (float(t[3]), float(t[4]))
        else:
            Pm[(int(t[1]), int(t[2]))] = Pm.get((int(t[1]), int(t[2])), 0.0) + float(t[3])
    return A, Pm


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("domain,nc,L,kind", [(0, 2, 1, 0), (0, 2, 2, 1), (2, 3, 1, 1),
                                               (1, 4, 1, 0)])
def test_p2_stencils_and_interpolation_match_oracle(tmp_path, domain, nc, L, kind):
    rng = np.random.Generator(np.random.PCG64(90 + nc + L + kind))
    kap = W.loguniform_coarse_kappa(nc, rng) if kind == 1 else None
    prob = W.Problem(domain, nc, L, 1, 1, 1, 1, kind, kap, order=2)
    n = prob.n_cells(L)
    A, Pm = _run(tmp_path, n, kind, nc, prob.side, kap)
    mesh = fem_p2.make_mesh_p2(domain, n, prob.side, prob.origin)
    K, M = fem_p2.assemble_p2(mesh, triangle_kappa(mesh, kind, kap, nc))
    K = K.tocsr()
    M = M.tocsr()
    d = set(mesh.dof.tolist())
    scale_k = abs(K).max()
    scale_m = abs(M).max()
    # every interior row: the stencil entries equal the oracle's, and no entry is missing
    for r in mesh.dof:
        row_k = {int(c): v for c, v in zip(K.indices[K.indptr[r]:K.indptr[r + 1]],
                                           K.data[K.indptr[r]:K.indptr[r + 1]])}
        row_m = {int(c): v for c, v in zip(M.indices[M.indptr[r]:M.indptr[r + 1]],
                                           M.data[M.indptr[r]:M.indptr[r + 1]])}
        cols = set(row_k) | {c for (a, c) in A if a == r}
        for c in cols:
            gk, gm = A.get((int(r), c), (0.0, 0.0))
            assert abs(gk - row_k.get(c, 0.0)) <= 1e-14 * scale_k, (r, c, gk, row_k.get(c))
            assert abs(gm - row_m.get(c, 0.0)) <= 1e-14 * scale_m, (r, c, gm, row_m.get(c))
    # interpolation from the mesh of n/2 cells, on interior rows and columns
    coarse = fem_p2.make_mesh_p2(domain, n // 2, prob.side, prob.origin)
    Po = fem_p2.interpolation_p2(domain, coarse, mesh, prob.side).tocoo()
    want = {(int(mesh.dof[i]), int(coarse.dof[j])): v for i, j, v in zip(Po.row, Po.col, Po.data)}
    cd = set(coarse.dof.tolist())
    got = {k: v for k, v in Pm.items() if k[0] in d and k[1] in cd}
    # (the oracle locates points in floating point: with a non-dyadic h its barycentric
    # coordinates carry rounding, so it may list entries of size ~1e-16 the device omits)
    for k in set(got) | set(want):
        assert abs(got.get(k, 0.0) - want.get(k, 0.0)) < 1e-14, (k, got.get(k), want.get(k))
