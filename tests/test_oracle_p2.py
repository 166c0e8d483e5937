"""Pins of the oracle's P2 elements (CPU only), each against something other than the
oracle's own formulas.

* Element matrices: on every triangle the P2 function with given nodal values is the
  quadratic polynomial through them; the test finds it by solving the 6 x 6 monomial
  system in cell-local coordinates and integrates kappa |grad p|^2 and p^2 exactly with
  the closed form of monomial integrals over the two right triangles of a cell.  No
  barycentric shape function and no quadrature rule is involved.
* Interpolation: every column of the level-to-level interpolation is a coarse basis
  function, found the same monomial way, evaluated at the fine nodes.
* Nested spaces: the Galerkin product P^T K P of the finer level equals the direct
  assembly on the coarser one.
* The P2 eigenvalue converges to 2 pi^2 from above at fourth order (Section 6, the P2
  sensitivity figure: the error order is 2k for P_k); the multilevel eigenvalue keeps
  above the direct one (min-max), and with one subdomain covering the domain a
  correction step is one inverse-iteration step.
* Planted mistakes in the shape functions and the interpolation fail these pins.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import fem_p2
from oracle import mlc
from oracle.fem import triangle_kappa
from oracle.mlc import Hierarchy, correction


def _monomials(x, y):
    """[1, x, y, x^2, xy, y^2] at points (x, y)."""
    return np.stack([np.ones_like(x), x, y, x * x, x * y, y * y], axis=-1)


# exponents (a, b) of the monomials above and of the derivatives' monomials
EXP = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]


def _tri_monomial_integral(a, b, h, upper):
    """Integral of x^a y^b over the cell-local triangle 0 <= y <= x <= h (lower) or
    0 <= x <= y <= h (upper)."""
    return h ** (a + b + 2) / (((a + 1) if upper else (b + 1)) * (a + b + 2))


def _poly_mul_integral(c1, c2, h, upper):
    """Integral of the product of two polynomials given by coefficient dicts."""
    s = 0.0
    for (a1, b1), v1 in c1.items():
        for (a2, b2), v2 in c2.items():
            s += v1 * v2 * _tri_monomial_integral(a1 + a2, b1 + b2, h, upper)
    return s


def _local_quadratic(mesh, t, vals):
    """Coefficients (dict of exponents) of the quadratic through the 6 nodal values of
    triangle t, in coordinates local to its cell's lower-left corner."""
    I = mesh.tri_cell[t] % mesh.n
    J = mesh.tri_cell[t] // mesh.n
    x0 = mesh.origin + I * mesh.h
    y0 = mesh.origin + J * mesh.h
    pts = mesh.xy[mesh.tri[t]] - np.array([x0, y0])
    c = np.linalg.solve(_monomials(pts[:, 0], pts[:, 1]), vals)
    return {e: v for e, v in zip(EXP, c)}


def _grad(coef):
    gx, gy = {}, {}
    for (a, b), v in coef.items():
        if a:
            gx[(a - 1, b)] = gx.get((a - 1, b), 0.0) + a * v
        if b:
            gy[(a, b - 1)] = gy.get((a, b - 1), 0.0) + b * v
    return gx, gy


def _energies(mesh, kt, u):
    """sum over triangles of kappa int |grad p|^2 and of int p^2 for the piecewise
    quadratic p with nodal values u, by exact polynomial integration."""
    ek, em = 0.0, 0.0
    for t in range(mesh.tri.shape[0]):
        c = _local_quadratic(mesh, t, u[mesh.tri[t]])
        up = bool(mesh.tri_upper[t])
        gx, gy = _grad(c)
        ek += kt[t] * (_poly_mul_integral(gx, gx, mesh.h, up) + _poly_mul_integral(gy, gy, mesh.h, up))
        em += _poly_mul_integral(c, c, mesh.h, up)
    return ek, em


@pytest.mark.parametrize("domain,n,side,origin", [(0, 3, 1.0, 0.0), (1, 4, 2.0, -1.0),
                                                  (2, 2, 2.0, -1.0)])
def test_p2_matrices_are_exact_polynomial_integrals(domain, n, side, origin):
    rng = np.random.Generator(np.random.PCG64(70 + domain))
    mesh = fem_p2.make_mesh_p2(domain, n, side, origin)
    kt = np.exp(rng.uniform(-1.0, 1.0, size=mesh.tri.shape[0]))
    K, M = fem_p2.assemble_p2(mesh, kt)
    for _ in range(3):
        u = rng.standard_normal(mesh.n_nodes)
        ek, em = _energies(mesh, kt, u)
        assert abs(u @ (K @ u) - ek) < 1e-12 * abs(ek)
        assert abs(u @ (M @ u) - em) < 1e-12 * abs(em)
    # polarisation: a bilinear form is fixed by its quadratic form; spot-check entries
    for a, b in [(0, 1), (3, 5), (mesh.n_nodes // 2, mesh.n_nodes // 2 + 1)]:
        ea = np.zeros(mesh.n_nodes)
        ea[a] = 1.0
        eb = np.zeros(mesh.n_nodes)
        eb[b] = 1.0
        kp, mp = _energies(mesh, kt, ea + eb)
        km, mm = _energies(mesh, kt, ea - eb)
        assert abs(K[a, b] - (kp - km) / 4) < 1e-12 * max(1.0, abs(K[a, a]))
        assert abs(M[a, b] - (mp - mm) / 4) < 1e-12 * max(1e-3, abs(M[a, a]))


def test_p2_interior_nodes():
    """(2n-1)^2 interior nodes on the square; on the L-shape the nodes of the removed
    quadrant's closure and of the re-entrant edges are not interior."""
    m = fem_p2.make_mesh_p2(0, 4, 1.0, 0.0)
    assert m.dof.size == 7 * 7
    L = fem_p2.make_mesh_p2(1, 4, 2.0, -1.0)
    g = L.grid
    i, j = L.dof % (g + 1), L.dof // (g + 1)
    assert not np.any((i >= g // 2) & (j <= g // 2))
    assert L.dof.size == 7 * 7 - 4 * 4


@pytest.mark.parametrize("domain,nc", [(0, 2), (1, 4), (0, 3)])
def test_p2_interpolation_columns_are_coarse_basis_functions(domain, nc):
    p = W.Problem(domain, nc, 1, 1, 1, 1, 1, 0, None, order=2)
    side, origin = p.side, p.origin
    coarse = fem_p2.make_mesh_p2(domain, nc, side, origin)
    fine = fem_p2.make_mesh_p2(domain, 2 * nc, side, origin)
    P = fem_p2.interpolation_p2(domain, coarse, fine, side).toarray()
    pts = fine.xy[fine.dof]
    from oracle.fem import locate, make_mesh
    t, _ = locate(make_mesh(domain, nc, side, origin), pts)
    for col, node in enumerate(coarse.dof):
        vals = np.zeros(coarse.n_nodes)
        vals[node] = 1.0
        want = np.zeros(pts.shape[0])
        for r in range(pts.shape[0]):
            c = _local_quadratic(coarse, t[r], vals[coarse.tri[t[r]]])
            I = coarse.tri_cell[t[r]] % coarse.n
            J = coarse.tri_cell[t[r]] // coarse.n
            x = pts[r, 0] - (origin + I * coarse.h)
            y = pts[r, 1] - (origin + J * coarse.h)
            want[r] = _monomials(np.array(x), np.array(y)) @ np.array([c[e] for e in EXP])
        assert np.max(np.abs(P[:, col] - want)) < 1e-12, col


@pytest.mark.parametrize("kind", [0, 1])
def test_p2_galerkin_equals_direct_assembly(kind):
    rng = np.random.Generator(np.random.PCG64(71))
    kap = W.loguniform_coarse_kappa(4, rng) if kind == 1 else None
    p = W.Problem(1, 4, 2, 2, 2, 1, 1, kind, kap, order=2)
    hier = Hierarchy(p)
    for m in range(2):
        mesh = hier.meshes[m]
        K, M = fem_p2.assemble_p2(mesh, triangle_kappa(mesh, kind, kap, 4))
        d = mesh.dof
        assert abs(hier.K[m] - K[d][:, d]).max() < 1e-12 * abs(K).max()
        assert abs(hier.M[m] - M[d][:, d]).max() < 1e-12 * abs(M).max()


def test_p2_eigenvalue_fourth_order_from_above():
    """Direct P2 eigenvalues on the unit square, h = 1/4 .. 1/32: above 2 pi^2 and 8 pi^2,
    each halving of h dividing the error by about 16."""
    lam_true = np.array([2.0, 8.0]) * np.pi ** 2
    errs = []
    for n in (4, 8, 16, 32):
        hier = Hierarchy(W.Problem(0, n, 0, 1, 1, 1, 4, 0, None, order=2))
        lam, _ = mlc.direct_eigs(hier, 0, 4)
        e = lam[[0, 3]] - lam_true
        assert np.all(e > 0)
        errs.append(e)
    ratios = [a / b for a, b in zip(errs[:-1], errs[1:])]
    for r in ratios[1:]:
        assert np.all((r > 14.0) & (r < 17.5)), ratios
    assert np.all(np.abs(np.log2(ratios[-1]) - 4.0) < 0.1)


def test_p2_multilevel_above_direct_and_fourth_order():
    """Multilevel P2 correction (H = 1/4, 2 x 2 subdomains as in Example 6.1, overlap one
    coarse cell): every level's eigenvalue lies above the direct one of its mesh and
    within 1e-6 of it, and the error against 2 pi^2 falls by about 16 per level."""
    p = W.Problem(0, 4, 3, 2, 2, 1, 1, 0, None, order=2)
    res = mlc.solve(p)
    hier = res.hier
    errs = []
    for m in range(1, p.n_refine + 1):
        lam_h, _ = mlc.direct_eigs(hier, m, 1)
        lam_ml = res.lam_levels[m][0]
        assert lam_ml >= lam_h[0] * (1 - 1e-13)
        assert (lam_ml - lam_h[0]) / lam_h[0] < 1e-6
        errs.append(lam_ml - 2 * np.pi ** 2)
    r = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all((r > 12.0) & (r < 18.0)), r


@pytest.mark.parametrize("pou", [0, 1])
def test_p2_single_subdomain_is_inverse_iteration(pou):
    """One subdomain covering the domain: u~ = lambda K^-1 M I u on the P2 space, and the
    Ritz values from an independent M-orthonormal basis agree."""
    rng = np.random.Generator(np.random.PCG64(72))
    p = W.Problem(0, 4, 2, 1, 1, 1, 2, 1, W.loguniform_coarse_kappa(4, rng), pou=pou, order=2)
    hier = Hierarchy(p)
    lam0, U0 = mlc.coarse_eigs(hier, 2)
    lam1, U1, aux = correction(hier, 0, lam0, U0)
    K, M = hier.K[1].tocsc(), hier.M[1]
    ut = np.column_stack([lam0[i] * spla.spsolve(K, M @ (hier.P[0] @ U0[:, i])) for i in range(2)])
    assert np.allclose(aux["ut"], ut, rtol=1e-10, atol=1e-12)
    S = np.hstack([hier.P0[1].toarray(), ut])
    Bm = S.T @ (M @ S)
    w, Q = np.linalg.eigh(Bm)
    Bih = Q @ np.diag(w ** -0.5) @ Q.T
    C = Bih @ (S.T @ (K @ S)) @ Bih
    ritz = np.linalg.eigvalsh(0.5 * (C + C.T))[:2]
    assert np.allclose(lam1, ritz, rtol=1e-9)


def test_p2_subdomain_tiles_and_weights():
    """Tile dofs are the P2 nodes strictly inside Omega_j (half-cell node grid), and the
    gluing weights at P2 nodes sum to one."""
    p = W.config1_p2()
    hier = Hierarchy(p)
    m = 2
    s = hier.subs[5]   # an inner block: D = [2,4] x [2,4] coarse cells, Omega = [1,5]^2
    idx = hier.tile_dofs(m, s)
    r = 2 << m         # node-grid intervals per coarse cell
    assert idx.size == (4 * r - 1) ** 2
    chi = hier.pou(m)
    assert np.allclose(chi.sum(axis=0), 1.0)


@pytest.mark.parametrize("planted", ["edge_factor", "vertex_shape", "p1_interp"])
def test_p2_pins_catch_planted_mistakes(monkeypatch, planted):
    """A wrong factor on the edge functions, a wrong vertex function, or P1-style
    interpolation of the vertex values must fail the pins above."""
    good_shape = fem_p2.shape_p2
    if planted == "edge_factor":
        def shape(lam):
            v = good_shape(lam).copy()
            v[..., 3:] *= 0.5
            return v
        monkeypatch.setattr(fem_p2, "shape_p2", shape)
        with pytest.raises(AssertionError):
            test_p2_interpolation_columns_are_coarse_basis_functions(0, 2)
    elif planted == "vertex_shape":
        good_grad = fem_p2.shape_grad_p2

        def grad(lam, g):
            d = good_grad(lam, g).copy()
            d[..., 0, :] = (2 * lam[..., 0, None] - 1) * g[..., 0, :]
            return d
        monkeypatch.setattr(fem_p2, "shape_grad_p2", grad)
        with pytest.raises(AssertionError):
            test_p2_matrices_are_exact_polynomial_integrals(0, 3, 1.0, 0.0)
    else:
        def shape(lam):
            v = np.zeros(lam.shape[:-1] + (6,))
            v[..., :3] = lam
            return v
        monkeypatch.setattr(fem_p2, "shape_p2", shape)
        with pytest.raises(AssertionError):
            test_p2_interpolation_columns_are_coarse_basis_functions(0, 2)
