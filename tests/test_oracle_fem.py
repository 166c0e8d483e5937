"""Pins for the oracle's finite element layer (CPU only).

Every check compares the oracle against something other than itself: the
textbook five-point Laplacian, a quadrature of the P1 functions evaluated by
barycentric interpolation, the closed form of a hat function on this mesh, and
direct assembly on the coarse mesh with averaged coefficients.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.fem import assemble, interpolation, make_mesh, triangle_kappa, barycentric

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _tridiag(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])


@pytest.mark.parametrize("n", [4, 7])
def test_stiffness_is_five_point_laplacian(n):
    """kappa == 1 on the unit square: P1 stiffness on the SW-NE mesh equals the
    five-point finite difference Laplacian kron(I,T)+kron(T,I) (no h scaling in 2-D)."""
    mesh = make_mesh(0, n, 1.0, 0.0)
    K, _ = assemble(mesh, np.ones(mesh.tri.shape[0]))
    Kd = K[mesh.dof][:, mesh.dof].toarray()
    T = _tridiag(n - 1)
    ref = (sp.kron(sp.identity(n - 1), T) + sp.kron(T, sp.identity(n - 1))).toarray()
    assert np.allclose(Kd, ref, atol=1e-14)


def _tri_gradients_by_legs(mesh, u):
    """Gradient of the P1 function on each triangle from finite differences along
    the two legs of the right triangle (independent of the assembly formula)."""
    n1 = mesh.n + 1
    t = mesh.tri
    h = mesh.h
    g = np.empty((t.shape[0], 2))
    low = ~mesh.tri_upper
    # lower triangle (sw, se, ne): d/dx along sw->se, d/dy along se->ne
    g[low, 0] = (u[t[low, 1]] - u[t[low, 0]]) / h
    g[low, 1] = (u[t[low, 2]] - u[t[low, 1]]) / h
    up = mesh.tri_upper
    # upper triangle (sw, ne, nw): d/dy along sw->nw, d/dx along nw->ne
    g[up, 1] = (u[t[up, 2]] - u[t[up, 0]]) / h
    g[up, 0] = (u[t[up, 1]] - u[t[up, 2]]) / h
    assert n1 > 0
    return g


@pytest.mark.parametrize("domain,n,side,origin", [(0, 6, 1.0, 0.0), (1, 8, 2.0, -1.0)])
def test_stiffness_energy_random_kappa(domain, n, side, origin):
    """u^T K u = sum_T kappa_T |T| |grad u_T|^2 for random nodal u and random
    per-triangle kappa; hypotenuse (SW-NE) couplings vanish."""
    rng = np.random.default_rng(1)
    mesh = make_mesh(domain, n, side, origin)
    kt = np.exp(rng.normal(size=mesh.tri.shape[0]))
    K, _ = assemble(mesh, kt)
    u = rng.normal(size=mesh.n_nodes)
    g = _tri_gradients_by_legs(mesh, u)
    energy = np.sum(kt * 0.5 * mesh.h ** 2 * (g ** 2).sum(axis=1))
    assert u @ (K @ u) == pytest.approx(energy, rel=1e-12)
    n1 = n + 1
    for j in range(n):
        for i in range(n):
            a = j * n1 + i
            assert abs(K[a, a + n1 + 1]) < 1e-14
            assert K[a + 1, a + n1] == 0.0  # SE-NW is not an edge of this mesh


def _duffy_rule(order=6):
    """Quadrature on the reference triangle from a collapsed tensor Gauss-Legendre rule."""
    x, w = np.polynomial.legendre.leggauss(order)
    x = 0.5 * (x + 1)
    w = 0.5 * w
    s, t = np.meshgrid(x, x, indexing="ij")
    ws, wt = np.meshgrid(w, w, indexing="ij")
    l1 = s.ravel()
    l2 = (t * (1 - s)).ravel()
    wts = (ws * wt * (1 - s)).ravel()
    return l1, l2, wts   # integrates over {l1,l2 >= 0, l1+l2 <= 1} (area 1/2)


def _quad_inner(mesh, u, v):
    l1, l2, wq = _duffy_rule()
    p = mesh.xy[mesh.tri]
    d1 = p[:, 1] - p[:, 0]
    d2 = p[:, 2] - p[:, 0]
    det = np.abs(d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0])
    total = 0.0
    for a, b, w in zip(l1, l2, wq):
        pts = p[:, 0] + a * d1 + b * d2
        bc = barycentric(mesh, np.arange(mesh.tri.shape[0]), pts)
        uq = (bc * u[mesh.tri]).sum(axis=1)
        vq = (bc * v[mesh.tri]).sum(axis=1)
        total += w * np.sum(det * uq * vq)
    return total


@pytest.mark.parametrize("domain,n,side,origin", [(0, 5, 1.0, 0.0), (1, 6, 2.0, -1.0)])
def test_mass_matches_quadrature(domain, n, side, origin):
    """u^T M v equals the integral of u_h v_h computed by Gauss quadrature."""
    rng = np.random.default_rng(2)
    mesh = make_mesh(domain, n, side, origin)
    _, M = assemble(mesh, np.ones(mesh.tri.shape[0]))
    u = rng.normal(size=mesh.n_nodes)
    v = rng.normal(size=mesh.n_nodes)
    assert u @ (M @ v) == pytest.approx(_quad_inner(mesh, u, v), rel=1e-12)
    one = np.ones(mesh.n_nodes)
    area = 1.0 if domain == 0 else 3.0
    assert one @ (M @ one) == pytest.approx(area, rel=1e-13)


def test_mass_pattern_follows_diagonal():
    """Mass couples SW-NE neighbours (shared hypotenuse) but not SE-NW ones."""
    mesh = make_mesh(0, 4, 1.0, 0.0)
    _, M = assemble(mesh, np.ones(mesh.tri.shape[0]))
    n1 = 5
    a = 1 * n1 + 1
    h2 = mesh.h ** 2
    assert M[a, a] == pytest.approx(h2 / 2)
    assert M[a, a + n1 + 1] == pytest.approx(h2 / 12)
    assert M[a, a - n1 - 1] == pytest.approx(h2 / 12)
    assert M[a, a + n1 - 1] == 0.0


def _hat(s, t):
    """Closed form of the P1 hat function on the SW-NE mesh (unit spacing)."""
    return np.maximum(0.0, 1.0 - np.maximum(np.maximum(np.abs(s), np.abs(t)), np.abs(s - t)))


@pytest.mark.parametrize("domain,nc,side,origin,ratio", [(0, 4, 1.0, 0.0, 2), (0, 3, 1.0, 0.0, 4),
                                                         (1, 4, 2.0, -1.0, 2)])
def test_interpolation_is_hat_function(domain, nc, side, origin, ratio):
    coarse = make_mesh(domain, nc, side, origin)
    fine = make_mesh(domain, nc * ratio, side, origin)
    P = interpolation(coarse, fine).toarray()
    H = coarse.h
    pf = fine.xy[fine.dof]
    for c, node in enumerate(coarse.dof):
        xc, yc = coarse.xy[node]
        ref = _hat((pf[:, 0] - xc) / H, (pf[:, 1] - yc) / H)
        assert np.allclose(P[:, c], ref, atol=1e-14)


def test_galerkin_equals_child_average():
    """P^T K_h P equals the coarse stiffness assembled with, on each coarse triangle,
    the mean kappa of the fine triangles it contains (children found by locating
    fine-triangle centroids)."""
    rng = np.random.default_rng(3)
    for domain, nc, side, origin in [(0, 4, 1.0, 0.0), (1, 4, 2.0, -1.0)]:
        coarse = make_mesh(domain, nc, side, origin)
        fine = make_mesh(domain, 2 * nc, side, origin)
        kf = np.exp(rng.normal(size=fine.tri.shape[0]))
        Kf, _ = assemble(fine, kf)
        P = interpolation(coarse, fine)
        KG = (P.T @ Kf[fine.dof][:, fine.dof] @ P).toarray()
        cen = fine.xy[fine.tri].mean(axis=1)
        from oracle.fem import locate
        t, _ = locate(coarse, cen)
        kc = np.bincount(t, weights=kf, minlength=coarse.tri.shape[0]) / np.bincount(
            t, minlength=coarse.tri.shape[0])
        Kc, _ = assemble(coarse, kc)
        assert np.allclose(KG, Kc[coarse.dof][:, coarse.dof].toarray(), rtol=1e-12, atol=1e-12)


def test_lshape_interior_nodes():
    """On the L-shape, nodes on the re-entrant sides are boundary nodes."""
    mesh = make_mesh(1, 4, 2.0, -1.0)
    # interior nodes of (-1,1)^2 with 4 cells: (i,j) in 1..3; removed: x>=0 and y<=0
    want = [j * 5 + i for j in range(1, 4) for i in range(1, 4) if not (i >= 2 and j <= 2)]
    assert mesh.dof.tolist() == want


def test_triangle_kappa_layouts():
    mesh = make_mesh(0, 8, 1.0, 0.0)
    kc = np.arange(16.0).reshape(4, 4) + 1
    kt = triangle_kappa(mesh, 1, kc, 4)
    J = mesh.tri_cell // 8
    I = mesh.tri_cell % 8
    assert np.all(kt == kc[J // 2, I // 2])
