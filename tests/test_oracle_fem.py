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


# ---- coefficient kind 3: full tensor A and weighted mass (Example 6.2) ----

def _random_tensor(mesh, seed):
    rng = np.random.default_rng(seed)
    T = mesh.tri.shape[0]
    a11 = np.exp(rng.normal(size=T))
    a22 = np.exp(rng.normal(size=T))
    a12 = rng.uniform(-0.9, 0.9, size=T) * np.sqrt(a11 * a22)
    A = np.empty((T, 2, 2))
    A[:, 0, 0], A[:, 0, 1], A[:, 1, 0], A[:, 1, 1] = a11, a12, a12, a22
    return A, np.exp(rng.normal(size=T))


@pytest.mark.parametrize("domain,n,side,origin", [(0, 6, 1.0, 0.0), (2, 6, 2.0, -1.0),
                                                  (1, 8, 2.0, -1.0)])
def test_tensor_stiffness_energy(domain, n, side, origin):
    """u^T K u = sum_T |T| g_T . A_T g_T with the gradient g_T of the P1 function taken
    from differences along the legs, for a random symmetric positive definite A per
    triangle (the tensor form of Example 6.2)."""
    rng = np.random.default_rng(3)
    mesh = make_mesh(domain, n, side, origin)
    A, phi = _random_tensor(mesh, 4)
    K, _ = assemble(mesh, None, A, phi)
    u = rng.normal(size=mesh.n_nodes)
    g = _tri_gradients_by_legs(mesh, u)
    energy = np.sum(0.5 * mesh.h ** 2 * np.einsum("ti,tij,tj->t", g, A, g))
    assert u @ (K @ u) == pytest.approx(energy, rel=1e-12)


def test_tensor_hypotenuse_coupling():
    """With an off-diagonal a12 the SW-NE hypotenuse couples: on a right triangle with
    legs along x and y the coupling of the two acute vertices is -a12/2, so the cell's
    SW and NE nodes couple by -(a12(lower) + a12(upper))/2; SE-NW stays uncoupled."""
    mesh = make_mesh(0, 4, 1.0, 0.0)
    A, phi = _random_tensor(mesh, 5)
    K, _ = assemble(mesh, None, A, phi)
    n1 = 5
    for t in range(0, mesh.tri.shape[0], 2):     # lower, upper of one cell
        cell = mesh.tri_cell[t]
        j, i = divmod(cell, 4)
        a = j * n1 + i
        assert K[a, a + n1 + 1] == pytest.approx(-0.5 * (A[t, 0, 1] + A[t + 1, 0, 1]), rel=1e-13)
        assert K[a + 1, a + n1] == 0.0


@pytest.mark.parametrize("domain,n,side,origin", [(0, 5, 1.0, 0.0), (2, 4, 2.0, -1.0)])
def test_weighted_mass_matches_quadrature(domain, n, side, origin):
    """u^T M v equals sum_T phi_T times the Gauss-quadrature integral of u_h v_h over T."""
    rng = np.random.default_rng(6)
    mesh = make_mesh(domain, n, side, origin)
    A, phi = _random_tensor(mesh, 7)
    _, M = assemble(mesh, None, A, phi)
    u = rng.normal(size=mesh.n_nodes)
    v = rng.normal(size=mesh.n_nodes)
    l1, l2, wq = _duffy_rule()
    p = mesh.xy[mesh.tri]
    d1 = p[:, 1] - p[:, 0]
    d2 = p[:, 2] - p[:, 0]
    det = np.abs(d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0])
    total = 0.0
    for a, b, w in zip(l1, l2, wq):
        bc = barycentric(mesh, np.arange(mesh.tri.shape[0]), p[:, 0] + a * d1 + b * d2)
        total += w * np.sum(phi * det * (bc * u[mesh.tri]).sum(axis=1) * (bc * v[mesh.tri]).sum(axis=1))
    assert u @ (M @ v) == pytest.approx(total, rel=1e-12)


def test_tensor_identity_reduces_to_scalar():
    """A = kappa I and phi = 1 give the matrices of the scalar coefficient kappa."""
    mesh = make_mesh(1, 8, 2.0, -1.0)
    rng = np.random.default_rng(8)
    kt = np.exp(rng.normal(size=mesh.tri.shape[0]))
    A = kt[:, None, None] * np.eye(2)[None]
    K1, M1 = assemble(mesh, kt)
    K3, M3 = assemble(mesh, None, A, np.ones(mesh.tri.shape[0]))
    assert abs(K1 - K3).max() < 1e-13 and abs(M1 - M3).max() < 1e-15


def test_example62_extrapolated_eigenvalues():
    """Example 6.2 (Section 6): A = [[e^(1+x^2), e^(xy)], [e^(xy), e^(1+y^2)]] and
    phi = (1+x^2)(1+y^2) on (-1,1)^2, sampled at the triangle centroids.  The direct
    discrete eigenvalues on two meshes (h = 1/40, 1/80), extrapolated in h^2, reproduce
    the six values the paper prints to its six decimals (relative 2e-7)."""
    import json, os
    import scipy.sparse.linalg as spla
    import workloads as W
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "example62_eigenvalues.json")))["eigenvalues"]
    lam = []
    for n in (80, 160):
        mesh = make_mesh(2, n, 2.0, -1.0)
        from oracle.fem import triangle_tensor
        A, phi = triangle_tensor(mesh, W.example62_coefficients(n))
        K, M = assemble(mesh, None, A, phi)
        d = mesh.dof
        ev = spla.eigsh(K[d][:, d].tocsc(), k=6, M=M[d][:, d].tocsc(), sigma=0.0,
                        which="LM", tol=1e-14)[0]
        lam.append(np.sort(ev))
    ext = (4.0 * lam[1] - lam[0]) / 3.0
    assert np.all(lam[1] > np.array(ref))          # conforming P1 approximates from above
    assert np.max(np.abs(ext - ref) / np.array(ref)) < 2e-7, ext
