"""Pins for the oracle's multilevel correction (CPU only).

What fixes the expected values here, none of which is the oracle itself:
  * lambda_1 = 2 pi^2 on the unit square and the O(h^2) rate of P1 (Section 3,
    a-priori estimates; Table 1 orders ~2), the O(h) H^1 rate (Table 2 orders ~1)
    against the exact eigenfunction 2 sin(pi x) sin(pi y);
  * the min-max principle (Section 3): every Rayleigh-Ritz value on a subspace of
    V_0h lies above the direct discrete eigenvalue;
  * special cases: one subdomain covering the domain (the correction is one
    inverse-iteration step, checked with a global sparse solve and an independent
    orthonormal-basis Rayleigh-Ritz), an exact eigenpair as input (zero residual,
    fixed point), degree-1 homogeneity in kappa;
  * the partition of unity sums to one and each chi_j vanishes outside Omega_j.
Tests that plant a mistake in a copy of the oracle check that these pins catch it.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import workloads as W
from oracle import mlc
from oracle.mlc import Hierarchy, correction, direct_eigs, solve

TWO_PI2 = 2 * np.pi ** 2


@pytest.fixture(scope="module")
def c1():
    p = W.config1()
    return p, solve(p)


def test_direct_eigenvalue_rate():
    """(lambda_1,h - 2 pi^2)/h^2 settles (P1 O(h^2) convergence from above)."""
    p = W.Problem(0, 8, 3, 1, 1, 1, 1, 0, None)
    hier = Hierarchy(p)
    c = []
    for m in range(hier.L + 1):
        lam, _ = direct_eigs(hier, m, 1)
        h = p.h(m)
        assert lam[0] > TWO_PI2
        c.append((lam[0] - TWO_PI2) / h ** 2)
    c = np.array(c)
    # the constant converges (differences shrink by ~4) to about 48.7
    d = np.abs(np.diff(c))
    assert np.all(d[1:] < 0.4 * d[:-1])
    assert 48.6 < c[-1] < 48.9


def test_multilevel_above_direct_and_close(c1):
    p, res = c1
    hier = res.hier
    prev_gap = None
    for m, lam in enumerate(res.lam_levels):
        lam_h, _ = direct_eigs(hier, m, p.n_eig)
        gap = lam[0] - lam_h[0]
        assert gap >= -1e-12 * lam_h[0], "min-max: RR on a subspace of V_0h is above lambda_h"
        if m >= 1:
            assert gap / lam_h[0] < 1e-4
        if prev_gap is not None and m >= 2:
            assert gap < prev_gap
        prev_gap = gap


def test_multilevel_rate_to_2pi2():
    """lambda_ML - 2 pi^2 falls by ~4 per level (order ~2, as Table 1)."""
    p = W.Problem(0, 8, 3, 4, 4, 1, 1, 0, None)
    res = solve(p)
    err = np.array([l[0] - TWO_PI2 for l in res.lam_levels])
    assert np.all(err > 0)
    order = np.log2(err[:-1] / err[1:])
    assert np.all(order[1:] > 1.9) and np.all(order < 2.1)


def _duffy_rule(order=5):
    x, w = np.polynomial.legendre.leggauss(order)
    x = 0.5 * (x + 1)
    w = 0.5 * w
    s, t = np.meshgrid(x, x, indexing="ij")
    ws, wt = np.meshgrid(w, w, indexing="ij")
    return s.ravel(), (t * (1 - s)).ravel(), (ws * wt * (1 - s)).ravel()


def _h1_error(hier, m, u_dof):
    """|u - u_h|_1 for u = 2 sin(pi x) sin(pi y) (b-normalised, lambda = 2 pi^2) using
    a(u, u_h) = lambda (u, u_h) (integration by parts; u_h vanishes on the boundary)."""
    mesh = hier.meshes[m]
    uh = hier.to_grid(m, u_dof)
    p = mesh.xy[mesh.tri]
    d1 = p[:, 1] - p[:, 0]
    d2 = p[:, 2] - p[:, 0]
    det = np.abs(d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0])
    l1, l2, wq = _duffy_rule()
    inner = 0.0
    for a, b, w in zip(l1, l2, wq):
        pts = p[:, 0] + a * d1 + b * d2
        bc = np.stack([1 - a - b, a, b])
        uhq = (uh[mesh.tri] * bc).sum(axis=1)
        uq = 2 * np.sin(np.pi * pts[:, 0]) * np.sin(np.pi * pts[:, 1])
        inner += w * np.sum(det * uq * uhq)
    lam_uh = u_dof @ (hier.K[m] @ u_dof)
    return np.sqrt(max(TWO_PI2 - 2 * TWO_PI2 * inner + lam_uh, 0.0))


def test_h1_rate_order_one():
    """|u - u_h|_1 halves per level (order ~1, as Table 2)."""
    p = W.Problem(0, 8, 3, 4, 4, 1, 1, 0, None)
    res = solve(p)
    e = np.array([_h1_error(res.hier, m, U[:, 0]) for m, U in enumerate(res.U_levels)])
    order = np.log2(e[:-1] / e[1:])
    assert np.all(order[1:] > 0.95) and np.all(order < 1.05)


def test_b_orthonormal_output():
    p = W.small_ragged()
    res = solve(p)
    hier = res.hier
    for m, U in enumerate(res.U_levels):
        G = U.T @ (hier.M[m] @ U)
        assert np.allclose(G, np.eye(p.n_eig), atol=1e-11)
        lam = np.diag(U.T @ (hier.K[m] @ U))
        assert np.allclose(lam, res.lam_levels[m], rtol=1e-11)


@pytest.mark.parametrize("pou", [0, 1, 2])
def test_single_subdomain_is_inverse_iteration(pou):
    """m = 1: Omega_1 = Omega, so u~ = lambda K^-1 M (I u_k) whatever the gluing (with the
    paper's gluing the interface problem on the boundary strip is solved by the
    restriction of the global solution); the Ritz values on V_0H + span{u~} from an
    independent M-orthonormal basis must agree."""
    p = W.Problem(0, 6, 2, 1, 1, 1, 2, 1, np.exp(np.random.default_rng(4).normal(size=(6, 6))),
                  pou=pou)
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


@pytest.mark.parametrize("pou", [0, 1, 2])
def test_covering_subdomains_give_inverse_iteration(pou):
    """Every Omega_j = Omega (overlap = n_coarse): each e^j is the global solution K^-1 r,
    so every gluing returns u~ = I u + K^-1 r whatever the partition (for the paper's
    gluing the interface problem's Dirichlet data then match the global solution)."""
    p = W.Problem(1, 8, 2, 3, 2, 8, 1, 1, np.exp(np.random.default_rng(5).normal(size=(8, 8))),
                  pou=pou)
    hier = Hierarchy(p)
    lam0, U0 = mlc.coarse_eigs(hier, 1)
    _, _, aux = correction(hier, 0, lam0, U0)
    K = hier.K[1].tocsc()
    e = spla.spsolve(K, aux["rhs"][:, 0])
    assert np.allclose(aux["ut"][:, 0], aux["ubar"][:, 0] + e, rtol=1e-10, atol=1e-12)


def test_exact_eigenpair_is_fixed_point():
    """Zero residual: with an exact discrete eigenpair as input and no refinement,
    e^j = 0 and the correction returns the same eigenpair."""
    p = W.Problem(0, 6, 1, 3, 3, 1, 1, 1, np.exp(np.random.default_rng(5).normal(size=(6, 6))))
    hier = Hierarchy(p)
    lam, U = direct_eigs(hier, 1, 1)
    lam2, U2, aux = correction(hier, 1, lam, U, refine=False)
    assert np.max(np.abs(aux["rhs"])) < 1e-10
    assert lam2[0] == pytest.approx(lam[0], rel=1e-12)
    assert abs(U2[:, 0] @ (hier.M[1] @ U[:, 0])) == pytest.approx(1.0, abs=1e-10)


def test_homogeneity_in_kappa():
    """lambda(c kappa) = c lambda(kappa): the method is degree-1 homogeneous in kappa."""
    p = W.small_ragged()
    a = solve(p).lam
    b = solve(p.with_(kappa=3.25 * p.kappa)).lam
    assert np.allclose(b, 3.25 * a, rtol=1e-11)


def test_sign_equivariance():
    """Flipping the input eigenvector leaves the corrected eigenvalue unchanged."""
    p = W.small_ragged()
    hier = Hierarchy(p)
    lam0, U0 = mlc.coarse_eigs(hier, 2)
    a, Ua, _ = correction(hier, 0, lam0, U0)
    b, Ub, _ = correction(hier, 0, lam0, -U0)
    assert np.allclose(a, b, rtol=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_partition_of_unity(seed):
    p = W.random_problem(seed)
    hier = Hierarchy(p)
    m = hier.L
    chi = hier.pou(m)
    assert np.allclose(chi.sum(axis=0), 1.0, atol=1e-15)
    n_in = 0
    for s, c in zip(hier.subs, chi):
        idx = hier.tile_dofs(m, s)
        outside = np.ones(hier.n_dof(m), dtype=bool)
        outside[idx] = False
        assert np.all(c[outside] == 0.0)
        assert np.all((c >= 0) & (c <= 1))
        n_in += idx.size
    assert n_in >= hier.n_dof(m)


@pytest.mark.parametrize("overlap", [0, 1, 2])
def test_partition_of_unity_indicator(overlap):
    """Indicator weights: chi_j = 1/(number of closed D_l holding the node) on the closed
    D_j, 0 elsewhere; they sum to one at every node."""
    p = W.Problem(1, 12, 2, 3, 4, overlap, 1, 0, None, pou=1)
    hier = Hierarchy(p)
    m = hier.L
    chi = hier.pou(m)
    assert np.allclose(chi.sum(axis=0), 1.0, atol=1e-15)
    mesh = hier.meshes[m]
    H = p.side / p.n_coarse
    xs = (mesh.xy[mesh.dof, 0] - p.origin) / H   # node coordinates in coarse-cell units
    ys = (mesh.xy[mesh.dof, 1] - p.origin) / H
    count = np.zeros(chi.shape[1])
    for s in hier.subs:
        inside = (xs >= s.D[0] - 1e-12) & (xs <= s.D[1] + 1e-12) & (ys >= s.D[2] - 1e-12) & (ys <= s.D[3] + 1e-12)
        count += inside
    for s, c in zip(hier.subs, chi):
        inside = (xs >= s.D[0] - 1e-12) & (xs <= s.D[1] + 1e-12) & (ys >= s.D[2] - 1e-12) & (ys <= s.D[3] + 1e-12)
        assert np.all(c[~inside] == 0.0)
        assert np.allclose(c[inside], 1.0 / count[inside])


def test_gluing_overlap_sensitivity():
    """Every gluing keeps u~ in V_0h, so the multilevel eigenvalue stays above the direct
    discrete one at every level (min-max, Section 3).  Without overlap (indicator gluing,
    Omega_j = D_j) the correction stalls near 1e-3 of the direct eigenvalue; with one or
    two coarse cells of overlap it converges to it (the paper's sensitivity experiments:
    the overlap must not be too small)."""
    final = {}
    for ov, pou in [(0, 1), (1, 0), (1, 1), (2, 0), (2, 1), (0, 2), (1, 2)]:
        p = W.Problem(0, 8, 3, 4, 4, ov, 1, 0, None, pou=pou)
        res = solve(p)
        errs = []
        for k, lv in enumerate(res.lam_levels):
            d = direct_eigs(res.hier, k, 1)[0][0]
            errs.append((lv[0] - d) / d)
        assert min(errs) >= -1e-13, (ov, pou, errs)
        final[(ov, pou)] = errs[-1]
    assert final[(0, 1)] > 1e-4
    for key in [(1, 0), (1, 1), (2, 0), (2, 1), (0, 2), (1, 2)]:
        assert final[key] < 1e-6, (key, final[key])
        assert final[(0, 1)] > 100 * final[key]


def test_lshape_first_eigenvalue_sane():
    """L-shape, kappa = 1: lambda_1 approaches 9.6397 (a literature value for this
    domain) slowly from above, because of the re-entrant corner."""
    p = W.Problem(1, 8, 2, 2, 2, 1, 1, 0, None)
    res = solve(p)
    lam = res.lam_levels[-1][0]
    assert 9.6397 < lam < 9.6397 * 1.03


def test_config2_levels_against_direct():
    """Configuration 2 (q = 3): every level stays above the direct eigenvalues and the
    gap shrinks faster than the discretisation error."""
    p = W.config2().with_(n_refine=3)
    res = solve(p)
    for m, lam in enumerate(res.lam_levels):
        lam_h, _ = direct_eigs(res.hier, m, 3)
        assert np.all(lam >= lam_h * (1 - 1e-12))
        if m >= 2:
            assert np.all((lam - lam_h) / lam_h < 1e-4)


# --- planted mistakes: the pins above must catch them --------------------------------

def _planted_rhs_sign(hier, k, lam_k, u_k, refine=True):
    m = k + 1
    ubar = hier.P[k] @ u_k
    rhs = hier.K[m] @ ubar - (hier.M[m] @ ubar) * lam_k[None, :]   # wrong sign
    chi = hier.pou(m)
    ut = ubar.copy()
    for (idx, e_j), chi_j in zip(mlc.local_solves(hier, m, rhs), chi):
        ut[idx] += chi_j[idx, None] * e_j
    mu, U, _ = mlc.rayleigh_ritz(hier, m, ut, lam_k.size)
    return mu, mlc.sign_normalise(U), {}


def _planted_no_normalisation(hier, k, lam_k, u_k, refine=True):
    m = k + 1
    ubar = hier.P[k] @ u_k
    rhs = (hier.M[m] @ ubar) * lam_k[None, :] - hier.K[m] @ ubar
    ut = ubar.copy()
    for idx, e_j in mlc.local_solves(hier, m, rhs):
        ut[idx] += e_j       # sum of local corrections without the partition of unity
    mu, U, _ = mlc.rayleigh_ritz(hier, m, ut, lam_k.size)
    return mu, mlc.sign_normalise(U), {}


@pytest.mark.parametrize("planted", [_planted_rhs_sign, _planted_no_normalisation])
def test_pins_catch_planted_mistakes(monkeypatch, planted):
    p = W.Problem(0, 8, 3, 4, 4, 1, 1, 0, None)
    monkeypatch.setattr(mlc, "correction", planted)
    res = mlc.solve(p)
    err = np.array([l[0] - TWO_PI2 for l in res.lam_levels])
    lam_h, _ = direct_eigs(res.hier, 3, 1)
    rate_ok = np.all(np.log2(err[:-1] / err[1:])[1:] > 1.9)
    close_ok = (res.lam_levels[-1][0] - lam_h[0]) / lam_h[0] < 1e-4
    assert not (rate_ok and close_ok)


def test_example62_multilevel():
    """Example 6.2 with H = 0.1 (20 coarse cells on (-1,1)^2), 2 x 2 subdomains and four
    level grids (three corrections): the six multilevel eigenvalues lie above the direct
    discrete ones (min-max) and within 1e-7 of them."""
    import workloads as W
    prob = W.example62(n_refine=3, sub=2, n_eig=6)
    hier = Hierarchy(prob)
    res = solve(prob, hier)
    lam_h = direct_eigs(hier, 3, 6)[0]
    rel = (res.lam - lam_h) / lam_h
    assert np.all(rel >= -1e-12), rel
    assert np.all(rel < 1e-7), rel
    # every level stays above the direct eigenvalues of its own mesh
    for k, lk in enumerate(res.lam_levels):
        assert np.all(lk >= direct_eigs(hier, k, 6)[0] * (1 - 1e-12))
