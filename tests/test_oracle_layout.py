"""Value pins for the oracle's domain decomposition, gluing weights and sign rule (CPU only).

Every expected value below is written out by hand from the readings of the paper's
Section 4 (the blocks D_j of whole coarse cells and their enlargements Omega_j aligned with
T_H) and of Algorithm 4.1 step 2 (the gluing weights), not computed by the oracle:
  * D_j: block boundaries at floor(b n_c / s) coarse cells; Omega_j = D_j grown by the
    overlap on every side and clipped to the bounding box; on the L-shape, a block is
    dropped exactly when none of its coarse cells lies in the domain;
  * phi_j = rho(x) rho(y) with rho = 1 on the closed D_j range, falling linearly to 0 at
    distance delta = overlap (coarse cells) outside it; chi_j = phi_j / sum_l phi_l;
  * the free sign of b-normalised eigenvectors: positive nodal sum, or, for a sum that is
    rounding noise, the first near-largest entry positive.
Tests at the end plant plausible misreadings in the oracle and check that these pins fail.
"""
import numpy as np
import pytest

import workloads as W
from oracle import mlc
from oracle.mlc import Hierarchy

# --- subdomains -----------------------------------------------------------------------

# n_c = 10, 3 x 3 blocks: boundaries floor(10 b / 3) = 0, 3, 6, 10
D_10_3 = [(0, 3), (3, 6), (6, 10)]
OMEGA_10_3 = {1: [(0, 4), (2, 7), (5, 10)],     # grown by one coarse cell, clipped to [0, 10]
              2: [(0, 5), (1, 8), (4, 10)]}     # grown by two


def _expected_square(xr, yr, om_x, om_y):
    return [((xr[a][0], xr[a][1], yr[b][0], yr[b][1]),
             (om_x[a][0], om_x[a][1], om_y[b][0], om_y[b][1]))
            for b in range(len(yr)) for a in range(len(xr))]


def check_subdomain_layout():
    for ov in (1, 2):
        p = W.Problem(0, 10, 1, 3, 3, ov, 1, 0, None)
        got = [(s.D, s.Omega) for s in mlc.subdomains(p)]
        assert got == _expected_square(D_10_3, D_10_3, OMEGA_10_3[ov], OMEGA_10_3[ov]), (ov, got)
    # uneven and different splits per axis: n_c = 10, 4 blocks along x (0, 2, 5, 7, 10),
    # 2 along y (0, 5, 10), overlap 1
    p = W.Problem(0, 10, 1, 4, 2, 1, 1, 0, None)
    xr = [(0, 2), (2, 5), (5, 7), (7, 10)]
    ox = [(0, 3), (1, 6), (4, 8), (6, 10)]
    yr = [(0, 5), (5, 10)]
    oy = [(0, 6), (4, 10)]
    got = [(s.D, s.Omega) for s in mlc.subdomains(p)]
    assert got == _expected_square(xr, yr, ox, oy), got
    # one block covering everything: Omega_1 = D_1 = the whole box
    p = W.Problem(0, 6, 1, 1, 1, 1, 1, 0, None)
    assert [(s.D, s.Omega) for s in mlc.subdomains(p)] == [((0, 6, 0, 6), (0, 6, 0, 6))]


def test_subdomain_layout():
    check_subdomain_layout()


def check_lshape_drop():
    # n_c = 10, 3 x 3: only the block x in [6, 10], y in [0, 3] lies in the removed
    # quadrant (coarse cells with x >= 5 and y < 5); block (1, 0) straddles it and stays
    p = W.Problem(1, 10, 1, 3, 3, 1, 1, 0, None)
    got = [s.D for s in mlc.subdomains(p)]
    want = [(0, 3, 0, 3), (3, 6, 0, 3),
            (0, 3, 3, 6), (3, 6, 3, 6), (6, 10, 3, 6),
            (0, 3, 6, 10), (3, 6, 6, 10), (6, 10, 6, 10)]
    assert got == want, got
    # n_c = 8, 4 x 4 (boundaries 0, 2, 4, 6, 8): the four blocks with x >= 4 and y <= 4 go
    p = W.Problem(1, 8, 1, 4, 4, 1, 1, 0, None)
    got = [s.D for s in mlc.subdomains(p)]
    r = [(0, 2), (2, 4), (4, 6), (6, 8)]
    want = [(a[0], a[1], b[0], b[1]) for b in r for a in r if not (a[0] >= 4 and b[1] <= 4)]
    assert got == want and len(got) == 12, got


def test_lshape_drop_rule():
    check_lshape_drop()


@pytest.mark.parametrize("n, s", [(8, 3), (10, 4), (12, 5), (6, 6)])
def test_lshape_drop_brute_force(n, s):
    """A block is kept exactly when one of its coarse cells has its centre in the L-shape
    (-1,1)^2 minus [0,1)x(-1,0] (cells tested one by one)."""
    p = W.Problem(1, n, 1, s, s, 1, 1, 0, None)
    kept = {s_.D for s_ in mlc.subdomains(p)}
    H = 2.0 / n
    bx = [(b * n) // s for b in range(s + 1)]
    for sy in range(s):
        for sx in range(s):
            D = (bx[sx], bx[sx + 1], bx[sy], bx[sy + 1])
            inside = any(not ((-1 + (i + 0.5) * H) > 0 and (-1 + (j + 0.5) * H) < 0)
                         for i in range(D[0], D[1]) for j in range(D[2], D[3]))
            assert (D in kept) == inside, (D, inside)


# --- gluing weights -------------------------------------------------------------------

def check_ramp_values():
    # D range [3, 6], delta = 1: 0 beyond 1 cell, linear across it, 1 on the closed range
    t = np.array([1.0, 2.0, 2.25, 2.5, 3.0, 4.5, 6.0, 6.5, 6.75, 7.0, 8.0])
    want = np.array([0.0, 0.0, 0.25, 0.5, 1.0, 1.0, 1.0, 0.5, 0.25, 0.0, 0.0])
    assert np.array_equal(mlc.ramp(t, 3.0, 6.0, 1.0), want), mlc.ramp(t, 3.0, 6.0, 1.0)
    # delta = 2
    t = np.array([0.5, 1.0, 2.0, 3.0, 7.0, 8.0, 8.5])
    want = np.array([0.0, 0.0, 0.5, 1.0, 0.5, 0.0, 0.0])
    assert np.array_equal(mlc.ramp(t, 3.0, 6.0, 2.0), want), mlc.ramp(t, 3.0, 6.0, 2.0)


def test_ramp_values():
    check_ramp_values()


def _chi_by_block(prob, pts):
    subs = mlc.subdomains(prob)
    ti = np.array([p[0] for p in pts], dtype=float)
    tj = np.array([p[1] for p in pts], dtype=float)
    chi = mlc.pou_weights(prob, subs, ti, tj)
    return [{s.D: chi[k, i] for k, s in enumerate(subs) if chi[k, i] != 0.0}
            for i in range(len(pts))]


# blocks of n_c = 10, 3 x 3 named by their (x, y) block index
_B = {(a, b): (D_10_3[a][0], D_10_3[a][1], D_10_3[b][0], D_10_3[b][1])
      for a in range(3) for b in range(3)}

# points in coarse-cell units and their weights, worked out by hand (overlap 1)
POU_CASES = [
    ((1.0, 1.0), {(0, 0): 1.0}),                            # inside D_00, away from others
    ((3.0, 1.0), {(0, 0): 0.5, (1, 0): 0.5}),               # on a shared edge: both phi = 1
    ((2.5, 1.0), {(0, 0): 2 / 3, (1, 0): 1 / 3}),           # phi 1 and 1/2
    ((3.5, 1.0), {(0, 0): 1 / 3, (1, 0): 2 / 3}),
    ((2.5, 2.5), {(0, 0): 4 / 9, (1, 0): 2 / 9, (0, 1): 2 / 9, (1, 1): 1 / 9}),
    ((4.5, 5.5), {(1, 1): 2 / 3, (1, 2): 1 / 3}),
    ((6.5, 5.5), {(2, 1): 4 / 9, (1, 1): 2 / 9, (2, 2): 2 / 9, (1, 2): 1 / 9}),
    ((0.0, 9.75), {(0, 2): 1.0}),                           # at the box edge (unclipped ramp)
]


def check_pou_values(domain):
    p = W.Problem(domain, 10, 1, 3, 3, 1, 1, 0, None)
    pts = [c[0] for c in POU_CASES]
    got = _chi_by_block(p, pts)
    for (pt, want), g in zip(POU_CASES, got):
        if domain == 1 and pt[0] > 5 and pt[1] < 5:
            continue
        w = {_B[k]: v for k, v in want.items()}
        assert set(g) == set(w), (pt, g, w)
        for k in w:
            assert abs(g[k] - w[k]) < 1e-15, (pt, k, g[k], w[k])


@pytest.mark.parametrize("domain", [0, 1])
def test_pou_values(domain):
    check_pou_values(domain)


def check_pou_at_nodes():
    """The same weights at mesh nodes (level 1 of n_c = 10: fine node (i, j) sits at coarse
    coordinates (i/2, j/2)) through the hierarchy used by the correction step."""
    p = W.Problem(0, 10, 1, 3, 3, 1, 1, 0, None)
    hier = Hierarchy(p)
    chi = hier.pou(1)
    mesh = hier.meshes[1]
    pos = {int(n): k for k, n in enumerate(mesh.dof)}
    for pt, want in POU_CASES:
        i, j = int(round(2 * pt[0])), int(round(2 * pt[1]))
        node = j * 21 + i
        if node not in pos:
            continue   # boundary node
        col = chi[:, pos[node]]
        got = {s.D: col[k] for k, s in enumerate(hier.subs) if col[k] != 0.0}
        w = {_B[k]: v for k, v in want.items()}
        assert set(got) == set(w), (pt, got, w)
        for k in w:
            assert abs(got[k] - w[k]) < 1e-15


def test_pou_at_nodes():
    check_pou_at_nodes()


# --- sign rule ------------------------------------------------------------------------

SIGN_CASES = [
    # (vector, flipped?)
    ([1.0, 2.0, -0.5], False),                              # positive sum
    ([-1.0, -2.0, 0.5], True),                              # negative sum
    ([-3.0, 1.0, -1.0, 3.0], True),                         # zero sum: first of the tied maxima
    ([3.0, -1.0, 1.0, -3.0], False),
    ([3.0 - 3e-7, -3.0, 0.5, -0.5 + 3e-7], False),          # first entry within 1e-6 of the max
    ([3.0 - 3e-5, -3.0, 0.5, -0.5 + 3e-5], True),           # outside the band: the max decides
    ([1e-3, -1e-3 + 1e-12, 0.0], False),                    # |sum| = 1e-12 < 1e-8 * 2e-3: max rule
]


def check_sign_rule():
    for v, flip in SIGN_CASES:
        u = np.array(v)[:, None]
        out = mlc.sign_normalise(u)[:, 0]
        assert np.array_equal(out, -u[:, 0] if flip else u[:, 0]), (v, out)


def test_sign_rule():
    check_sign_rule()


def test_sign_rule_stable_under_perturbation():
    """On the unit square with the SW-NE mesh, the eigenfunctions of the double eigenvalue
    5 pi^2 are odd under the point reflection of the square, so their nodal sums vanish up
    to rounding and the largest-entry rule fixes their sign.  The multilevel eigenvectors
    approximate the direct ones to ~1e-6; after the sign rule the two agree entry by entry
    (a sign decided by noise would differ by twice the vector)."""
    p = W.Problem(0, 8, 3, 4, 4, 1, 3, 0, None)
    res = mlc.solve(p)
    lam_h, U_h = mlc.direct_eigs(res.hier, 3, 3)
    for c in (1, 2):
        assert abs(U_h[:, c].sum()) < 1e-8 * np.abs(U_h[:, c]).sum()
    d = np.max(np.abs(res.U - U_h), axis=0) / np.max(np.abs(U_h), axis=0)
    assert np.all(d < 1e-3), d


# --- planted misreadings: the pins above must catch them ------------------------------

def _ramp_half_width(t, a, b, delta):
    d = 0.5 * delta
    return np.clip(np.minimum((t - a + d) / d, (b + d - t) / d), 0.0, 1.0)


def _ramp_zero_at_edge(t, a, b, delta):
    return np.clip(np.minimum((t - a) / delta, (b - t) / delta), 0.0, 1.0)


def _subdomains_unclipped(prob):
    n = prob.n_coarse
    bx = [(b * n) // prob.sub_x for b in range(prob.sub_x + 1)]
    by = [(b * n) // prob.sub_y for b in range(prob.sub_y + 1)]
    ov = prob.overlap
    return [mlc.Subdomain((bx[a], bx[a + 1], by[b], by[b + 1]),
                          (bx[a] - ov, bx[a + 1] + ov, by[b] - ov, by[b + 1] + ov))
            for b in range(prob.sub_y) for a in range(prob.sub_x)
            if not (prob.domain == 1 and bx[a] >= n // 2 and by[b + 1] <= n // 2)]


def _subdomains_no_drop(prob):
    n = prob.n_coarse
    bx = [(b * n) // prob.sub_x for b in range(prob.sub_x + 1)]
    by = [(b * n) // prob.sub_y for b in range(prob.sub_y + 1)]
    ov = prob.overlap
    return [mlc.Subdomain((bx[a], bx[a + 1], by[b], by[b + 1]),
                          (max(0, bx[a] - ov), min(n, bx[a + 1] + ov),
                           max(0, by[b] - ov), min(n, by[b + 1] + ov)))
            for b in range(prob.sub_y) for a in range(prob.sub_x)]


def _subdomains_ceil_bounds(prob):
    n = prob.n_coarse
    bx = [-((-b * n) // prob.sub_x) for b in range(prob.sub_x + 1)]
    by = [-((-b * n) // prob.sub_y) for b in range(prob.sub_y + 1)]
    ov = prob.overlap
    return [mlc.Subdomain((bx[a], bx[a + 1], by[b], by[b + 1]),
                          (max(0, bx[a] - ov), min(n, bx[a + 1] + ov),
                           max(0, by[b] - ov), min(n, by[b + 1] + ov)))
            for b in range(prob.sub_y) for a in range(prob.sub_x)]


def _sign_sum_only(U):
    U = U.copy()
    for c in range(U.shape[1]):
        if U[:, c].sum() < 0:
            U[:, c] = -U[:, c]
    return U


def _sign_strict_max(U):
    U = U.copy()
    for c in range(U.shape[1]):
        u = U[:, c]
        if abs(u.sum()) > 1e-8 * np.abs(u).sum():
            flip = u.sum() < 0
        else:
            flip = u[np.argmax(np.abs(u))] < 0
        if flip:
            U[:, c] = -u
    return U


@pytest.mark.parametrize("name, planted, checks", [
    ("ramp", _ramp_half_width, [check_ramp_values, lambda: check_pou_values(0)]),
    ("ramp", _ramp_zero_at_edge, [check_ramp_values, lambda: check_pou_values(0),
                                  check_pou_at_nodes]),
    ("subdomains", _subdomains_unclipped, [check_subdomain_layout]),
    ("subdomains", _subdomains_no_drop, [check_lshape_drop]),
    ("subdomains", _subdomains_ceil_bounds, [check_subdomain_layout]),
    ("sign_normalise", _sign_sum_only, [check_sign_rule]),
    ("sign_normalise", _sign_strict_max, [check_sign_rule]),
])
def test_pins_catch_planted_layout_mistakes(monkeypatch, name, planted, checks):
    monkeypatch.setattr(mlc, name, planted)
    for check in checks:
        with pytest.raises(AssertionError):
            check()
