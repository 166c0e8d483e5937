"""Multilevel local-and-parallel eigen-correction, CPU FP64 oracle (test infrastructure only).

Follows Algorithm 4.2 (multilevel correction scheme) and Algorithm 4.1 (one
correction step) in their own order and notation:

  Algorithm 4.2, step 1: solve the eigenproblem directly on the first space
      V_0h1 (here h_1 = H, so this is the coarse space V_0H itself);
  Algorithm 4.2, step 3: for k = 1..n-1,
      (lambda_{h_k+1}, u_{h_k+1}) = Correction(V_0H, lambda_{h_k}, u_{h_k}, V_0h_{k+1}).

  Algorithm 4.1 (Correction):
    step 1, equation (Aux_Problem): on every subdomain Omega_j find
        e^j in V_0h_{k+1}(Omega_j) with
        a(e^j, v) = lambda_{h_k} b(u_{h_k}, v) - a(u_{h_k}, v)   for all v in V_0h_{k+1}(Omega_j),
      and set u~^j = u_{h_k} + e^j;
    step 2: glue the u~^j into one u~ in V_0h_{k+1}(Omega).  The paper glues with
      the regions G_j and one more boundary value problem on G_{m+1} (interface_gluing
      below); the default here is a partition of unity (chi_j, sum chi_j = 1),
      u~ = u_{h_k} + sum_j chi_j e^j;
    step 3, equation (Eigen_Augment_Problem): Rayleigh-Ritz on
        V_{H,h_{k+1}} = V_0H + span{u~}, normalised so that b(u, u) = 1.

For q > 1 eigenpairs (the multiple-eigenvalue remark of Section 4.1) the block
form is used: q local solves per subdomain, one per eigenpair with its own
lambda, and Rayleigh-Ritz on V_0H + span{u~_1..u~_q}, keeping the lowest q.

Readings of points the paper leaves open (mesh, h_1 = H, overlap width,
subdomain layout, gluing, kappa on coarser levels, sign) are those stated in
the design notes; each is marked "reading" where it is used below.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import Mesh, assemble, interpolation, make_mesh, triangle_kappa, triangle_tensor
from .fem_p2 import assemble_p2, interpolation_p2, make_mesh_p2


# ---------------------------------------------------------------------------
# Domain decomposition (Section 4, first paragraph)
# ---------------------------------------------------------------------------

@dataclass
class Subdomain:
    D: tuple       # (x0, x1, y0, y1) in coarse-cell units: the disjoint block D_j
    Omega: tuple   # the enlarged block Omega_j, clipped to the bounding box


def subdomains(prob) -> List[Subdomain]:
    """D_j: sub_x x sub_y blocks of whole coarse cells with block boundaries at
    floor(b * n_coarse / s) (reading: uneven splits allowed); Omega_j: D_j grown by
    ``overlap`` coarse cells on every side, clipped to the bounding box, so it is
    aligned with T_H.  On the L-shape, blocks lying wholly in the removed quadrant
    are dropped."""
    n = prob.n_coarse
    bx = [(b * n) // prob.sub_x for b in range(prob.sub_x + 1)]
    by = [(b * n) // prob.sub_y for b in range(prob.sub_y + 1)]
    ov = prob.overlap
    out = []
    for sy in range(prob.sub_y):
        for sx in range(prob.sub_x):
            D = (bx[sx], bx[sx + 1], by[sy], by[sy + 1])
            if prob.domain == 1 and D[0] >= n // 2 and D[3] <= n // 2:
                continue   # block inside the removed quadrant
            Om = (max(0, D[0] - ov), min(n, D[1] + ov), max(0, D[2] - ov), min(n, D[3] + ov))
            out.append(Subdomain(D, Om))
    return out


def ramp(t: np.ndarray, a: float, b: float, delta: float) -> np.ndarray:
    """1 on [a, b], falling linearly to 0 at distance delta outside it (reading of the gluing)."""
    return np.clip(np.minimum((t - a + delta) / delta, (b + delta - t) / delta), 0.0, 1.0)


def pou_weights(prob, subs: List[Subdomain], ti: np.ndarray, tj: np.ndarray) -> np.ndarray:
    """chi_j at points with coarse-cell coordinates (ti, tj): phi_j / sum_l phi_l, with
    phi_j(x, y) = ramp(x; D_j) ramp(y; D_j), ramp width delta = overlap coarse cells
    (prob.pou = 0), or phi_j = indicator of the closed D_j (prob.pou = 1).
    Returns an (m, P) array."""
    if getattr(prob, "pou", 0) == 1:
        phi = np.stack([((ti >= s.D[0]) & (ti <= s.D[1]) & (tj >= s.D[2]) & (tj <= s.D[3]))
                        .astype(np.float64) for s in subs])
    else:
        delta = float(prob.overlap)
        phi = np.stack([ramp(ti, s.D[0], s.D[1], delta) * ramp(tj, s.D[2], s.D[3], delta)
                        for s in subs])
    tot = phi.sum(axis=0)
    chi = np.zeros_like(phi)
    nz = tot > 0
    chi[:, nz] = phi[:, nz] / tot[nz]
    return chi


# ---------------------------------------------------------------------------
# Level hierarchy: meshes, Galerkin operators, interpolations
# ---------------------------------------------------------------------------

class Hierarchy:
    """Nested meshes T_H = T_{h_1} (level 0) ... T_{h_n} (level L) with
    a(.,.) and b(.,.) on every level obtained as P^T A P from the finest level,
    i.e. the exact restriction of the bilinear forms to the nested subspaces
    (Section 4.2 nested spaces)."""

    def __init__(self, prob):
        self.prob = prob
        L = prob.n_refine
        self.L = L
        self.order = getattr(prob, "order", 1)
        if self.order == 2:
            # P2 elements (Section 2.1 with k = 2): nodes on the grid of half cells
            self.meshes = [make_mesh_p2(prob.domain, prob.n_cells(m), prob.side, prob.origin)
                           for m in range(L + 1)]
            fine = self.meshes[L]
            assert prob.coef_kind in (0, 1), "P2 elements: kappa constant or per coarse cell"
            Kf, Mf = assemble_p2(fine, triangle_kappa(fine, prob.coef_kind, prob.kappa,
                                                      prob.n_coarse))
            P = [interpolation_p2(prob.domain, self.meshes[m], self.meshes[m + 1], prob.side)
                 for m in range(L)]
            self._galerkin(Kf, Mf, P)
            return
        self.meshes: List[Mesh] = [make_mesh(prob.domain, prob.n_cells(m), prob.side, prob.origin)
                                   for m in range(L + 1)]
        fine = self.meshes[L]
        if prob.coef_kind == 3:
            # reading: A and phi constant on each finest triangle, every level integrating
            # exactly (the Galerkin products below)
            A_tri, phi_tri = triangle_tensor(fine, prob.kappa)
            Kf, Mf = assemble(fine, None, A_tri, phi_tri)
        else:
            ktri = triangle_kappa(fine, prob.coef_kind, prob.kappa, prob.n_coarse)
            Kf, Mf = assemble(fine, ktri)
        # P[m]: level m -> level m+1 nodal interpolation on dofs
        self._galerkin(Kf, Mf, [interpolation(self.meshes[m], self.meshes[m + 1])
                                for m in range(L)])

    def _galerkin(self, Kf, Mf, P):
        """Finest operators on the dofs, coarser ones as P^T A P (nested spaces)."""
        prob, L = self.prob, self.L
        d = self.meshes[L].dof
        self.K = [None] * (L + 1)
        self.M = [None] * (L + 1)
        self.K[L] = Kf[d][:, d].tocsr()
        self.M[L] = Mf[d][:, d].tocsr()
        self.P = P
        for m in range(L - 1, -1, -1):
            Pm = self.P[m]
            self.K[m] = (Pm.T @ self.K[m + 1] @ Pm).tocsr()
            self.M[m] = (Pm.T @ self.M[m + 1] @ Pm).tocsr()
        # P0[m]: level 0 -> level m
        self.P0 = [sp.identity(self.meshes[0].dof.size, format="csr")]
        for m in range(L):
            self.P0.append((self.P[m] @ self.P0[m]).tocsr())
        self.subs = subdomains(prob)

    def n_dof(self, m: int) -> int:
        return self.meshes[m].dof.size

    def per_coarse(self, m: int) -> int:
        """Node-grid intervals per coarse cell at level m (2^m, twice that for P2)."""
        return self.order << m

    def node_ij(self, m: int, nodes: np.ndarray):
        n1 = self.order * self.meshes[m].n + 1
        return nodes % n1, nodes // n1

    def tile_dofs(self, m: int, s: Subdomain) -> np.ndarray:
        """Positions (into the level-m dof list) of the dofs strictly inside Omega_j:
        V_0h(Omega_j) = functions of V_0h supported in Omega_j."""
        i, j = self.node_ij(m, self.meshes[m].dof)
        r = self.per_coarse(m)
        x0, x1, y0, y1 = s.Omega
        inside = (i > x0 * r) & (i < x1 * r) & (j > y0 * r) & (j < y1 * r)
        return np.nonzero(inside)[0]

    def pou(self, m: int) -> np.ndarray:
        """chi_j at the level-m dofs, shape (m_sub, n_dof)."""
        i, j = self.node_ij(m, self.meshes[m].dof)
        r = float(self.per_coarse(m))
        return pou_weights(self.prob, self.subs, i / r, j / r)

    def to_grid(self, m: int, v: np.ndarray) -> np.ndarray:
        """Scatter a level-m dof vector (or columns) onto the full (n+1)^2 node grid."""
        mesh = self.meshes[m]
        v = np.asarray(v)
        shape = (mesh.n_nodes,) + v.shape[1:]
        g = np.zeros(shape)
        g[mesh.dof] = v
        return g


# ---------------------------------------------------------------------------
# The algorithm
# ---------------------------------------------------------------------------

SIGN_SUM_RTOL = 1e-8    # a nodal sum below this fraction of sum |u| does not fix the sign
SIGN_MAX_RTOL = 1e-6    # entries within this relative distance of max |u| tie for the largest


def sign_normalise(U: np.ndarray) -> np.ndarray:
    """Reading of the free sign (b(u, u) = 1 fixes u only up to sign): each eigenvector
    gets a positive nodal sum when |sum u| > 1e-8 sum |u|; otherwise (an eigenvector odd
    under a symmetry of the problem, whose sum is rounding noise) the first entry in node
    order whose magnitude is within a relative 1e-6 of the largest is made positive.  The
    relative band makes the choice stable under rounding: the largest magnitudes of an odd
    eigenvector come in pairs of opposite sign that tie in exact arithmetic."""
    U = U.copy()
    for c in range(U.shape[1]):
        u = U[:, c]
        s = u.sum()
        a = np.abs(u)
        if abs(s) > SIGN_SUM_RTOL * a.sum():
            flip = s < 0
        else:
            first = np.nonzero(a >= (1.0 - SIGN_MAX_RTOL) * a.max())[0][0]
            flip = u[first] < 0
        if flip:
            U[:, c] = -u
    return U


def coarse_eigs(hier: Hierarchy, q: int):
    """Algorithm 4.2 step 1 on V_0h1 = V_0H: lowest q eigenpairs, b(u_i, u_j) = delta_ij."""
    K0 = hier.K[0].toarray()
    M0 = hier.M[0].toarray()
    lam, U = sla.eigh(K0, M0, subset_by_index=[0, q - 1])
    return lam, sign_normalise(U)


@dataclass
class StepRecord:
    level: int
    lam: np.ndarray
    seconds: float
    residual_norms: Optional[np.ndarray] = None


def local_solve(hier: Hierarchy, m: int, s: Subdomain, rhs: np.ndarray):
    """Equation (Aux_Problem) on one subdomain: e^j = K_j^-1 rhs|_{T_j} with K_j the
    stiffness on V_0h(Omega_j) (sparse LU, exact to rounding).  rhs is (n_dof, q);
    returns (tile_dofs, e_j)."""
    idx = hier.tile_dofs(m, s)
    if idx.size == 0:
        return idx, np.zeros((0, rhs.shape[1]))
    Kj = hier.K[m][idx][:, idx].tocsc()
    lu = spla.splu(Kj)
    return idx, lu.solve(np.ascontiguousarray(rhs[idx]))


def local_solves(hier: Hierarchy, m: int, rhs: np.ndarray):
    """Algorithm 4.1 step 1: the independent solves of (Aux_Problem) on every subdomain;
    returns a list of (tile_dofs, e_j) pairs."""
    return [local_solve(hier, m, s, rhs) for s in hier.subs]


def rayleigh_ritz(hier: Hierarchy, m: int, Ut: np.ndarray, q: int):
    """Algorithm 4.1 step 3, equation (Eigen_Augment_Problem): the lowest q eigenpairs
    of a(.,.) = mu b(.,.) on V_0H + span{u~_1..u~_q} at level m.  With
    S = [P_{0->m}, U~]: A = S^T K S, B = S^T M S written blockwise."""
    K = hier.K[m]
    M = hier.M[m]
    P0 = hier.P0[m]
    KP0 = K @ P0
    MP0 = M @ P0
    KU = K @ Ut
    MU = M @ Ut
    A = np.block([[(P0.T @ KP0).toarray(), P0.T @ KU],
                  [(P0.T @ KU).T, Ut.T @ KU]])
    B = np.block([[(P0.T @ MP0).toarray(), P0.T @ MU],
                  [(P0.T @ MU).T, Ut.T @ MU]])
    A = 0.5 * (A + A.T)
    B = 0.5 * (B + B.T)
    mu, C = sla.eigh(A, B, subset_by_index=[0, q - 1])
    nH = P0.shape[1]
    U = P0 @ C[:nH] + Ut @ C[nH:]
    return mu, U, C


def interface_gluing(hier: Hierarchy, m: int, rhs: np.ndarray, sols) -> np.ndarray:
    """Algorithm 4.1 step 2 as the paper states it (prob.pou = 2): u~ = u~^j on G_j, and on
    G_{m+1} = Omega minus the closed G_j the solution of a(u~, v) = lambda b(u, v) for
    v in V_0h(G_{m+1}) with u~ = u~^j on the boundary of each G_j (and 0 on the boundary
    of Omega).  Reading: G_j = D_j shrunk by half a coarse cell on every side (aligned
    with every mesh from h_1 = H/2 on).  In correction form (u~ = I u + e): e = e^j on
    each closed G_j, and on the remaining dofs S the Dirichlet problem
    K_SS e_S = rhs_S - K_SG e_G (sparse LU).  Returns e at the level-m dofs."""
    i, j = hier.node_ij(m, hier.meshes[m].dof)
    r = hier.per_coarse(m)
    half = r // 2
    n = hier.n_dof(m)
    e = np.zeros_like(rhs)
    in_g = np.zeros(n, dtype=bool)
    for s, (idx, e_j) in zip(hier.subs, sols):
        x0, x1, y0, y1 = s.D
        sel = ((i >= x0 * r + half) & (i <= x1 * r - half) &
               (j >= y0 * r + half) & (j <= y1 * r - half))
        full = np.zeros_like(rhs)
        full[idx] = e_j
        assert not np.any(in_g & sel)   # the closed G_j are disjoint
        e[sel] = full[sel]
        in_g |= sel
    S = np.nonzero(~in_g)[0]
    G = np.nonzero(in_g)[0]
    K = hier.K[m].tocsr()
    if S.size:
        b = rhs[S] - K[S][:, G] @ e[G]
        e[S] = spla.splu(K[S][:, S].tocsc()).solve(np.ascontiguousarray(b))
    return e


def correction(hier: Hierarchy, k: int, lam_k: np.ndarray, u_k: np.ndarray, refine: bool = True):
    """Algorithm 4.1: one correction step from level k to level k+1 (or, with
    refine=False, within level k itself, used only to test the fixed point)."""
    m = k + 1 if refine else k
    q = lam_k.size
    # u_{h_k} viewed as an element of V_0h_{k+1} (nested spaces)
    ubar = hier.P[k] @ u_k if refine else u_k.copy()
    K = hier.K[m]
    M = hier.M[m]
    # right-hand side of (Aux_Problem): lambda_{h_k} b(u_{h_k}, v) - a(u_{h_k}, v)
    rhs = (M @ ubar) * lam_k[None, :] - K @ ubar
    # step 1: local solves; step 2: gluing (partition of unity, or the paper's interface
    # problem on G_{m+1})
    sols = local_solves(hier, m, rhs)
    if getattr(hier.prob, "pou", 0) == 2:
        ut = ubar + interface_gluing(hier, m, rhs, sols)
    else:
        chi = hier.pou(m)
        ut = ubar.copy()
        for (idx, e_j), chi_j in zip(sols, chi):
            ut[idx] += chi_j[idx, None] * e_j
    # step 3: Rayleigh-Ritz on V_0H + span{u~}
    mu, U, _ = rayleigh_ritz(hier, m, ut, q)
    return mu, sign_normalise(U), dict(rhs=rhs, ubar=ubar, ut=ut)


@dataclass
class OracleResult:
    lam: np.ndarray                  # final q eigenvalues
    U: np.ndarray                    # final eigenvectors on the finest dofs (n_dof x q)
    lam_levels: List[np.ndarray] = field(default_factory=list)
    U_levels: List[np.ndarray] = field(default_factory=list)
    seconds: List[float] = field(default_factory=list)
    hier: Optional[Hierarchy] = None


def solve(prob, hier: Optional[Hierarchy] = None, keep_levels: bool = True) -> OracleResult:
    """Algorithm 4.2 with h_1 = H (reading): direct coarse solve, then n_refine corrections."""
    if hier is None:
        hier = Hierarchy(prob)
    q = prob.n_eig
    t0 = time.perf_counter()
    lam, U = coarse_eigs(hier, q)
    res = OracleResult(lam, U, hier=hier)
    res.lam_levels.append(lam.copy())
    res.seconds.append(time.perf_counter() - t0)
    if keep_levels:
        res.U_levels.append(U.copy())
    for k in range(hier.L):
        t0 = time.perf_counter()
        lam, U, _ = correction(hier, k, lam, U)
        res.seconds.append(time.perf_counter() - t0)
        res.lam_levels.append(lam.copy())
        if keep_levels:
            res.U_levels.append(U.copy())
    res.lam = lam
    res.U = U
    return res


def direct_eigs(hier: Hierarchy, m: int, q: int):
    """The discrete eigenproblem (Discrete_Weak_Eigen_Problem) solved directly on V_0h at
    level m by shift-invert Lanczos: the lowest q eigenpairs, ascending."""
    K = hier.K[m].tocsc()
    M = hier.M[m].tocsc()
    n = K.shape[0]
    if n <= 400:
        lam, U = sla.eigh(K.toarray(), M.toarray(), subset_by_index=[0, q - 1])
        return lam, sign_normalise(U)
    lam, U = spla.eigsh(K, k=q, M=M, sigma=0.0, which="LM", tol=1e-14)
    o = np.argsort(lam)
    return lam[o], sign_normalise(U[:, o])
