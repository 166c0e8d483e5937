"""P2 elements on the nested uniform right-triangle meshes (oracle; test infrastructure only).

Section 2.1 defines V_h as the continuous piecewise-P_k functions on the triangulation and
V_0h as those with zero trace; Example 6.1 reports P2 results as well as P1.  A P2
function is fixed by its values at the vertices and at the edge midpoints.  On the mesh
with n cells per side (every cell cut by its SW-NE diagonal) these points are exactly the
nodes of the grid with 2n intervals per side: vertices at (even, even) positions,
midpoints of horizontal edges at (odd, even), of vertical edges at (even, odd), of the
diagonals at (odd, odd).  Node (i, j) of that grid has id j * (2n + 1) + i.

Everything is computed the plain way:
  * shape functions from the barycentric coordinates lambda_a of a triangle:
    lambda_a (2 lambda_a - 1) at vertex a, 4 lambda_a lambda_b at the midpoint of edge ab;
  * element matrices by quadrature on the reference triangle (a collapsed tensor
    Gauss-Legendre rule with 4 x 4 points, exact for polynomials up to degree 6; the
    products here have degree 2 (stiffness) and 4 (mass));
  * interior nodes: the nodes on no boundary edge (an edge of exactly one triangle);
  * nodal interpolation between nested meshes: each fine node is located in a coarse
    triangle and the six coarse shape functions are evaluated there.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .fem import DOMAIN_LSHAPE, locate, make_mesh


@dataclass
class MeshP2:
    n: int                 # cells per side of the bounding box
    h: float               # cell size
    origin: float
    grid: int              # intervals per side of the node grid (2n)
    xy: np.ndarray         # (2n+1)^2 x 2 node coordinates, node id = j*(2n+1)+i
    tri: np.ndarray        # T x 6 node ids: vertices v0, v1, v2, midpoints of v0v1, v1v2, v2v0
    tri_cell: np.ndarray   # T: cell J*n+I of each triangle
    tri_upper: np.ndarray  # T: True for the triangle above the diagonal
    dof: np.ndarray        # ids of the interior nodes, ascending
    n_nodes: int


def make_mesh_p2(domain: int, n: int, side: float, origin: float) -> MeshP2:
    """P2 nodes of the uniform mesh of [origin, origin+side]^2 with n cells per side (the
    cells of the removed quadrant dropped for the L-shape)."""
    h = side / n
    g = 2 * n
    ii, jj = np.meshgrid(np.arange(g + 1), np.arange(g + 1), indexing="xy")
    xy = np.stack([origin + ii.ravel() * (h / 2), origin + jj.ravel() * (h / 2)], axis=1)
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    I = I.ravel()
    J = J.ravel()
    keep = np.ones(I.size, dtype=bool)
    if domain == DOMAIN_LSHAPE:
        xc = origin + (I + 0.5) * h
        yc = origin + (J + 0.5) * h
        keep = ~((xc > 0.0) & (yc < 0.0))
    I = I[keep]
    J = J[keep]

    def nid(a, b):
        return b * (g + 1) + a

    sw = nid(2 * I, 2 * J)
    se = nid(2 * I + 2, 2 * J)
    ne = nid(2 * I + 2, 2 * J + 2)
    nw = nid(2 * I, 2 * J + 2)
    # lower triangle (SW, SE, NE): midpoints of SW-SE, SE-NE, NE-SW
    lower = np.stack([sw, se, ne, nid(2 * I + 1, 2 * J), nid(2 * I + 2, 2 * J + 1),
                      nid(2 * I + 1, 2 * J + 1)], axis=1)
    # upper triangle (SW, NE, NW): midpoints of SW-NE, NE-NW, NW-SW
    upper = np.stack([sw, ne, nw, nid(2 * I + 1, 2 * J + 1), nid(2 * I + 1, 2 * J + 2),
                      nid(2 * I, 2 * J + 1)], axis=1)
    tri = np.empty((2 * I.size, 6), dtype=np.int64)
    tri[0::2] = lower
    tri[1::2] = upper
    tri_cell = np.repeat(J * n + I, 2)
    tri_upper = np.tile(np.array([False, True]), I.size)
    n_nodes = (g + 1) ** 2
    dof = _interior_nodes_p2(tri, n_nodes)
    return MeshP2(n, h, origin, g, xy, tri, tri_cell, tri_upper, dof, n_nodes)


def _interior_nodes_p2(tri: np.ndarray, n_nodes: int) -> np.ndarray:
    """Nodes that belong to some triangle and lie on no boundary edge; the nodes of an
    edge are its two vertices and its midpoint."""
    edges = [(0, 1, 3), (1, 2, 4), (2, 0, 5)]
    ends = np.concatenate([tri[:, [a, b]] for a, b, _ in edges])
    mids = np.concatenate([tri[:, c] for _, _, c in edges])
    ends.sort(axis=1)
    key = ends[:, 0] * n_nodes + ends[:, 1]
    _, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
    bnd = cnt[inv] == 1
    on_bnd = np.zeros(n_nodes, dtype=bool)
    on_bnd[ends[bnd, 0]] = True
    on_bnd[ends[bnd, 1]] = True
    on_bnd[mids[bnd]] = True
    used = np.zeros(n_nodes, dtype=bool)
    used[tri.ravel()] = True
    return np.nonzero(used & ~on_bnd)[0]


def shape_p2(lam: np.ndarray) -> np.ndarray:
    """The six P2 shape functions at barycentric coordinates lam (... x 3)."""
    l0, l1, l2 = lam[..., 0], lam[..., 1], lam[..., 2]
    return np.stack([l0 * (2 * l0 - 1), l1 * (2 * l1 - 1), l2 * (2 * l2 - 1),
                     4 * l0 * l1, 4 * l1 * l2, 4 * l2 * l0], axis=-1)


def shape_grad_p2(lam: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Gradients of the six shape functions (... x 6 x 2) from lam (... x 3) and the
    gradients g (... x 3 x 2) of the barycentric coordinates."""
    l0, l1, l2 = (lam[..., a, None] for a in range(3))
    g0, g1, g2 = g[..., 0, :], g[..., 1, :], g[..., 2, :]
    return np.stack([(4 * l0 - 1) * g0, (4 * l1 - 1) * g1, (4 * l2 - 1) * g2,
                     4 * (l1 * g0 + l0 * g1), 4 * (l2 * g1 + l1 * g2),
                     4 * (l0 * g2 + l2 * g0)], axis=-2)


def _triangle_rule(npts: int = 4):
    """Points (s, t) and weights of the collapsed Gauss-Legendre rule on the reference
    triangle s, t >= 0, s + t <= 1 (weights sum to its area 1/2)."""
    x, w = np.polynomial.legendre.leggauss(npts)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    S, T = np.meshgrid(x, x, indexing="ij")
    WS, WT = np.meshgrid(w, w, indexing="ij")
    s = S.ravel()
    t = ((1.0 - S) * T).ravel()
    wt = (WS * WT * (1.0 - S)).ravel()
    return s, t, wt


def assemble_p2(mesh: MeshP2, kappa_tri: np.ndarray):
    """Global P2 stiffness a(u, v) = (kappa grad u, grad v) and mass b(u, v) = (u, v) over
    all nodes, as CSR matrices (kappa constant on each triangle)."""
    p = mesh.xy[mesh.tri[:, :3]]                 # T x 3 x 2 vertex coordinates
    d1 = p[:, 1] - p[:, 0]
    d2 = p[:, 2] - p[:, 0]
    det = d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0]
    # x = p0 + s d1 + t d2: the rows of [d1 d2]^-1 are grad s = grad lambda_1 and
    # grad t = grad lambda_2; grad lambda_0 = -grad lambda_1 - grad lambda_2
    g1 = np.stack([d2[:, 1], -d2[:, 0]], axis=1) / det[:, None]
    g2 = np.stack([-d1[:, 1], d1[:, 0]], axis=1) / det[:, None]
    g = np.stack([-g1 - g2, g1, g2], axis=1)     # T x 3 x 2
    s, t, wq = _triangle_rule()
    lam = np.stack([1.0 - s - t, s, t], axis=1)  # Q x 3
    phi = shape_p2(lam)                           # Q x 6
    T = p.shape[0]
    Kloc = np.zeros((T, 6, 6))
    Mloc = np.zeros((T, 6, 6))
    jac = np.abs(det)
    for qi in range(s.size):
        dphi = shape_grad_p2(np.broadcast_to(lam[qi], (T, 3)), g)   # T x 6 x 2
        Kloc += wq[qi] * np.einsum("tai,tbi->tab", dphi, dphi)
        Mloc += wq[qi] * np.outer(phi[qi], phi[qi])[None]
    Kloc *= (kappa_tri * jac)[:, None, None]
    Mloc *= jac[:, None, None]
    rows = np.repeat(mesh.tri, 6, axis=1).ravel()
    cols = np.tile(mesh.tri, (1, 6)).ravel()
    K = sp.coo_matrix((Kloc.ravel(), (rows, cols)), shape=(mesh.n_nodes, mesh.n_nodes)).tocsr()
    M = sp.coo_matrix((Mloc.ravel(), (rows, cols)), shape=(mesh.n_nodes, mesh.n_nodes)).tocsr()
    K.sum_duplicates()
    M.sum_duplicates()
    return K, M


def interpolation_p2(domain: int, coarse: MeshP2, fine: MeshP2, side: float) -> sp.csr_matrix:
    """Nodal interpolation V_H -> V_h of P2 functions on nested meshes, restricted to
    interior nodes (rows: fine dofs, columns: coarse dofs): the fine value at a node is
    the coarse P2 function evaluated there.  The node is located in a coarse triangle
    (of the P1 mesh with the same cells) and the six coarse shape functions are
    evaluated at its barycentric coordinates."""
    cmesh = make_mesh(domain, coarse.n, side, coarse.origin)
    pts = fine.xy[fine.dof]
    t, b = locate(cmesh, pts)
    assert (t >= 0).all(), "every fine interior node lies in a coarse triangle"
    # the P1 mesh lists the same triangles in the same order as the P2 mesh
    nodes = coarse.tri[t]                       # P x 6 coarse node ids
    vals = shape_p2(b)                           # P x 6
    col_of_node = -np.ones(coarse.n_nodes, dtype=np.int64)
    col_of_node[coarse.dof] = np.arange(coarse.dof.size)
    cols = col_of_node[nodes]
    rows = np.repeat(np.arange(pts.shape[0])[:, None], 6, axis=1)
    keep = (cols >= 0) & (vals != 0.0)
    P = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])),
                      shape=(fine.dof.size, coarse.dof.size)).tocsr()
    P.sum_duplicates()
    return P
