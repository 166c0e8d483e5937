"""P1 finite elements on nested uniform right-triangle meshes (oracle; test infrastructure only).

Section 2.1 defines V_h as the continuous piecewise-P_k functions on a
shape-regular triangulation and V_0h = V_h with zero trace.  Here k = 1 and the
triangulation is the uniform mesh whose square cells are cut by the diagonal
from the lower-left to the upper-right corner; regular refinement (connecting
edge midpoints, beta = 2, Section 6 Example 6.1) keeps that pattern, so the
meshes are nested.

Everything is computed the plain way:
  * interior (degree-of-freedom) nodes are the nodes not on any boundary edge,
    a boundary edge being an edge that belongs to exactly one triangle;
  * element matrices come from the vertex coordinates of each triangle
    (gradients of the barycentric functions, area/12 (1 + delta_ab) mass); for the
    operator of Example 6.2 (a full tensor A and a mass weight phi, both constant on
    each triangle) the stiffness is area * G A G^T and the mass is scaled by phi;
  * the nodal interpolation from a coarse to a fine mesh evaluates the coarse
    P1 function at every fine node by locating the node in a coarse triangle
    and using its barycentric coordinates.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

DOMAIN_SQUARE = 0
DOMAIN_LSHAPE = 1


@dataclass
class Mesh:
    n: int                 # cells per side of the bounding box
    h: float
    origin: float
    xy: np.ndarray         # (n+1)^2 x 2 node coordinates, node id = j*(n+1)+i
    tri: np.ndarray        # T x 3 vertex ids (counter-clockwise)
    tri_cell: np.ndarray   # T: (J, I) cell of each triangle, as J*n+I
    tri_upper: np.ndarray  # T: True for the triangle above the diagonal
    dof: np.ndarray        # node ids of interior nodes, ascending
    n_nodes: int


def make_mesh(domain: int, n: int, side: float, origin: float) -> Mesh:
    """Uniform mesh of the bounding box [origin, origin+side]^2 with n cells per side.

    For the L-shape the cells of the removed quadrant [0,1)x(-1,0] are dropped.
    """
    h = side / n
    ii, jj = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="xy")
    xy = np.stack([origin + ii.ravel() * h, origin + jj.ravel() * h], axis=1)
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
    sw = J * (n + 1) + I
    se = sw + 1
    nw = sw + (n + 1)
    ne = nw + 1
    lower = np.stack([sw, se, ne], axis=1)   # below the SW-NE diagonal
    upper = np.stack([sw, ne, nw], axis=1)   # above it
    tri = np.empty((2 * I.size, 3), dtype=np.int64)
    tri[0::2] = lower
    tri[1::2] = upper
    cell = J * n + I
    tri_cell = np.repeat(cell, 2)
    tri_upper = np.tile(np.array([False, True]), I.size)
    n_nodes = (n + 1) ** 2
    dof = _interior_nodes(tri, n_nodes)
    return Mesh(n, h, origin, xy, tri, tri_cell, tri_upper, dof, n_nodes)


def _interior_nodes(tri: np.ndarray, n_nodes: int) -> np.ndarray:
    """Nodes that belong to some triangle and lie on no boundary edge."""
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    e.sort(axis=1)
    key = e[:, 0] * n_nodes + e[:, 1]
    uniq, cnt = np.unique(key, return_counts=True)
    bnd = uniq[cnt == 1]
    on_bnd = np.zeros(n_nodes, dtype=bool)
    on_bnd[bnd // n_nodes] = True
    on_bnd[bnd % n_nodes] = True
    used = np.zeros(n_nodes, dtype=bool)
    used[tri.ravel()] = True
    return np.nonzero(used & ~on_bnd)[0]


def triangle_kappa(mesh: Mesh, coef_kind: int, kappa: np.ndarray, n_coarse: int) -> np.ndarray:
    """kappa of every triangle from the problem's coefficient layout (scalar kinds 0-2)."""
    J = mesh.tri_cell // mesh.n
    I = mesh.tri_cell % mesh.n
    if coef_kind == 0:
        return np.ones(mesh.tri.shape[0])
    if coef_kind == 1:
        r = mesh.n // n_coarse
        return np.asarray(kappa)[J // r, I // r].astype(np.float64)
    if coef_kind == 2:
        k = np.asarray(kappa)
        assert k.shape == (mesh.n, mesh.n)
        return k[J, I].astype(np.float64)
    raise ValueError(coef_kind)


def triangle_tensor(mesh: Mesh, coef: np.ndarray):
    """Coefficient kind 3: the symmetric tensor A (T x 2 x 2) and the mass weight phi (T,)
    of every triangle, from the layout [component (a11, a12, a22, phi)][triangle (0 below
    the diagonal, 1 above)][J][I] of the finest cells."""
    c = np.asarray(coef, dtype=np.float64)
    assert c.shape == (4, 2, mesh.n, mesh.n)
    J = mesh.tri_cell // mesh.n
    I = mesh.tri_cell % mesh.n
    t = mesh.tri_upper.astype(np.int64)
    A = np.empty((mesh.tri.shape[0], 2, 2))
    A[:, 0, 0] = c[0, t, J, I]
    A[:, 0, 1] = A[:, 1, 0] = c[1, t, J, I]
    A[:, 1, 1] = c[2, t, J, I]
    return A, c[3, t, J, I]


def assemble(mesh: Mesh, kappa_tri: np.ndarray, A_tri: np.ndarray = None,
             phi_tri: np.ndarray = None):
    """Global P1 stiffness a(u,v) = (kappa grad u, grad v) and mass b(u,v) = (u,v)
    over all nodes (Section 2.2 weak form, Section 3 eigenproblem), as CSR matrices.
    With A_tri and phi_tri (Example 6.2): a(u,v) = (A grad u, grad v) and
    b(u,v) = (phi u, v), A and phi constant on each triangle."""
    p = mesh.xy[mesh.tri]                       # T x 3 x 2
    d1 = p[:, 1] - p[:, 0]
    d2 = p[:, 2] - p[:, 0]
    det = d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0]
    area = 0.5 * np.abs(det)
    # x = p0 + l1 d1 + l2 d2, so (l1, l2) = J^-1 (x - p0) with J = [d1 d2];
    # the rows of J^-1 are grad l1 and grad l2, and grad l0 = -grad l1 - grad l2.
    Jinv = np.empty((p.shape[0], 2, 2))
    Jinv[:, 0, 0] = d2[:, 1] / det
    Jinv[:, 0, 1] = -d2[:, 0] / det
    Jinv[:, 1, 0] = -d1[:, 1] / det
    Jinv[:, 1, 1] = d1[:, 0] / det
    ref = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])   # l_a in terms of (l1, l2)
    G = np.einsum("am,tmc->tac", ref, Jinv)
    # G[t, a, :] = physical gradient of barycentric function a on triangle t
    if A_tri is None:
        Kloc = np.einsum("tai,tbi->tab", G, G) * (kappa_tri * area)[:, None, None]
        Mloc = (np.ones((3, 3)) + np.eye(3))[None] * (area / 12.0)[:, None, None]
    else:
        Kloc = np.einsum("tai,tij,tbj->tab", G, A_tri, G) * area[:, None, None]
        Mloc = (np.ones((3, 3)) + np.eye(3))[None] * (phi_tri * area / 12.0)[:, None, None]
    rows = np.repeat(mesh.tri, 3, axis=1).ravel()
    cols = np.tile(mesh.tri, (1, 3)).ravel()
    K = sp.coo_matrix((Kloc.ravel(), (rows, cols)), shape=(mesh.n_nodes, mesh.n_nodes)).tocsr()
    M = sp.coo_matrix((Mloc.ravel(), (rows, cols)), shape=(mesh.n_nodes, mesh.n_nodes)).tocsr()
    K.sum_duplicates()
    M.sum_duplicates()
    return K, M


def barycentric(mesh: Mesh, t: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Barycentric coordinates of points pts (P x 2) in triangles t (P,)."""
    p = mesh.xy[mesh.tri[t]]
    d1 = p[:, 1] - p[:, 0]
    d2 = p[:, 2] - p[:, 0]
    det = d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0]
    w = pts - p[:, 0]
    l1 = (w[:, 0] * d2[:, 1] - w[:, 1] * d2[:, 0]) / det
    l2 = (d1[:, 0] * w[:, 1] - d1[:, 1] * w[:, 0]) / det
    return np.stack([1.0 - l1 - l2, l1, l2], axis=1)


def locate(mesh: Mesh, pts: np.ndarray):
    """For each point, a triangle of ``mesh`` containing it and the barycentric coordinates.

    The candidate cell is the one with lower-left corner floor((p - origin)/h),
    clamped into the box; both of its triangles are tested, together with the
    triangles of the neighbouring cells, and the first triangle whose barycentric
    coordinates are all >= -1e-12 is taken.
    """
    n = mesh.n
    cell_of_tri = -np.ones((n * n, 2), dtype=np.int64)
    cell_of_tri[mesh.tri_cell, mesh.tri_upper.astype(int)] = np.arange(mesh.tri.shape[0])
    ci = np.clip(np.floor((pts[:, 0] - mesh.origin) / mesh.h + 1e-9).astype(np.int64), 0, n - 1)
    cj = np.clip(np.floor((pts[:, 1] - mesh.origin) / mesh.h + 1e-9).astype(np.int64), 0, n - 1)
    found_t = -np.ones(pts.shape[0], dtype=np.int64)
    found_b = np.zeros((pts.shape[0], 3))
    for di in (0, -1, 1):
        for dj in (0, -1, 1):
            for up in (0, 1):
                todo = found_t < 0
                if not todo.any():
                    break
                ii = np.clip(ci + di, 0, n - 1)
                jj = np.clip(cj + dj, 0, n - 1)
                t = cell_of_tri[jj * n + ii, up]
                sel = todo & (t >= 0)
                if not sel.any():
                    continue
                b = barycentric(mesh, t[sel], pts[sel])
                ok = (b >= -1e-12).all(axis=1)
                idx = np.nonzero(sel)[0][ok]
                found_t[idx] = t[sel][ok]
                found_b[idx] = b[ok]
    return found_t, found_b


def interpolation(coarse: Mesh, fine: Mesh) -> sp.csr_matrix:
    """Nodal interpolation I: V_H -> V_h on nested meshes, restricted to interior nodes
    (rows: fine dofs, columns: coarse dofs).  The fine value at a node is the coarse
    P1 function evaluated at that node; fine nodes outside the coarse mesh's
    triangles (the removed quadrant) get no row entries."""
    pts = fine.xy[fine.dof]
    t, b = locate(coarse, pts)
    assert (t >= 0).all(), "every fine interior node lies in a coarse triangle"
    verts = coarse.tri[t]                          # P x 3 coarse node ids
    col_of_node = -np.ones(coarse.n_nodes, dtype=np.int64)
    col_of_node[coarse.dof] = np.arange(coarse.dof.size)
    cols = col_of_node[verts]
    rows = np.repeat(np.arange(pts.shape[0])[:, None], 3, axis=1)
    keep = (cols >= 0) & (np.abs(b) > 0.0)
    P = sp.coo_matrix((b[keep], (rows[keep], cols[keep])),
                      shape=(fine.dof.size, coarse.dof.size)).tocsr()
    P.sum_duplicates()
    return P
