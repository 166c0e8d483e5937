"""Seeded synthetic problem descriptions shared by the oracle, the tests and the bench.

This module holds no arithmetic of the method itself: it only fixes the
problem geometry (domain, coarse mesh, refinement count, subdomain grid,
overlap, number of eigenpairs) and draws the coefficient kappa from a seed.
Both the CPU oracle and the GPU library consume the same ``Problem`` objects.

Problem statement: -div(kappa grad u) = lambda u with homogeneous Dirichlet
data (the eigenproblem of Section 3; the elliptic operator of Section 2.2 with
A = kappa I).  The workloads are those of the scope table: the unit square
(the analogue of Example 6.1, whose own square is (-1,1)^2) and the L-shape
(-1,1)^2 minus [0,1)x(-1,0], with kappa constant, piecewise constant per
coarse cell, or per finest cell (a log-normal Gaussian random field).

Coefficient layouts (row-major, index = row * ncols + col, row along y):
  coef_kind 0: kappa == 1, ``kappa`` is None.
  coef_kind 1: one value per coarse cell, shape (n_coarse, n_coarse).
  coef_kind 2: one value per finest square cell, shape (N, N), N = n_coarse*2^n_refine.
Both triangles of a square cell share the cell's value.
  coef_kind 3 (the operator of Example 6.2: a(u,v) = (A grad u, grad v), b(u,v) =
  (phi u, v)): shape (4, 2, N, N), [component (a11, a12, a22, phi)][triangle (0 below
  the SW-NE diagonal, 1 above)][J][I], one symmetric positive definite tensor and one
  positive weight per finest triangle.

Domains: 0 the unit square (0,1)^2, 1 the L-shape, 2 the square (-1,1)^2 of Example 6.2.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np

DOMAIN_SQUARE = 0   # (0,1)^2
DOMAIN_LSHAPE = 1   # (-1,1)^2 \ [0,1)x(-1,0]
DOMAIN_SQUARE2 = 2  # (-1,1)^2


@dataclass
class Problem:
    domain: int = DOMAIN_SQUARE
    n_coarse: int = 8          # coarse cells per side of the bounding box
    n_refine: int = 2          # number of correction levels L (finest h = H / 2^L)
    sub_x: int = 4             # subdomain blocks along x
    sub_y: int = 4             # subdomain blocks along y
    overlap: int = 1           # coarse cells added to each side of D_j
    n_eig: int = 1             # q, number of eigenpairs
    coef_kind: int = 0
    kappa: Optional[np.ndarray] = field(default=None, repr=False)
    name: str = ""
    pou: int = 0               # gluing weights: 0 ramp across the overlap, 1 indicator of D_j
    order: int = 1             # polynomial degree of the elements: 1 (P1) or 2 (P2)

    # --- geometry helpers (no method arithmetic) ---
    @property
    def side(self) -> float:
        return 1.0 if self.domain == DOMAIN_SQUARE else 2.0

    @property
    def origin(self) -> float:
        return 0.0 if self.domain == DOMAIN_SQUARE else -1.0

    @property
    def n_fine(self) -> int:
        return self.n_coarse << self.n_refine

    def n_cells(self, level: int) -> int:
        return self.n_coarse << level

    def h(self, level: int) -> float:
        return self.side / self.n_cells(level)

    def kappa_array(self) -> np.ndarray:
        """kappa as a float64 array in its native layout (ones for coef_kind 0)."""
        if self.coef_kind == 0:
            return np.ones((self.n_coarse, self.n_coarse))
        return np.ascontiguousarray(self.kappa, dtype=np.float64)

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


def loguniform_coarse_kappa(n_coarse: int, rng: np.random.Generator,
                            lo: float = 0.1, hi: float = 10.0) -> np.ndarray:
    """Per coarse cell kappa = exp(U(ln lo, ln hi))."""
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=(n_coarse, n_coarse)))


def gaussian_field_kappa(n: int, seed: int, std: float = 0.5, corr_len: float = 0.1,
                         side: float = 1.0) -> np.ndarray:
    """kappa = exp(g) per finest cell, g a Gaussian field with squared-exponential
    covariance exp(-r^2/(2 l^2)) (l = corr_len), sampled at the n x n cell centres.

    White noise (PCG64, ``seed``) on a 2n x 2n zero-padded grid is convolved (by FFT)
    with a Gaussian kernel of standard deviation l/sqrt(2), whose self-convolution has
    the wanted covariance shape; the n x n crop is then shifted and scaled to sample
    mean 0 and sample standard deviation ``std``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    m = 2 * n
    noise = np.zeros((m, m))
    noise[:n, :n] = rng.standard_normal((n, n))
    h = side / n
    s = corr_len / np.sqrt(2.0)
    k = np.fft.fftfreq(m, d=h) * 2.0 * np.pi
    kx, ky = np.meshgrid(k, k, indexing="xy")
    # Fourier transform of a unit-mass Gaussian kernel of std s
    ghat = np.exp(-0.5 * s * s * (kx * kx + ky * ky))
    g = np.real(np.fft.ifft2(np.fft.fft2(noise) * ghat))[:n, :n]
    g = (g - g.mean()) / g.std() * std
    return np.exp(g)


# ---------------------------------------------------------------------------
# The five workloads of the scope table
# ---------------------------------------------------------------------------

def config1() -> Problem:
    """Unit square, H=1/8 -> h=1/32, 4x4 subdomains, overlap 1, q=1, kappa=1."""
    return Problem(DOMAIN_SQUARE, 8, 2, 4, 4, 1, 1, 0, None, "c1_square_H8_h32_4x4_q1")


def config2() -> Problem:
    """Unit square, H=1/16 -> h=1/512, 8x8 subdomains, overlap 1, q=3, kappa=1."""
    return Problem(DOMAIN_SQUARE, 16, 5, 8, 8, 1, 3, 0, None, "c2_square_H16_h512_8x8_q3")


def config3() -> Problem:
    """Unit square, H=1/32 -> h=1/2048, 16x16 subdomains, overlap 1, q=1, kappa=1."""
    return Problem(DOMAIN_SQUARE, 32, 6, 16, 16, 1, 1, 0, None, "c3_square_H32_h2048_16x16_q1")


def config4(n_problems: int = 256, seed: int = 4) -> List[Problem]:
    """Batch of independent problems: domain ~ Bernoulli(1/2) {square, L-shape},
    n_coarse=16 per bounding-box side, finest h ~ U{1/128, 1/256, 1/512} of the unit
    length, s ~ U{4..8} (s x s subdomains), kappa per coarse cell log-uniform [0.1, 10]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for p in range(n_problems):
        dom = int(rng.integers(0, 2))
        inv_h = int(rng.choice([128, 256, 512]))
        s = int(rng.integers(4, 9))
        n_c = 16
        side = 1.0 if dom == DOMAIN_SQUARE else 2.0
        n_fine = int(round(inv_h * side))
        L = int(np.log2(n_fine // n_c))
        kap = loguniform_coarse_kappa(n_c, rng)
        out.append(Problem(dom, n_c, L, s, s, 1, 1, 1, kap,
                           f"c4_p{p}_{'sq' if dom == 0 else 'L'}_h{inv_h}_s{s}"))
    return out


def config5(seed: int = 5) -> Problem:
    """Unit square, H=1/16 -> h=1/1024, 8x8 subdomains, q=1, kappa per finest cell = exp(g)."""
    n = 16 << 6
    return Problem(DOMAIN_SQUARE, 16, 6, 8, 8, 1, 1, 2, gaussian_field_kappa(n, seed),
                   "c5_square_H16_h1024_8x8_grf")


def triangle_centroids(domain: int, n: int):
    """Centroids (x, y) of the finest triangles, each of shape (2, n, n) in the kind-3
    layout [triangle][J][I]."""
    side = 1.0 if domain == DOMAIN_SQUARE else 2.0
    origin = 0.0 if domain == DOMAIN_SQUARE else -1.0
    h = side / n
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    x0 = origin + I * h
    y0 = origin + J * h
    # lower triangle (SW, SE, NE): centroid at (x0 + 2h/3, y0 + h/3); upper (SW, NE, NW):
    # at (x0 + h/3, y0 + 2h/3)
    x = np.stack([x0 + 2.0 * h / 3.0, x0 + h / 3.0])
    y = np.stack([y0 + h / 3.0, y0 + 2.0 * h / 3.0])
    return x, y


def example62_coefficients(n: int) -> np.ndarray:
    """Example 6.2: A = [[exp(1+x^2), exp(xy)], [exp(xy), exp(1+y^2)]] and
    phi = (1+x^2)(1+y^2) on (-1,1)^2, each evaluated at the centroid of every finest
    triangle (n cells per side), in the kind-3 layout."""
    x, y = triangle_centroids(DOMAIN_SQUARE2, n)
    return np.stack([np.exp(1.0 + x * x), np.exp(x * y), np.exp(1.0 + y * y),
                     (1.0 + x * x) * (1.0 + y * y)])


def random_tensor_coefficients(domain: int, n: int, seed: int) -> np.ndarray:
    """A seeded kind-3 field: per triangle a11, a22 log-uniform in [0.5, 2], a12 =
    t sqrt(a11 a22) with t uniform in [-0.4, 0.4] (so A is positive definite), phi
    log-uniform in [0.5, 2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shp = (2, n, n)
    a11 = np.exp(rng.uniform(np.log(0.5), np.log(2.0), size=shp))
    a22 = np.exp(rng.uniform(np.log(0.5), np.log(2.0), size=shp))
    a12 = rng.uniform(-0.4, 0.4, size=shp) * np.sqrt(a11 * a22)
    phi = np.exp(rng.uniform(np.log(0.5), np.log(2.0), size=shp))
    return np.stack([a11, a12, a22, phi])


def example62(n_refine: int = 3, sub: int = 2, n_eig: int = 6, overlap: int = 1,
              n_coarse: int = 20) -> Problem:
    """Example 6.2 on (-1,1)^2 with H = 0.1 (20 coarse cells per side), n_refine
    corrections, sub x sub subdomains, the lowest n_eig eigenpairs."""
    n = n_coarse << n_refine
    return Problem(DOMAIN_SQUARE2, n_coarse, n_refine, sub, sub, overlap, n_eig, 3,
                   example62_coefficients(n),
                   f"ex62_H{n_coarse}_h{n}_{sub}x{sub}_q{n_eig}")



def kappa_directions(kappa: np.ndarray, seed: int = 501) -> List[np.ndarray]:
    """Seeded perturbation directions d for directional derivatives of lambda_1 along
    kappa + t d: a cellwise Gaussian scaling, a block patch of cells, and a smooth
    sinusoid, each multiplied by kappa so that t is a relative step."""
    k = np.asarray(kappa, dtype=np.float64)
    ny, nx = k.shape
    rng = np.random.Generator(np.random.PCG64(seed))
    d1 = k * rng.standard_normal(k.shape)
    d2 = np.zeros_like(k)
    d2[ny * 5 // 16:ny * 9 // 16, nx * 3 // 16:nx * 7 // 16] = 1.0
    d2 *= k
    y = (np.arange(ny) + 0.5) / ny
    x = (np.arange(nx) + 0.5) / nx
    d3 = k * np.outer(np.sin(np.pi * y), np.cos(2 * np.pi * x))
    return [d1, d2, d3]


# ---------------------------------------------------------------------------
# P2 elements (Example 6.1 runs P1 and P2)
# ---------------------------------------------------------------------------

def config1_p2() -> Problem:
    """P2 on the unit square, H=1/8 -> h=1/32 (63^2 = 3,969 fine dofs), 4x4 subdomains,
    overlap 1, q=1, kappa=1."""
    return Problem(DOMAIN_SQUARE, 8, 2, 4, 4, 1, 1, 0, None, "c1p2_square_H8_h32_4x4_q1",
                   order=2)


def config2_p2() -> Problem:
    """P2 on the unit square, H=1/16 -> h=1/256: 511^2 = 261,121 fine dofs, the size of
    configuration 2; 8x8 subdomains, overlap 1, q=3 (lambda ~ 2 pi^2, 5 pi^2, 5 pi^2)."""
    return Problem(DOMAIN_SQUARE, 16, 4, 8, 8, 1, 3, 0, None, "c2p2_square_H16_h256_8x8_q3",
                   order=2)


def config3_p2() -> Problem:
    """P2 on the unit square, H=1/16 -> h=1/512: 1023^2 = 1,046,529 fine dofs; 16x16
    subdomains of one coarse cell (Omega_j of 3x3 cells: tiles of 191^2 P2 nodes), overlap 1,
    q=1.  The tiles' storage (about 0.6 GB) is far beyond the last-level cache."""
    return Problem(DOMAIN_SQUARE, 16, 5, 16, 16, 1, 1, 0, None, "c3p2_square_H16_h512_16x16_q1",
                   order=2)


def small_ragged_p2(seed: int = 13) -> Problem:
    """P2 on the L-shape with uneven subdomain splits and a per-coarse-cell kappa, q=2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return Problem(DOMAIN_LSHAPE, 10, 2, 3, 3, 1, 2, 1, loguniform_coarse_kappa(10, rng),
                   "ragged_p2_L_nc10_L2_3x3_q2", order=2)


def small_ragged(seed: int = 11) -> Problem:
    """Small L-shape with uneven subdomain splits and random per-coarse-cell kappa."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return Problem(DOMAIN_LSHAPE, 10, 2, 3, 3, 1, 2, 1, loguniform_coarse_kappa(10, rng),
                   "ragged_L_nc10_L2_3x3_q2")


def small_field(seed: int = 12, n_coarse: int = 8, n_refine: int = 2) -> Problem:
    """Small unit square with a per-finest-cell log-normal kappa."""
    n = n_coarse << n_refine
    return Problem(DOMAIN_SQUARE, n_coarse, n_refine, 3, 2, 1, 1, 2,
                   gaussian_field_kappa(n, seed), f"field_nc{n_coarse}_L{n_refine}_3x2")


def random_problem_wide(seed: int, max_fine: int = 64) -> Tuple[Problem, int]:
    """A small random problem over the whole input space, and a precision (0: FP64, 1:
    FP32 inner solves): any of the three domains, coefficient kinds 0-3 (kind 3 from
    random_tensor_coefficients), q in 1..5 (1..3 on the coarsest grids), overlap 0..2,
    any of the three gluings (the ramp needs an overlap), uneven subdomain splits."""
    rng = np.random.Generator(np.random.PCG64(10_000 + seed))
    dom = int(rng.integers(0, 3))
    n_c = int(rng.choice([4, 6, 8]))
    L = 1
    while (n_c << (L + 1)) <= max_fine and rng.uniform() < 0.6:
        L += 1
    s = int(rng.integers(1, min(n_c, 4) + 1))
    t = int(rng.integers(1, min(n_c, 4) + 1))
    q = int(rng.integers(1, (4 if n_c == 4 else 6)))
    kind = int(rng.integers(0, 4))
    pou = int(rng.integers(0, 3))
    overlap = int(rng.integers(1 if pou == 0 else 0, 3))
    # every Omega_j must span at least two coarse cells each way
    while s > 1 and n_c // s + overlap < 2:
        s -= 1
    while t > 1 and n_c // t + overlap < 2:
        t -= 1
    precision = int(rng.integers(0, 2))
    n = n_c << L
    kap = None
    if kind == 1:
        kap = loguniform_coarse_kappa(n_c, rng)
    elif kind == 2:
        kap = np.exp(rng.uniform(np.log(0.2), np.log(5.0), size=(n, n)))
    elif kind == 3:
        kap = random_tensor_coefficients(dom, n, 20_000 + seed)
    prob = Problem(dom, n_c, L, s, t, overlap, q, kind, kap, f"wide{seed}", pou=pou)
    return prob, precision


def random_problem(seed: int, max_fine: int = 64) -> Problem:
    """A small random problem for property sweeps (any domain/kappa kind/splits)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dom = int(rng.integers(0, 2))
    n_c = int(rng.choice([4, 6, 8, 10]))
    L = 1
    while (n_c << (L + 1)) <= max_fine and rng.uniform() < 0.6:
        L += 1
    s = int(rng.integers(1, min(n_c, 5) + 1))
    t = int(rng.integers(1, min(n_c, 5) + 1))
    q = int(rng.integers(1, 4))
    kind = int(rng.integers(0, 3))
    kap = None
    if kind == 1:
        kap = loguniform_coarse_kappa(n_c, rng)
    elif kind == 2:
        kap = np.exp(rng.uniform(np.log(0.2), np.log(5.0), size=(n_c << L, n_c << L)))
    return Problem(dom, n_c, L, s, t, 1, q, kind, kap, f"rand{seed}")
