"""GPU parity of the P2 path (Section 2.1 with k = 2; Example 6.1 runs P1 and P2) against
the CPU oracle's P2 elements: eigenvalues to 1e-10 at every level, finest eigenvectors
node by node with their signs (projectors for close pairs), on the unit square and the
L-shape, with per-coarse-cell kappa, uneven splits, both partition-of-unity gluings and
overlap 0-2; the configuration-2-sized workload (h = 1/256, 261,121 fine dofs, q = 3)
against stored oracle values; a batch bitwise equal to single runs."""
import json
import os

import numpy as np
import pytest

import workloads as W
from test_gpu_parity import LAM_RTOL, compare, gpu_solve

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_p2_config1():
    _torch()
    lam, u, levels, stats, ref = compare(W.config1_p2())
    assert stats[-1]["n_dofs"] == 63 * 63
    # P2 reaches 2 pi^2 to 2e-5 at h = 1/32 (P1: 5e-2)
    assert 0 < lam[0] - 2 * np.pi ** 2 < 2e-5
    # the P1 V-cycle on the same nodes keeps the P2 tile solves short
    assert max(s["it_max"] for s in stats) <= 40


def test_p2_lshape_ragged_coarse_kappa():
    _torch()
    compare(W.small_ragged_p2())


@pytest.mark.parametrize("kw", [dict(overlap=2), dict(sub_x=1, sub_y=1), dict(n_eig=4),
                                dict(sub_x=3, sub_y=5), dict(pou=1, overlap=0),
                                dict(pou=1, overlap=1), dict(n_refine=3)])
def test_p2_variants(kw):
    _torch()
    compare(W.config1_p2().with_(**kw))


@pytest.mark.parametrize("kw", [dict(nu=1), dict(nu=3, omega=0.6), dict(smoother=0)])
def test_p2_solver_options(kw):
    """Smoothing counts without the LDS rings (nu = 1, 3: the gathering CG passes) and damped
    Jacobi in place of the Chebyshev weights: same results."""
    _torch()
    compare(W.small_ragged_p2(), **kw)


def test_p2_rows_wider_than_banded_cg_passes():
    """One subdomain over n_c = 9 at h = 1/576: P2 tile rows of 287 nodes, past the 256 of
    the banded CG passes but within the smoothing rings."""
    _torch()
    compare(W.Problem(0, 9, 4, 1, 1, 1, 1, 0, None, "wide_rows_p2", order=2))


@pytest.mark.parametrize("block", [256, 512])
def test_p2_block_sizes(block):
    _torch()
    compare(W.small_ragged_p2(), block=block)


def test_p2_config2_size_against_stored_oracle():
    """P2 at h = 1/256 (n_c = 16, 8 x 8 subdomains, q = 3): every level's eigenvalues against
    the stored oracle values, the first eigenvector at 512 seeded nodes (signed)."""
    torch = _torch()
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_c2p2.json")) as f:
        gold = json.load(f)
    prob = W.config2_p2()
    lam, u, levels, stats = gpu_solve(prob)
    for k, (a, b) in enumerate(zip(levels, gold["lam_levels"])):
        rel = np.max(np.abs(np.asarray(a) - np.asarray(b)) / np.abs(np.asarray(b)))
        assert rel < LAM_RTOL, (k, a, b, rel)
    idx = torch.as_tensor(np.asarray(gold["sample_nodes"]), device=u.device)
    vals = u[0].reshape(-1)[idx].cpu().numpy()
    ref = np.asarray(gold["sample_values"][0])
    err = np.max(np.abs(vals - ref)) / np.max(np.abs(ref))
    print(f"c2p2 vector 0: max sample error {err:.2e}")
    assert err < 1e-8
    for s in stats:
        assert s["relres_max"] <= 1e-12 * 1.0000001
    assert stats[-1]["n_dofs"] == 511 * 511


def test_p2_batch_equals_single_runs():
    torch = _torch()
    from paper_1401_4969_amd import binding as B
    rng = np.random.Generator(np.random.PCG64(81))
    # one coefficient kind per batch: kappa per coarse cell everywhere
    probs = [W.config1_p2().with_(coef_kind=1, kappa=W.loguniform_coarse_kappa(8, rng)),
             W.small_ragged_p2().with_(n_eig=1),
             W.Problem(0, 6, 3, 2, 3, 1, 1, 1, W.loguniform_coarse_kappa(6, rng), "p2_b2",
                       order=2),
             W.Problem(1, 8, 1, 2, 2, 1, 1, 1, np.ones((8, 8)), "p2_b3", order=2)]
    bs = B.BatchSolver(probs)
    bs.setup()
    bs.run(use_graph=True)
    for i, p in enumerate(probs):
        lam, u = bs.get(i)
        lam1, u1, _, _ = B.solve(p, stats=False)
        assert np.array_equal(lam, lam1), i
        assert torch.equal(u, u1), i
    bs.close()


def test_p2_config3_size_against_stored_oracle():
    """P2 at h = 1/512 (1,046,529 fine dofs, 16 x 16 subdomains of one coarse cell, tiles of
    191^2 P2 nodes): every level's eigenvalue against the stored oracle values and the
    eigenvector at 512 seeded nodes (signed)."""
    torch = _torch()
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_c3p2.json")) as f:
        gold = json.load(f)
    prob = W.config3_p2()
    lam, u, levels, stats = gpu_solve(prob)
    for k, (a, b) in enumerate(zip(levels, gold["lam_levels"])):
        rel = np.max(np.abs(np.asarray(a) - np.asarray(b)) / np.abs(np.asarray(b)))
        assert rel < LAM_RTOL, (k, a, b, rel)
    idx = torch.as_tensor(np.asarray(gold["sample_nodes"]), device=u.device)
    vals = u[0].reshape(-1)[idx].cpu().numpy()
    ref = np.asarray(gold["sample_values"][0])
    err = np.max(np.abs(vals - ref)) / np.max(np.abs(ref))
    print(f"c3p2 vector 0: max sample error {err:.2e}; local iterations",
          [s["it_max"] for s in stats])
    assert err < 1e-8
    assert stats[-1]["n_dofs"] == 1023 * 1023
