"""The paper's sensitivity experiments on the coarse mesh size H and the overlap (the
error figures of Section 6), reproduced qualitatively with the GPU path.

Setting: unit square, kappa = 1, lambda_1, m = 4 subdomains (2 x 2 blocks, as in
Example 6.1), finest h = 1/256, H = 1/4 .. 1/32, overlap 0 (indicator gluing, Omega_j =
D_j), 1 and 2 coarse cells.  The reference is the direct discrete eigenvalue of the same
finest mesh (oracle, sparse eigensolver).  Properties checked: every multilevel value
lies above it (min-max, Section 3), and for every H the run without overlap is the
worst one.  The table is printed (pytest -s).
"""
import numpy as np
import pytest

import workloads as W
from oracle.mlc import Hierarchy, direct_eigs

pytestmark = pytest.mark.gpu

FINE = 256
N_COARSE = [4, 8, 16, 32]
OVERLAPS = [(0, 1), (1, 0), (2, 0)]  # (overlap, pou)


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_overlap_and_H_sensitivity():
    _torch()
    from paper_1401_4969_amd import binding as B
    ref_prob = W.Problem(0, 32, 3, 2, 2, 1, 1, 0, None)
    lam_h = direct_eigs(Hierarchy(ref_prob), 3, 1)[0][0]
    table = {}
    for nc in N_COARSE:
        L = int(np.log2(FINE // nc))
        for ov, pou in OVERLAPS:
            prob = W.Problem(0, nc, L, 2, 2, ov, 1, 0, None, f"sens_H{nc}_ov{ov}", pou=pou)
            lam, _, _, _ = B.solve(prob, stats=False)
            table[(nc, ov)] = (lam[0] - lam_h) / lam_h
    print("\nrelative error of lambda_1 against the direct eigenvalue at h = 1/256")
    print("H      " + "  ".join(f"overlap {ov}" for ov, _ in OVERLAPS))
    for nc in N_COARSE:
        print(f"1/{nc:<4d} " + "  ".join(f"{table[(nc, ov)]:9.2e}" for ov, _ in OVERLAPS))
    for key, err in table.items():
        assert err >= -1e-12, (key, err)
    for nc in N_COARSE:
        assert table[(nc, 0)] > max(table[(nc, 1)], table[(nc, 2)]), nc
