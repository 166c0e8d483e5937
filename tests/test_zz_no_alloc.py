"""The allocation-free entry point mlc_solve_static (the library's static device scratch as
the workspace) against the existing path (mlc_create with a caller's workspace,
mlc_coarse_setup, mlc_run, mlc_get_eigenpairs) through the C ABI: two calls in a row, the
second on a smaller problem (the scratch then holds the first call's data), each bitwise
equal to the existing path, P1 and P2."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _existing(prob):
    from paper_1401_4969_amd import binding as B
    lam, u, _, _ = B.solve(prob, stats=False)
    return lam, u


@pytest.mark.parametrize("first,second", [
    (W.small_ragged().with_(n_refine=3), W.config1().with_(n_refine=1)),
    (W.config1_p2().with_(n_refine=3), W.small_field()),
])
def test_solve_static_two_calls_match_existing_path(first, second):
    torch = _torch()
    from paper_1401_4969_amd import binding as B
    for prob in (first, second):
        lam_s, u_s = B.solve_static(prob)
        lam_e, u_e = _existing(prob)
        assert np.array_equal(lam_s, lam_e), (prob.name, lam_s, lam_e)
        assert torch.equal(u_s, u_e), prob.name
    # and once more in the other order
    lam_s, _ = B.solve_static(first, with_vectors=False)
    assert np.array_equal(lam_s, _existing(first)[0])


def test_solve_static_rejects_too_large():
    _torch()
    from paper_1401_4969_amd import binding as B
    with pytest.raises(B.MLCError) as e:
        B.solve_static(W.config2(), with_vectors=False)   # 180 MiB of workspace
    assert e.value.status == B.MLC_ENOMEM
