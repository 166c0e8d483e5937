"""Host-side checks of the benchmark script (CPU only): the one-GPU contract, the
algorithmic byte model behind the roofline figure, and its node counts against the
oracle's meshes."""
import os
import subprocess
import sys

import numpy as np
import pytest

import bench
import workloads as W
from oracle.mlc import Hierarchy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}),
                                      ([], {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_exits_with_message(argv, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], env=e,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_byte_model_small_tile_by_hand():
    """A 3 x 3 tile over one coarser level (2 x 2 coarse cells, m = 1): 8 level-0 vector
    passes (direction 3, update 5) on 9 unknowns, the banded pre- (2) and post-smoothing (3)
    on them, the restriction write and correction read (2) and the coarsest b, z (2) on the
    single coarse unknown, and its 1 x 1 dense inverse: 8 * (8*9 + 5*9 + 2 + 2 + 1) bytes."""
    assert bench.pcg_bytes_per_iteration(2, 2, 1, 2) == 8 * (8 * 9 + 5 * 9 + 2 + 2 + 1)
    # FP32 elements halve it; sweeps apart (mode 0) count 2 + 3 + 1 before and 2 + 3 nu after
    assert bench.pcg_bytes_per_iteration(2, 2, 1, 2, elem=4) == 4 * (8 * 9 + 5 * 9 + 5)
    assert bench.pcg_bytes_per_iteration(2, 2, 1, 2, mode=0) == 8 * (8 * 9 + (6 + 8) * 9 + 5)


@pytest.mark.parametrize("cw,m,expect", [(4, 5, 122.1), (4, 6, 122.4)])
def test_byte_model_per_unknown_of_the_headline_tiles(cw, m, expect):
    """The figures the design notes quote: 127^2 tiles of config 2, 255^2 of config 3."""
    S0 = (cw * (1 << m) - 1) ** 2
    assert round(bench.pcg_bytes_per_iteration(cw, cw, m, 2) / S0, 1) == expect
    assert 2 * bench.pcg_bytes_per_iteration(cw, cw, m, 2, elem=4) == bench.pcg_bytes_per_iteration(cw, cw, m, 2)


@pytest.mark.parametrize("prob", [W.config2(), W.small_ragged(), W.config1(),
                                  W.example62(n_refine=2, sub=2, n_eig=1)])
def test_interior_nodes_match_oracle_mesh(prob):
    hier = Hierarchy(prob)
    for level in range(prob.n_refine + 1):
        assert bench.interior_nodes(prob, level) == hier.meshes[level].dof.size
