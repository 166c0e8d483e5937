"""The benchmark's one-line JSON contract on the GPU (a short run of the default workload:
the unit square at h = 1/2048, FP64, with the mixed-precision run beside it)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "2",
                        "--warmup", "1", "--no-cpu-baseline"],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["config"]["workload"] == "c3_square_H32_h2048_16x16_q1"
    assert d["config"]["fine_dofs"] == 2047 * 2047 and d["dtype"] == "f64"
    # whole-step throughput: fine interior nodes of the finest level per second
    assert abs(d["value"] * d["ms_per_step"] * 1e-3 - d["config"]["fine_dofs"]) < 1e-6 * d["config"]["fine_dofs"]
    rl = d["roofline"]
    assert rl["bound"] == "hbm" and rl["unit"] == "GB/s" and rl["peak"] == 8000.0
    assert abs(rl["frac"] - rl["achieved"] / rl["peak"]) < 1e-12
    assert 0 < rl["frac"] < 1
    # the reference count: 18 passes of 8 bytes per tile unknown and iteration
    ls = d["local_solve"]
    assert abs(rl["bytes_per_launch"] - (144.0 * ls["it_dofs"] + 8.0 * ls["tile_dofs"])) < 1.0
    assert abs(rl["achieved"] - rl["bytes_per_launch"] / (ls["ms"] * 1e-3) / 1e9) < 1e-6 * rl["achieved"]
    assert 0 < rl["schedule_count"]["frac"] < rl["frac"]
    assert "cache_resident" not in rl and rl["tile_working_set_bytes"] > 256 * 2 ** 20
    assert d["lambda_rel_err_vs_oracle"] < 1e-10
    mx = d["mixed"]
    assert mx["lambda_rel_err_vs_oracle"] < 1e-10 and mx["value"] > 0
    assert mx["roofline"]["kernel"] == "k_local_mixed"
