"""GPU tests of the batched path: many independent problems, one launch per kernel and
level step, optionally captured in a hipGraph, with an autotuned workgroup size.

The local solves of different problems are independent work items, so a problem's
results in a batch must be bitwise identical to a single-problem run with the same
workgroup size, and agree with the CPU oracle to 1e-10.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import solve as oracle_solve

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _small_batch(kind=1, q=1, n=7, seed0=100):
    rng = np.random.Generator(np.random.PCG64(seed0))
    out = []
    for i in range(n):
        dom = int(rng.integers(0, 2))
        nc = int(rng.choice([4, 6, 8]))
        L = int(rng.integers(1, 4))
        s = int(rng.integers(1, min(nc, 4) + 1))
        kap = None
        if kind == 1:
            kap = W.loguniform_coarse_kappa(nc, rng)
        elif kind == 2:
            kap = np.exp(rng.uniform(-1, 1, size=(nc << L, nc << L)))
        elif kind == 3:
            kap = W.random_tensor_coefficients(dom, nc << L, seed0 + i)
        out.append(W.Problem(dom, nc, L, s, s, 1, q, kind, kap, f"b{i}"))
    return out


def _single(prob, **kw):
    from paper_1401_4969_amd import binding as B
    s = B.Solver(prob, B.default_opts(**kw))
    s.coarse_setup()
    s.run()
    lam, u = s.eigenpairs()
    s.close()
    return lam, u


@pytest.mark.parametrize("kind,q,precision", [(1, 1, 0), (2, 1, 0), (0, 2, 0), (1, 1, 1),
                                              (3, 2, 0), (3, 1, 1)])
def test_batch_matches_single_and_oracle(kind, q, precision):
    torch = _torch()
    from paper_1401_4969_amd import binding as B
    probs = _small_batch(kind, q)
    bs = B.BatchSolver(probs, B.default_opts(precision=precision))
    bs.setup()
    bs.run()
    st = bs.stats()
    assert st["relres_max"] <= 1e-12 * 1.0000001
    for i, p in enumerate(probs):
        lam, u = bs.get(i)
        lam1, u1 = _single(p, precision=precision)
        assert np.array_equal(lam, lam1), (i, lam, lam1)
        assert torch.equal(u, u1)
        ref = oracle_solve(p)
        assert np.allclose(lam, ref.lam, rtol=1e-10, atol=0), (i, lam, ref.lam)
    bs.close()


def _wide_batch(kind, q, n=6, seed0=300):
    """Problems of one coefficient kind and q over the three domains, uneven splits, overlap
    0-2 and both partition-of-unity gluings (every Omega_j at least two coarse cells)."""
    rng = np.random.Generator(np.random.PCG64(seed0 + 10 * kind + q))
    out = []
    for i in range(n):
        dom = int(rng.integers(0, 3))
        nc = int(rng.choice([4, 6, 8]))
        L = int(rng.integers(1, 4))
        pou = int(rng.integers(0, 2))
        ov = int(rng.integers(1 if pou == 0 else 0, 3))
        sx = int(rng.integers(1, min(nc, 4) + 1))
        sy = int(rng.integers(1, min(nc, 4) + 1))
        while sx > 1 and nc // sx + ov < 2:
            sx -= 1
        while sy > 1 and nc // sy + ov < 2:
            sy -= 1
        kap = None
        if kind == 1:
            kap = W.loguniform_coarse_kappa(nc, rng)
        elif kind == 2:
            kap = np.exp(rng.uniform(-1, 1, size=(nc << L, nc << L)))
        elif kind == 3:
            kap = W.random_tensor_coefficients(dom, nc << L, seed0 + 100 + i)
        out.append(W.Problem(dom, nc, L, sx, sy, ov, min(q, 3 if nc == 4 else q), kind, kap,
                             f"w{i}", pou=pou))
    # one q per batch
    qb = min(p.n_eig for p in out)
    return [p.with_(n_eig=qb) for p in out]


def test_batch_tile_widths_around_ring_caps():
    """Tiles of 95, 127, 191 and 255 nodes a row in one FP64 launch: 191 takes two band rows
    per wave only without the LDS V-cycle tail, 255 one row with it.  Each item chooses from
    its own width against caps that depend on the device only, so every problem of the
    batch is bitwise a single run of itself (whose widest tile differs)."""
    torch = _torch()
    from paper_1401_4969_amd import binding as B
    rng = np.random.Generator(np.random.PCG64(404))
    probs = [W.Problem(0, 6, 6, 3, 3, 1, 1, 1, W.loguniform_coarse_kappa(6, rng), "cap_a"),
             W.Problem(0, 8, 5, 4, 4, 1, 1, 1, W.loguniform_coarse_kappa(8, rng), "cap_b"),
             W.Problem(1, 6, 6, 6, 6, 1, 1, 1, W.loguniform_coarse_kappa(6, rng), "cap_c")]
    bs = B.BatchSolver(probs, B.default_opts())
    bs.setup()
    bs.run()
    assert bs.stats()["relres_max"] <= 1e-12 * 1.0000001
    res = [bs.get(i) for i in range(len(probs))]
    bs.close()
    for i, p in enumerate(probs):
        lam1, u1 = _single(p)
        assert np.array_equal(res[i][0], lam1), (i, res[i][0], lam1)
        assert torch.equal(res[i][1], u1)


@pytest.mark.parametrize("kind,q,precision", [(0, 3, 0), (1, 2, 1), (2, 1, 0), (3, 4, 0),
                                              (3, 1, 1)])
def test_wide_batch_matches_single_and_oracle(kind, q, precision):
    """Batches mixing the three domains, splits, overlaps and both partition-of-unity
    gluings: each problem bitwise as a single run, and the oracle's eigenvalues to 1e-10;
    a graph-replayed run reproduces the eager one bitwise."""
    torch = _torch()
    from paper_1401_4969_amd import binding as B
    probs = _wide_batch(kind, q)
    bs = B.BatchSolver(probs, B.default_opts(precision=precision))
    bs.setup()
    bs.run()
    assert bs.stats()["relres_max"] <= 1e-12 * 1.0000001
    res = [bs.get(i) for i in range(len(probs))]
    bs.close()
    for i, p in enumerate(probs):
        lam, u = res[i]
        lam1, u1 = _single(p, precision=precision)
        assert np.array_equal(lam, lam1), (i, lam, lam1)
        assert torch.equal(u, u1)
        ref = oracle_solve(p)
        assert np.allclose(lam, ref.lam, rtol=1e-10, atol=0), (i, lam, ref.lam)
    gs = B.BatchSolver(probs, B.default_opts(precision=precision))
    gs.setup()
    gs.run(use_graph=True)
    for i in range(len(probs)):
        lam, u = gs.get(i)
        assert np.array_equal(lam, res[i][0])
        assert torch.equal(u, res[i][1])
    gs.close()


@pytest.mark.parametrize("kind", [1, 3])
def test_graph_replays_match_eager(kind):
    """Every graph replay, with eager work and synchronisations in between, reproduces
    the eager step bitwise."""
    torch = _torch()
    from paper_1401_4969_amd import binding as B
    probs = _small_batch(kind, 1)
    eager = B.BatchSolver(probs)
    eager.setup()
    eager.run(use_graph=False)
    ref = [eager.get(i) for i in range(len(probs))]
    graph = B.BatchSolver(probs)
    graph.setup()
    graph.run(use_graph=True)
    for replay in range(3):
        for i in range(len(probs)):
            lam, u = graph.get(i)
            assert np.array_equal(lam, ref[i][0])
            assert torch.equal(u, ref[i][1])
        # eager work on the same stream between replays
        x = torch.randn(1 << 20, device="cuda:0", dtype=torch.float64)
        (x * 2).sum().item()
        torch.cuda.synchronize()
        graph.rewind()
        graph.step(use_graph=True)
    eager.close()
    graph.close()


def test_interface_gluing_graph_steps():
    """The paper's gluing in captured steps: the G_{m+1} CG runs a fixed number of
    iterations with converged right-hand sides frozen, so every replay (eager work and
    synchronisations in between) equals the eager run, which stops at convergence, bitwise;
    too few captured iterations are reported as MLC_ENOCONV."""
    torch = _torch()
    from paper_1401_4969_amd import binding as B
    rng = np.random.Generator(np.random.PCG64(77))
    prob = W.Problem(0, 8, 3, 4, 4, 1, 2, 1, W.loguniform_coarse_kappa(8, rng), "iface_graph",
                     pou=2)
    eager = B.BatchSolver([prob])
    eager.setup()
    eager.run(use_graph=False)
    ref = eager.get(0)
    graph = B.BatchSolver([prob])
    graph.setup()
    graph.run(use_graph=True)
    for replay in range(3):
        lam, u = graph.get(0)
        assert np.array_equal(lam, ref[0])
        assert torch.equal(u, ref[1])
        st = graph.stats()
        assert 0 < st["glue_it"] <= 24 and st["glue_relres"] <= 1e-12 * 1.0000001
        x = torch.randn(1 << 20, device="cuda:0", dtype=torch.float64)
        (x * 2).sum().item()
        torch.cuda.synchronize()
        graph.rewind()
        graph.step(use_graph=True)
    short = B.BatchSolver([prob], opts=B.default_opts(glue_graph_it=2))
    short.setup()
    with pytest.raises(B.MLCError) as e:
        short.run(use_graph=True)
    assert e.value.status == B.MLC_ENOCONV
    for s in (eager, graph, short):
        s.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_autotune_choices_and_results(precision, tmp_path, monkeypatch):
    """The autotuner picks, per step, a workgroup size, nu in 1..3 and (mixed precision) an
    inner tolerance among 1e-3, 3e-4, .. 1e-5; every choice solves to rtol, so the results match
    the oracle to 1e-10; the tuning transfers to another batch of the same problems, whose
    results are then bitwise those of the tuned batch."""
    torch = _torch()
    from paper_1401_4969_amd import binding as B
    monkeypatch.setenv("MLC_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    probs = _small_batch(1, 1)
    opts = B.default_opts(precision=precision)
    bs = B.BatchSolver(probs, opts)
    bs.setup()
    blocks = bs.autotune()
    t = bs.tuning()
    assert t["blocks"] == blocks and all(b in (256, 512, 1024) for b in blocks)
    assert len(blocks) == bs.n_steps and all(v in (1, 2, 3) for v in t["nu"])
    if precision:
        assert all(v in (1e-3, 3e-4, 1e-4, 3e-5, 1e-5) for v in t["inner_rtol"])
    else:
        assert all(v == opts.inner_rtol for v in t["inner_rtol"])
    assert bs.current_step == 0
    bs.run()
    res = [bs.get(i) for i in range(len(probs))]
    for i, p in enumerate(probs):
        ref = oracle_solve(p)
        assert np.allclose(res[i][0], ref.lam, rtol=1e-10, atol=0)
    other = B.BatchSolver(probs, opts)
    other.setup()
    other.set_tuning(t)
    assert other.tuning() == t
    other.run()
    for i in range(len(probs)):
        lam, u = other.get(i)
        assert np.array_equal(lam, res[i][0]) and torch.equal(u, res[i][1])
    with pytest.raises(B.MLCError) as e:
        other.set_tuning(dict(t, nu=[0] * len(blocks)))
    assert e.value.status == B.MLC_EINVAL
    bs.set_blocks(blocks)
    bs.close()
    other.close()


def test_batch_mixed_gluing():
    """Problems with different gluing weights and overlaps share a batch; each matches its
    single-problem run bitwise and the oracle to 1e-10."""
    torch = _torch()
    from paper_1401_4969_amd import binding as B
    probs = [p.with_(overlap=ov, pou=pou) for p, (ov, pou) in
             zip(_small_batch(1, 1, n=6, seed0=300), [(0, 1), (1, 1), (2, 1), (1, 0), (0, 1), (2, 0)])]
    probs = [p for p in probs if min(p.n_coarse // p.sub_x, p.n_coarse // p.sub_y) + 2 * p.overlap >= 2]
    bs = B.BatchSolver(probs)
    bs.setup()
    bs.run()
    for i, p in enumerate(probs):
        lam, u = bs.get(i)
        lam1, u1 = _single(p)
        assert np.array_equal(lam, lam1)
        assert torch.equal(u, u1)
        assert np.allclose(lam, oracle_solve(p).lam, rtol=1e-10, atol=0)
    bs.close()


def test_batch_rejects_mixed_q_or_kind():
    _torch()
    from paper_1401_4969_amd import binding as B
    a = W.config1()
    with pytest.raises(B.MLCError):
        B.batch_workspace_size([a, a.with_(n_eig=2)])
    with pytest.raises(B.MLCError):
        B.batch_workspace_size([a, a.with_(coef_kind=1, kappa=np.ones((8, 8)))])


def _golden_c4():
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_c4.json")
    if not os.path.exists(path):
        pytest.skip("stored oracle values for configuration 4 not generated")
    with open(path) as f:
        return json.load(f)["problems"]


def test_config4_full_batch():
    """Configuration 4: 256 problems (square and L-shape, h = 1/128..1/512 of the unit
    length, 4x4..8x8 uneven subdomains, log-uniform kappa), mixed precision, one graph
    per level step.  Every problem's every level against the stored oracle values; a
    sample of problems bitwise against single-problem runs."""
    torch = _torch()
    from paper_1401_4969_amd import binding as B
    gold = _golden_c4()
    probs = W.config4()
    bs = B.BatchSolver(probs, B.default_opts(precision=1))
    bs.setup()
    lams = [[bs.get(i, with_vectors=False)[0]] for i in range(len(probs))]
    for s in range(bs.n_steps):
        bs.step(use_graph=True)
        for i, p in enumerate(probs):
            if p.n_refine >= s + 1:
                lams[i].append(bs.get(i, with_vectors=False)[0])
        st = bs.stats()
        assert st["relres_max"] <= 1e-12 * 1.0000001
    worst = 0.0
    for i, g in enumerate(gold):
        assert g["name"] == probs[i].name
        for a, b in zip(lams[i], g["lam_levels"]):
            worst = max(worst, float(np.max(np.abs(a - np.asarray(b)) / np.abs(np.asarray(b)))))
    assert worst < 1e-10, worst
    for i in (0, 17, 100, 255):
        lam, u = bs.get(i)
        lam1, u1 = _single(probs[i], precision=1)
        assert np.array_equal(lam, lam1)
        assert torch.equal(u, u1)
    # finest eigenvectors of four problems at seeded nodes, signed, against the oracle
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_c4_vectors.json")) as f:
        vec_gold = json.load(f)["problems"]
    for g in vec_gold:
        _, u = bs.get(g["index"])
        idx = torch.as_tensor(np.asarray(g["sample_nodes"]), device=u.device)
        vals = u[0].reshape(-1)[idx].cpu().numpy()
        ref = np.asarray(g["sample_values"])
        err = np.max(np.abs(vals - ref)) / np.max(np.abs(ref))
        print(f"config 4 problem {g['index']}: max sample error {err:.2e} (signed)")
        assert err < 1e-8, (g["index"], err)
    bs.close()


def test_autotune_cache_across_processes(tmp_path, monkeypatch):
    """The autotuner's choice is stored under a key of the device architecture and the
    batch's launch signature (MLC_AUTOTUNE_CACHE); a later batch with the same signature,
    here in another process, takes it from the file without timing; a batch with another
    signature gets its own line."""
    _torch()
    import subprocess
    import sys
    from paper_1401_4969_amd import binding as B
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("MLC_AUTOTUNE_CACHE", str(cache))
    probs = _small_batch(1, 1)
    bs = B.BatchSolver(probs)
    bs.setup()
    blocks = bs.autotune()
    bs.close()
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    key, *vals = lines[0].split()
    assert key.startswith("gfx") and len(vals) == 3 * len(blocks)
    assert [int(v) for v in vals[0::3]] == blocks
    # another process: the cached choice comes back without timing
    code = ("import sys; sys.path.insert(0, %r); import workloads as W\n"
            "from test_gpu_batch import _small_batch\n"
            "from paper_1401_4969_amd import binding as B\n"
            "bs = B.BatchSolver(_small_batch(1, 1)); bs.setup()\n"
            "import time; t = time.perf_counter(); b = bs.autotune(); t = time.perf_counter() - t\n"
            "print(' '.join(map(str, b)), t)\n") % os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, MLC_AUTOTUNE_CACHE=str(cache),
               PYTHONPATH=os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    *got, secs = r.stdout.split()
    assert [int(v) for v in got] == blocks
    # a different batch: a second line
    bs = B.BatchSolver(_small_batch(1, 1, n=3, seed0=900))
    bs.setup()
    bs.autotune()
    bs.close()
    assert len(cache.read_text().splitlines()) == 2
