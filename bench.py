#!/usr/bin/env python3
"""Benchmark of the multilevel local-and-parallel eigen-correction on one MI355X.

A step is one correction (Algorithm 4.1) at the finest level of the workload, with the
previous level's eigenpairs already resident in HBM: prolongation and residual of
(Aux_Problem), every local solve, partition-of-unity gluing, the Rayleigh-Ritz step on
V_0H + span{u~} and the new eigenvectors.  The library rewinds its ping-pong state
between steps, so every step repeats exactly the same correction.

    python bench.py [--steps K] [--warmup W] [--workload c3|c2|c3mixed|c4|c5adj|c2iface|
                     c3iface|ex62|ex62mixed] [--no-cpu-baseline]

The default workload is the unit square at h = 1/2048 (4,190,209 fine DOFs, H = 1/32,
16 x 16 subdomains, q = 1) in FP64; the same workload in FP32 + FP64 refinement is
measured beside it and reported under ``mixed``.  (c4: a step is the whole multilevel run
of 256 batched problems; c5adj: one reverse sweep; *iface: the paper's own gluing in
place of the partition of unity; ex62*: the operator of Example 6.2.)

Prints one JSON line.  ``value`` is fine interior DOFs corrected per second at the finest
level (work of every eigenpair included).  ``roofline`` is for the local-solve kernel,
timed with HIP events the library records on its stream around that kernel; its
``achieved`` counts 18 vector passes of 8 bytes per tile unknown and PCG iteration (the
reference count of the method's work: SpMV with its dot 2, x/r update 6, V-cycle 7.3,
direction 3), and ``schedule_count`` gives the same figure under this kernel's own fused
schedule.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def tile_levels(cw: int, ch: int, m: int):
    """Interior node counts of a tile's nested grids, finest first."""
    return [(cw * (1 << (m - t)) - 1) * (ch * (1 << (m - t)) - 1) for t in range(m + 1)]


def ring_mode(nt: int, tile_nx: int, nu: int, elem: int = 8, lds_limit: int = 163840) -> int:
    """The library's rule for the banded smoothing passes of a tile: with nu = 2 they run
    (mode 2) when three LDS rings of nt/64 + 2 rows of the tile fit the per-workgroup
    LDS, else the sweeps run apart (mode 0)."""
    if nu != 2:
        return 0
    return 2 if 3 * (nt // 64 + 2) * tile_nx * elem + 4096 <= lds_limit else 0


def pcg_bytes_per_iteration(cw: int, ch: int, m: int, nu: int, elem: int = 8,
                            mode: int = 2, coef: int = 0) -> float:
    """Bytes the local-solve kernel must move per PCG iteration for one tile: every
    vector a pass reads or writes counted once per pass (a vector read at several
    stages of one banded pass counts once; the later reads are served from cache):
      level 0 outside the V-cycle: p = z + beta p with p.Ap (read z, p_old, write p) 3,
      x/r update with A p recomputed (read x, r, p, write x, r) 5  -> 8 passes;
      every V-cycle level t above the coarsest:
        pre-smoothing, residual and restriction: banded (mode 2) read b, write z -> 2;
        otherwise the first two sweeps from zero 2 (one sweep 2 when nu = 1), nu-2
        further sweeps 3 each, residual 3, restriction read 1;
        post-smoothing: banded (mode 2) read z, read b, write z -> 3; otherwise
        interpolation add 2 and nu sweeps 3 each;
        plus on level t+1 the restriction write 1 and the correction read 1;
      r.z rides on the last sweep of level 0;
      coarsest: read b, write z, and the dense inverse (n^2 values).
    coef: bytes per node of a stored operator (the tensor kind's three stiffness planes: 24
    in FP64, 12 in FP32), read once by every pass that applies the stiffness: on level 0 the direction and
    x/r passes, on every V-cycle level the banded pre- and post-smoothing passes (mode 2)
    or each sweep and the residual apart."""
    S = tile_levels(cw, ch, m)
    v = 0.0
    pre = 2 if (mode >= 2 and nu == 2) else 2 + 3 * max(nu - 2, 0) + 3 + 1
    post = 3 if (mode >= 2 and nu == 2) else 2 + 3 * nu
    k_passes = 2 if (mode >= 2 and nu == 2) else 1 + max(nu - 2, 0) + 1 + nu
    c = 0.0
    for t in range(m):
        v += S[t] * (pre + post) + S[t + 1] * 2
        c += S[t] * k_passes
    v += 2 * S[m] + S[m] ** 2
    c += 2 * S[0]
    return elem * (8 * S[0] + v) + coef * c


REFERENCE_PASSES = 18     # vector passes per PCG iteration in the reference count of the work


def reference_bytes_per_iteration(elem: int = 8, coef_kind: int = 0) -> float:
    """Reference count of the bytes per tile unknown and PCG iteration: 18 vector passes
    (SpMV + fused dot 2, x/r update 6, V-cycle about 7.3 fine-level passes, direction
    update 3) of elem bytes, and for a variable coefficient 2 more passes for each of the
    4 operator applications of an iteration."""
    return elem * (REFERENCE_PASSES + (8 if coef_kind != 0 else 0))


def reference_mixed_bytes(it_dofs: int, refine_dofs: int, tile_dofs: int,
                       coef_kind: int = 0) -> float:
    """The reference count for FP32 inner iterations with FP64 residual refinement: 18
    FP32 passes per inner iteration, per refinement step the FP64 residual r = b - K e
    (read b, e, write r: 24 bytes) and e += d (read e, d, write e: 20), and the first pass
    (read b, write e, r, d: 24)."""
    return (reference_bytes_per_iteration(4, coef_kind) * it_dofs + 44.0 * refine_dofs
            + 24.0 * tile_dofs)


def mixed_bytes(cw: int, ch: int, m: int, nu: int, it_dofs: int, refine_dofs: int,
                tile_dofs: int, mode: int = 2, coef: int = 0, coef64: int = 0) -> float:
    """Bytes of one mixed-precision local-solve launch: the FP32 inner iterations (the FP64
    schedule above with 4-byte elements, plus one pass per inner solve), and per
    refinement step the FP64 passes e += d (read e 8, d 4, write e 8) and r = b - K e
    (read b 8, e 8, write r 4, clear d 4, and the stored operator's FP64 planes, coef64);
    plus the first pass (read b, write e, r, d).  coef: the FP32 planes of the inner solves."""
    S0 = tile_levels(cw, ch, m)[0]
    per_it = pcg_bytes_per_iteration(cw, ch, m, nu, elem=4, mode=mode, coef=coef) / S0
    return per_it * it_dofs + (44.0 + 4.0 + coef64) * refine_dofs + 24.0 * tile_dofs


def code_text(src: str) -> str:
    """Source text without comments and blank space (a comment edit is no kernel change)."""
    import re
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(" ".join(line.split()) for line in src.splitlines() if line.strip())


def source_sha(kernel: str) -> str:
    """Hash of the code the kernel is built from (comments ignored)."""
    import hashlib
    c = os.path.join(ROOT, "paper_1401_4969_amd", "csrc")
    files = {"k_local_pcg64": ["kernels_pcg.hip", "pcg_ops.h", "mlc_launch.h", "mlc_device.h"],
             "k_local_mixed": ["kernels_mixed.hip", "pcg_ops.h", "mlc_launch.h", "mlc_device.h"],
             "k_local_p2": ["kernels_p2.hip", "p2_ops.h", "pcg_ops.h", "mlc_launch.h", "mlc_device.h"]}[kernel]
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(c, f)) as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """Counter-derived HBM bytes per launch from profiles/traffic.json, or None when the
    kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tab = json.load(f)
    rec = tab.get(f"{kernel}:{workload}")
    if not rec or rec.get("source_sha") != source_sha(kernel):
        return None
    return rec["bytes_per_launch"]


def subdomain_shapes(prob):
    """(cw, ch) of every kept Omega_j, in coarse cells (same layout rule as the library)."""
    n = prob.n_coarse
    bx = [(b * n) // prob.sub_x for b in range(prob.sub_x + 1)]
    by = [(b * n) // prob.sub_y for b in range(prob.sub_y + 1)]
    out = []
    ov = prob.overlap
    for sy in range(prob.sub_y):
        for sx in range(prob.sub_x):
            if prob.domain == 1 and bx[sx] >= n // 2 and by[sy + 1] <= n // 2:
                continue
            cw = min(n, bx[sx + 1] + ov) - max(0, bx[sx] - ov)
            ch = min(n, by[sy + 1] + ov) - max(0, by[sy] - ov)
            out.append((cw, ch))
    return out


def interior_nodes(prob, level: int) -> int:
    """Interior nodes of the level's node grid (mesh nodes for P1; vertices and edge
    midpoints, the grid of half cells, for P2)."""
    n = prob.n_coarse << (level + getattr(prob, "order", 1) - 1)
    if prob.domain != 1:
        return (n - 1) ** 2
    h = n // 2
    return (n - 1) ** 2 - h * h   # removed quadrant: nodes with i >= N/2 and j <= N/2


def bench_batch(args):
    """Configuration 4: 256 independent problems; a step is the whole multilevel run of
    the batch (every level step of every problem), each level step replayed from its
    hipGraph; value = fine DOFs corrected per second summed over problems and levels."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1401_4969_amd import binding as B
    probs = W.config4()
    opts = B.default_opts(precision=1)
    bs = B.BatchSolver(probs, opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bs.setup()   # Algorithm 4.2 step 1 for all problems (synchronises)
    setup_ms = (time.perf_counter() - t0) * 1e3
    blocks = bs.autotune()
    tuning = bs.tuning()
    print(f"[bench] c4: autotuned per step {tuning}", file=sys.stderr, flush=True)
    for _ in range(max(args.warmup, 1)):
        bs.restart()
        bs.run(use_graph=True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(bs.stream)
    for _ in range(args.steps):
        bs.restart()
        bs.run(use_graph=True)
    e1.record(bs.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    dofs = sum(interior_nodes(p, k) for p in probs for k in range(1, p.n_refine + 1))
    gold_path = os.path.join(ROOT, "tests", "golden", "oracle_c4.json")
    err = None
    if os.path.exists(gold_path):
        with open(gold_path) as f:
            gold = json.load(f)["problems"]
        err = 0.0
        for i, g in enumerate(gold):
            lam, _ = bs.get(i, with_vectors=False)
            ref = np.asarray(g["lam_levels"][-1])
            err = max(err, float(np.max(np.abs(lam - ref) / np.abs(ref))))
    # kernel time per level step without graphs (HIP events around the local solves)
    bs.close()
    opts_t = B.default_opts(precision=1, timing=1)
    bt = B.BatchSolver(probs, opts_t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.setup()   # again, with the kernels already loaded
    setup_warm_ms = (time.perf_counter() - t0) * 1e3
    bt.set_tuning(tuning)
    bt.phase_times()
    bt.run(use_graph=False)
    ph = bt.phase_times()
    bt.close()
    out = {
        "metric": "fine DOFs corrected/sec per level (1 GPU); lambda1 rel err vs FP64 oracle; HBM GB/s",
        "value": dofs / (ms * 1e-3), "unit": "fine DOFs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "c4_batch_256_problems", "problems": len(probs),
                   "fine_dofs_all_levels": dofs, "precision": "mixed", "graph": True,
                   "blocks_per_step": blocks, "nu_per_step": tuning["nu"],
                   "inner_rtol_per_step": tuning["inner_rtol"]},
        "lambda_rel_err_vs_oracle": err,
        "setup_ms": setup_warm_ms, "setup_first_call_ms": setup_ms,
        "local_solve": {"ms_all_steps": ph[0], "ms_all_steps_total": ph[1]},
    }
    print(json.dumps(out), flush=True)


def bench_adjoint(args):
    """Configuration 5 (h = 1/1024, kappa per finest cell): a step is one reverse sweep
    d lambda_1 / d kappa over all levels (1,048,576 gradient entries) after a forward run
    with the tape; value = gradient entries per second.  The forward levels are timed
    once for the ratio; the Euler identity sum kappa g = lambda and the stored oracle
    central differences along seeded directions check the result."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1401_4969_amd import binding as B
    prob = W.config5()
    s = B.Solver(prob, B.default_opts(record_tape=1))
    s.coarse_setup()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(prob.n_refine):
        s.level_correct()
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t0) * 1e3
    lam, _ = s.eigenpairs(with_vectors=False)
    for _ in range(max(args.warmup, 1)):
        g = s.backward(1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g = s.backward(1.0)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    gn = g.cpu().numpy()
    euler = abs(float(np.sum(gn * prob.kappa)) - lam[0]) / lam[0]
    fd_err = None
    path = os.path.join(ROOT, "tests", "golden", "oracle_c5_fd.json")
    if os.path.exists(path):
        with open(path) as f:
            gold = json.load(f)
        fd_err = max(abs(float(np.sum(gn * d)) - fd) / abs(fd)
                     for d, fd in zip(W.kappa_directions(prob.kappa), gold["directional_fd"]))
    s.close()
    out = {
        "metric": "d lambda_1 / d kappa entries per second (reverse sweep, 1 GPU)",
        "value": gn.size / (ms * 1e-3), "unit": "gradient entries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": prob.name + "_adjoint", "kappa_entries": int(gn.size),
                   "levels": prob.n_refine},
        "forward_all_levels_ms": fwd_ms, "backward_over_forward": ms / fwd_ms,
        "lambda": float(lam[0]), "euler_identity_rel": euler,
        "directional_fd_rel_err_vs_oracle": fd_err,
    }
    print(json.dumps(out), flush=True)


def workload(name: str):
    import workloads as W
    if name == "c2":
        return W.config2(), dict(precision=0)
    if name == "c3":
        return W.config3(), dict(precision=0)
    if name == "c3mixed":
        return W.config3(), dict(precision=1)
    if name == "c2iface":
        return W.config2().with_(pou=2, name="c2_iface"), dict(precision=0)
    if name == "c3iface":
        return W.config3().with_(pou=2, name="c3_iface"), dict(precision=0)
    if name == "ex62":
        return W.example62(n_refine=5, sub=5, n_eig=6), dict(precision=0)
    if name == "ex62mixed":
        return W.example62(n_refine=5, sub=5, n_eig=6), dict(precision=1)
    if name == "c2p2":
        return W.config2_p2(), dict(precision=0)
    if name == "c3p2":
        return W.config3_p2(), dict(precision=0)
    raise SystemExit(f"unknown workload {name}")


def golden_lambda(name: str):
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)["lam_levels"][-1]


_POOL_STATE = None   # (hierarchy, level, right-hand sides), inherited by forked workers


def _oracle_tile_solve(j: int):
    hier, m, rhs = _POOL_STATE
    from oracle import mlc as O
    return O.local_solve(hier, m, hier.subs[j], rhs)


def cpu_workers() -> int:
    """Host cores for the oracle's process pool: the CPUs this process may run on, at
    most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(prob, serial_budget_s: float = 8.0, glue_sample: int = 16):
    """The oracle's finest-level correction (Algorithm 4.1 at the last level) timed on the
    host: the local solves of every subdomain by a pool of P worker processes (the oracle's
    own per-subdomain sparse-LU solve), the right-hand side, partition-of-unity gluing and
    Rayleigh-Ritz in this process with P BLAS threads; and the same on one core (the
    local solves of as many subdomains as fit serial_budget_s, scaled by tile unknowns).
    The gluing weights (a dense subdomains x nodes array in the oracle) are evaluated for
    glue_sample subdomains and scaled by the subdomain count.  The correction starts from
    the prolonged coarse eigenpair instead of the previous level's (its cost does not
    depend on the values), so the earlier levels are not run."""
    import multiprocessing as mp
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import mlc as O
    global _POOL_STATE
    P = cpu_workers()
    t_setup = time.perf_counter()
    hier = O.Hierarchy(prob)
    lam, U0 = O.coarse_eigs(hier, prob.n_eig)
    k = prob.n_refine - 1
    m = k + 1
    u_k = hier.P0[k] @ U0
    t_setup = time.perf_counter() - t_setup

    def rhs_part():
        ubar = hier.P[k] @ u_k
        return ubar, (hier.M[m] @ ubar) * lam[None, :] - hier.K[m] @ ubar

    def glue_rr_part(ubar, sols):
        """Gluing and Rayleigh-Ritz: the weights of glue_sample subdomains timed and scaled,
        the accumulation over every subdomain (with a sampled weight row each: the same
        arithmetic), then Rayleigh-Ritz on V_0H + span{u~}."""
        ns = len(hier.subs)
        pick = list(range(0, ns, max(1, ns // glue_sample)))[:glue_sample]
        i, j = hier.node_ij(m, hier.meshes[m].dof)
        r = float(1 << m)
        t0 = time.perf_counter()
        chi = O.pou_weights(prob, [hier.subs[p] for p in pick], i / r, j / r)
        t_chi = (time.perf_counter() - t0) * ns / len(pick)
        t0 = time.perf_counter()
        ut = ubar.copy()
        for p, (idx, e) in enumerate(sols):
            ut[idx] += chi[p % len(pick)][idx, None] * e
        O.rayleigh_ritz(hier, m, ut, prob.n_eig)
        return t_chi + time.perf_counter() - t0

    out = {}
    sols = None
    for cores in (P, 1):
        if cores == 1 and P == 1 and 1 in out:
            break
        with threadpool_limits(cores):
            t0 = time.perf_counter()
            ubar, rhs = rhs_part()
            t_rhs = time.perf_counter() - t0
            if sols is None:   # every subdomain, P worker processes
                _POOL_STATE = (hier, m, rhs)
                with mp.get_context("fork").Pool(P) as pool:
                    pool.map(abs, range(P))   # workers started before the clock
                    t0 = time.perf_counter()
                    sols = pool.map(_oracle_tile_solve, range(len(hier.subs)), chunksize=1)
                    t_solve = time.perf_counter() - t0
                _POOL_STATE = None
                done = len(sols)
            else:              # one core: as many subdomains as fit the budget, scaled
                total = sum(hier.tile_dofs(m, s).size for s in hier.subs)
                t0 = time.perf_counter()
                done, done_dofs = 0, 0
                for s in hier.subs:
                    done_dofs += O.local_solve(hier, m, s, rhs)[0].size
                    done += 1
                    if time.perf_counter() - t0 > serial_budget_s:
                        break
                t_solve = (time.perf_counter() - t0) * total / done_dofs
            t_rest = glue_rr_part(ubar, sols) + t_rhs
        out[cores] = (t_solve + t_rest, t_solve, t_rest, done)
    n_dofs = hier.meshes[m].dof.size
    secs, t_solve, t_rest, _ = out[P]
    secs1, t_solve1, t_rest1, done1 = out[1]
    return dict(value=n_dofs / secs, unit="fine DOFs/s", cores=P, kind="oracle",
                sample=(f"oracle finest-level correction of {prob.name} (h = {prob.h(m):g}, "
                        f"{len(hier.subs)} subdomains): sparse-LU local solves of every subdomain "
                        f"in a pool of {P} processes; residual, gluing and Rayleigh-Ritz in one "
                        f"process with {P} BLAS threads (gluing weights sampled on "
                        f"{min(glue_sample, len(hier.subs))} subdomains and scaled); started "
                        f"from the prolonged coarse eigenpair"),
                seconds_per_step=secs, local_solve_seconds=t_solve, rest_seconds=t_rest,
                setup_seconds=t_setup,
                single_core=dict(value=n_dofs / secs1, cores=1, seconds_per_step=secs1,
                                 local_solve_seconds=t_solve1, rest_seconds=t_rest1,
                                 sample=(f"local solves of {done1} of {len(hier.subs)} subdomains "
                                         f"timed on one thread and scaled by tile unknowns")))


LLC_BYTES = 256 * 2 ** 20   # MI355X last-level (Infinity) cache


def autotuned_mixed_opts(prob, block):
    """Mixed-precision options for one problem from the library's autotuner
    (mlc_batch_autotune on a batch of this one problem): the workgroup size, nu and inner
    FP32 tolerance it picks for the finest step, which the timed step is."""
    from paper_1401_4969_amd import binding as B
    bs = B.BatchSolver([prob], B.default_opts(precision=1, block=block))
    bs.setup()
    bs.autotune()
    t = bs.tuning()
    bs.close()
    pick = {"block": t["blocks"][-1], "nu": t["nu"][-1], "inner_rtol": t["inner_rtol"][-1]}
    print(f"[bench] {prob.name} mixed: autotuned finest step {pick}", file=sys.stderr, flush=True)
    return B.default_opts(timing=1, precision=1, **pick), pick


def run_steps(prob, opts, args):
    """Bring a solver to the finest level, then time args.steps repetitions of the last
    correction (HIP events on the library's stream; the library's own events around the
    local-solve kernel), and the statistics of one more."""
    import numpy as np
    import torch
    from paper_1401_4969_amd import binding as B
    s = B.Solver(prob, opts)
    s.coarse_setup()
    for _ in range(prob.n_refine):
        s.level_correct()
    print(f"[bench] {prob.name} ({'fp64' if opts.precision == 0 else 'mixed'}): reached level "
          f"{s.level}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        s.rewind()
        s.level_correct()
    torch.cuda.synchronize()
    s.phase_times()  # reset the event accumulators
    stream = s.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        s.rewind()
        s.level_correct()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    ph = s.phase_times()
    pcg_ms = ph[0] / args.steps
    s.rewind()
    st = s.level_correct(stats=True)   # statistics of the same step (untimed)
    s.close()
    return ms_step, pcg_ms, st, np.array(st["lam"])


def roofline(prob, opts, st, pcg_ms, lds_limit):
    """The local-solve kernel against the HBM peak: algorithmic bytes of one launch by the
    reference count (18 passes per tile unknown and iteration) over its event-timed
    duration, and the same under the kernel's own fused schedule."""
    order = getattr(prob, "order", 1)
    m = prob.n_refine + order - 1   # level of the node grid (P2: the half-cell grid)
    shapes = subdomain_shapes(prob)
    cw, ch = max(shapes, key=lambda x: x[0] * x[1])
    S0 = tile_levels(cw, ch, m)[0]
    nt = opts.block or 1024
    tile_nx = max(c for c, _ in shapes) * (1 << m) - 1
    elem = 8 if opts.precision == 0 else 4
    rmode = ring_mode(nt, tile_nx, opts.nu, elem, lds_limit)
    # the tensor kind streams its three stiffness planes (FP64, or FP32 in inner solves)
    coef = (24 if opts.precision == 0 else 12) if prob.coef_kind == 3 else 0
    if opts.precision == 0:
        kernel = "k_local_pcg64" if order == 1 else "k_local_p2"
        sched_it = pcg_bytes_per_iteration(cw, ch, m, opts.nu, mode=rmode, coef=coef) / S0
        sched = sched_it * st["it_dofs"] + 8.0 * st["n_tile_dofs"]
        ref_it = reference_bytes_per_iteration(8, prob.coef_kind)
        ref_bytes = ref_it * st["it_dofs"] + 8.0 * st["n_tile_dofs"]
    else:
        kernel = "k_local_mixed"
        sched_it = pcg_bytes_per_iteration(cw, ch, m, opts.nu, elem=4, mode=rmode,
                                           coef=coef) / S0
        sched = mixed_bytes(cw, ch, m, opts.nu, st["it_dofs"], st["refine_dofs"],
                            st["n_tile_dofs"], mode=rmode, coef=coef,
                            coef64=24 if prob.coef_kind == 3 else 0)
        ref_it = reference_bytes_per_iteration(4, prob.coef_kind)
        ref_bytes = reference_mixed_bytes(st["it_dofs"], st["refine_dofs"], st["n_tile_dofs"],
                                  prob.coef_kind)
    # tile storage the launch works in (every item's vectors on every level of its V-cycle)
    ws = sum(8 * (6 * S[0] + 3 * sum(S[1:])) if opts.precision == 0 else
             8 * S[0] + 4 * (6 * S[0] + 3 * sum(S[1:]))
             for S in (tile_levels(a, b, m) for a, b in shapes)) * prob.n_eig
    achieved = ref_bytes / (pcg_ms * 1e-3) / 1e9
    a_sched = sched / (pcg_ms * 1e-3) / 1e9
    rl = {"kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
          "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
          "traffic": measured_traffic(kernel, prob.name),
          "count": (f"{ref_it:g} B per tile unknown per PCG iteration (18 vector passes of "
                    f"{elem} B{', +8 passes for the variable coefficient' if prob.coef_kind else ''}"
                    f"{'; FP64 refinement passes 44 B per unknown and step' if opts.precision else ''})"
                    f" + {8 if opts.precision == 0 else 24} B per tile unknown"),
          "bytes_per_launch": ref_bytes,
          "schedule_count": {"achieved": a_sched, "frac": a_sched / HBM_PEAK_GBS,
                             "bytes_per_launch": sched, "bytes_per_tile_dof_iter": sched_it},
          "tile_working_set_bytes": ws}
    if ws <= LLC_BYTES:
        rl["cache_resident"] = (f"the launch's tile storage ({ws / 2 ** 20:.0f} MiB) fits the "
                                f"{LLC_BYTES // 2 ** 20} MiB last-level cache: not a DRAM figure")
    return rl


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3",
                    choices=["c3", "c2", "c3mixed", "c4", "c5adj", "c2iface", "c3iface",
                             "ex62", "ex62mixed", "c2p2", "c3p2"],
                    help="c3 (default): unit square, h = 1/2048, 16x16 subdomains, q = 1, FP64, "
                         "with the same in FP32 + FP64 refinement beside it; c2: h = 1/512, "
                         "8x8 subdomains, q = 3; c3mixed: c3 in FP32 + FP64 refinement only; "
                         "c4: 256 problems batched; c5adj: reverse sweep at h = 1/1024; "
                         "c2iface, c3iface: c2 / c3 with the paper's own gluing (interface "
                         "problem); ex62, ex62mixed: the operator of Example 6.2 (tensor A, "
                         "weight phi) on (-1,1)^2, H = 0.1, h = 1/320, 5x5 subdomains, q = 6; "
                         "c2p2: P2 elements at h = 1/256 (the 261,121 dofs of c2), 8x8, q = 3; "
                         "c3p2: P2 at h = 1/512 (1,046,529 dofs), 16x16, q = 1")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="c3: skip the mixed-precision run beside the FP64 one")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run 4 plain device copies of 256 MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the subdomain solves of one problem run on one "
              "MI355X; sharding over several GPUs is described, not implemented.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1401_4969_amd import binding as B

    if args.workload == "c4":
        bench_batch(args)
        return
    if args.workload == "c5adj":
        bench_adjoint(args)
        return
    if args.calibrate_copy:
        src = torch.ones(32 * 2 ** 20, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration: 4 copies of {src.numel() * 8} bytes", file=sys.stderr,
              flush=True)
        del src, dst
    lds_limit = getattr(torch.cuda.get_device_properties(0), "shared_memory_per_block", 65536)
    prob, okw = workload(args.workload)
    opts = B.default_opts(timing=1, block=args.block, **okw)
    tuning = None
    if opts.precision == 1:
        opts, tuning = autotuned_mixed_opts(prob, args.block)
    ms_step, pcg_ms, st, lam = run_steps(prob, opts, args)
    n_dofs = st["n_dofs"]
    rl = roofline(prob, opts, st, pcg_ms, lds_limit)

    gold = golden_lambda(args.workload.replace("mixed", ""))  # ex62mixed -> ex62
    lam_err = None
    if gold is not None:
        lam_err = float(np.max(np.abs(lam - np.array(gold)) / np.abs(np.array(gold))))

    out = {
        "metric": "fine DOFs corrected/sec per level (1 GPU); lambda1 rel err vs FP64 oracle; HBM GB/s",
        "value": n_dofs / (ms_step * 1e-3),
        "unit": "fine DOFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if opts.precision == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": prob.name, "level": prob.n_refine, "h": prob.h(prob.n_refine),
                   "elements": f"P{getattr(prob, 'order', 1)}",
                   "fine_dofs": n_dofs, "n_eig": prob.n_eig,
                   "subdomains": f"{prob.sub_x}x{prob.sub_y}", "overlap": prob.overlap,
                   "precision": "fp64" if opts.precision == 0 else "mixed",
                   "local_rtol": opts.rtol,
                   "operator": ("Example 6.2: tensor A, mass weight phi, (-1,1)^2"
                                if prob.coef_kind == 3 else "kappa"),
                   "gluing": ["partition of unity (ramp)", "partition of unity (indicator)",
                              "interface problem on G_m+1"][getattr(prob, "pou", 0)]},
        "lambda": lam.tolist(),
        "lambda_rel_err_vs_oracle": lam_err,
        "local_solve": {"ms": pcg_ms, "items": st["n_items"], "tile_dofs": st["n_tile_dofs"],
                        "it_max": st["it_max"], "it_sum": st["it_sum"], "it_dofs": st["it_dofs"],
                        "refine_max": st["refine_max"], "refine_dofs": st["refine_dofs"],
                        "relres_max": st["relres_max"]},
        "roofline": rl,
    }
    if tuning is not None:
        out["config"]["tuning"] = dict(tuning, source="mlc_batch_autotune, finest step")
    if getattr(prob, "pou", 0) == 2:
        out["interface_problem"] = {"cg_iterations": st["glue_it"],
                                    "relres": st["glue_relres"]}
    if args.workload == "c3" and not args.no_mixed:
        # the same workload with FP32 inner solves and FP64 residual refinement
        mopts, mtuning = autotuned_mixed_opts(prob, args.block)
        mms, mpcg, mst, mlam = run_steps(prob, mopts, args)
        mrl = roofline(prob, mopts, mst, mpcg, lds_limit)
        out["mixed"] = {
            "value": mst["n_dofs"] / (mms * 1e-3), "unit": "fine DOFs/s", "ms_per_step": mms,
            "dtype": "f32+f64", "lambda": mlam.tolist(),
            "lambda_rel_err_vs_oracle": (None if gold is None else float(
                np.max(np.abs(mlam - np.array(gold)) / np.abs(np.array(gold))))),
            "lambda_rel_diff_vs_fp64_path": float(np.max(np.abs(mlam - lam) / np.abs(lam))),
            "speedup_vs_fp64": ms_step / mms,
            "local_solve": {"ms": mpcg, "it_max": mst["it_max"], "it_dofs": mst["it_dofs"],
                            "refine_max": mst["refine_max"], "refine_dofs": mst["refine_dofs"],
                            "relres_max": mst["relres_max"]},
            "roofline": mrl,
            "tuning": dict(mtuning, source="mlc_batch_autotune, finest step"),
        }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
