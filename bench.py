#!/usr/bin/env python3
"""Benchmark of the multilevel local-and-parallel eigen-correction on one MI355X.

A step is one correction (Algorithm 4.1) at the finest level of the workload, with the
previous level's eigenpairs already resident in HBM: prolongation and residual of
(Aux_Problem), every local solve, partition-of-unity gluing, the Rayleigh-Ritz step on
V_0H + span{u~} and the new eigenvectors.  The library rewinds its ping-pong state
between steps, so every step repeats exactly the same correction.

    python bench.py [--steps K] [--warmup W] [--workload c2|c3|c3mixed|c4|c5adj|c2iface|
                     c3iface|ex62|ex62mixed] [--no-cpu-baseline]

(c4: a step is the whole multilevel run of 256 batched problems; c5adj: one reverse sweep;
*iface: the paper's own gluing in place of the partition of unity; ex62*: the operator of
Example 6.2.)

Prints one JSON line.  ``value`` is fine interior DOFs corrected per second at the finest
level (work of every eigenpair included).  ``roofline`` is for the local-solve kernel,
timed with HIP events the library records on its stream around that kernel.
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
    files = {"k_local_pcg64": ["kernels_pcg.hip", "pcg_ops.h", "mlc_device.h"],
             "k_local_mixed": ["kernels_mixed.hip", "pcg_ops.h", "mlc_device.h"]}[kernel]
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
    n = prob.n_coarse << level
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
    bs.setup()
    blocks = bs.autotune()
    print(f"[bench] c4: autotuned blocks per step {blocks}", file=sys.stderr, flush=True)
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
    bt.setup()
    bt.set_blocks(blocks)
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
                   "blocks_per_step": blocks},
        "lambda_rel_err_vs_oracle": err,
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
    raise SystemExit(f"unknown workload {name}")


def golden_lambda(name: str):
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)["lam_levels"][-1]


def cpu_baseline(prob, budget_s: float = 30.0):
    """Time the oracle's finest-level correction (one thread) on a bounded sample."""
    import numpy as np
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    from oracle import mlc as O
    ctx = threadpool_limits(1) if threadpool_limits else None
    try:
        hier = O.Hierarchy(prob)
        lam, U = O.coarse_eigs(hier, prob.n_eig)
        for k in range(prob.n_refine - 1):
            lam, U, _ = O.correction(hier, k, lam, U)
        k = prob.n_refine - 1
        # bounded sample: the local solves of as many subdomains as fit the budget, scaled
        # to the whole level by tile unknowns; residual, gluing and Rayleigh-Ritz timed whole
        m = k + 1
        import scipy.sparse.linalg as spla
        t0 = time.perf_counter()
        ubar = hier.P[k] @ U
        rhs = (hier.M[m] @ ubar) * lam[None, :] - hier.K[m] @ ubar
        t_rhs = time.perf_counter() - t0
        total_dofs = sum(hier.tile_dofs(m, s).size for s in hier.subs)
        t0 = time.perf_counter()
        sols = []
        done_dofs = 0
        for s in hier.subs:
            idx = hier.tile_dofs(m, s)
            lu = spla.splu(hier.K[m][idx][:, idx].tocsc())
            sols.append((idx, lu.solve(np.ascontiguousarray(rhs[idx]))))
            done_dofs += idx.size
            if time.perf_counter() - t0 > budget_s:
                break
        t_solve = (time.perf_counter() - t0) * total_dofs / done_dofs
        t1 = time.perf_counter()
        chi = hier.pou(m)
        ut = ubar.copy()
        for (idx, e), c in zip(sols, chi):
            ut[idx] += c[idx, None] * e
        O.rayleigh_ritz(hier, m, ut, prob.n_eig)
        t_rest = time.perf_counter() - t1 + t_rhs
        done = len(sols)
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    secs = t_solve + t_rest
    n_dofs = hier.meshes[m].dof.size
    return dict(value=n_dofs / secs, unit="fine DOFs/s", cores=1, kind="oracle",
                sample=(f"oracle finest-level correction of {prob.name}: sparse-LU local solves of "
                        f"{done} of {len(hier.subs)} subdomains timed and scaled by tile unknowns, "
                        f"gluing + Rayleigh-Ritz timed whole; 1 thread"),
                seconds_per_step=secs)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2",
                    choices=["c2", "c3", "c3mixed", "c4", "c5adj", "c2iface", "c3iface",
                             "ex62", "ex62mixed"],
                    help="c2: h = 1/512, 8x8 subdomains, q = 3 (default); c3: h = 1/2048, "
                         "16x16, FP64; c3mixed: the same in FP32 + FP64 refinement; c4: 256 "
                         "problems batched; c5adj: reverse sweep at h = 1/1024; c2iface, "
                         "c3iface: c2 / c3 with the paper's own gluing (interface problem); "
                         "ex62, ex62mixed: the operator of Example 6.2 (tensor A, weight "
                         "phi) on (-1,1)^2, H = 0.1, h = 1/320, 5x5 subdomains, q = 6")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run 4 plain device copies of 256 MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the subdomain solves of one problem run on one "
              "MI355X; multi-GPU sharding is a design note, not part of this build.",
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
    prob, okw = workload(args.workload)
    opts = B.default_opts(timing=1, block=args.block, **okw)
    s = B.Solver(prob, opts)
    s.coarse_setup()
    for _ in range(prob.n_refine):
        s.level_correct()
    print(f"[bench] {prob.name}: reached level {s.level}", file=sys.stderr, flush=True)
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
    # statistics of the same step (untimed)
    s.rewind()
    st = s.level_correct(stats=True)
    lam = np.array(st["lam"])
    n_dofs = st["n_dofs"]
    s.close()

    # algorithmic bytes of one local-solve launch
    m = prob.n_refine
    shapes = subdomain_shapes(prob)
    cw, ch = max(shapes, key=lambda x: x[0] * x[1])
    S0 = tile_levels(cw, ch, m)[0]
    nt = opts.block or 1024
    lds_limit = getattr(torch.cuda.get_device_properties(0), "shared_memory_per_block", 65536)
    tile_nx = max(c for c, _ in shapes) * (1 << m) - 1
    elem = 8 if opts.precision == 0 else 4
    rmode = ring_mode(nt, tile_nx, opts.nu, elem, lds_limit)
    # the tensor kind streams its three stiffness planes (FP64, or FP32 in inner solves)
    coef = (24 if opts.precision == 0 else 12) if prob.coef_kind == 3 else 0
    if opts.precision == 0:
        kernel = "k_local_pcg64"
        per_dof_it = pcg_bytes_per_iteration(cw, ch, m, opts.nu, mode=rmode, coef=coef) / S0
        bytes_launch = per_dof_it * st["it_dofs"] + 8.0 * st["n_tile_dofs"]
    else:
        kernel = "k_local_mixed"
        per_dof_it = pcg_bytes_per_iteration(cw, ch, m, opts.nu, elem=4, mode=rmode,
                                              coef=coef) / S0
        bytes_launch = mixed_bytes(cw, ch, m, opts.nu, st["it_dofs"], st["refine_dofs"],
                                   st["n_tile_dofs"], mode=rmode, coef=coef,
                                   coef64=24 if prob.coef_kind == 3 else 0)
    achieved = bytes_launch / (pcg_ms * 1e-3) / 1e9
    traffic = measured_traffic(kernel, prob.name)

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
        "config": {"workload": prob.name, "level": m, "h": prob.h(m), "fine_dofs": n_dofs,
                   "n_eig": prob.n_eig, "subdomains": f"{prob.sub_x}x{prob.sub_y}",
                   "overlap": prob.overlap, "precision": "fp64" if opts.precision == 0 else "mixed",
                   "local_rtol": opts.rtol,
                   "operator": ("Example 6.2: tensor A, mass weight phi, (-1,1)^2"
                                if prob.coef_kind == 3 else "kappa"),
                   "gluing": ["partition of unity (ramp)", "partition of unity (indicator)",
                              "interface problem on G_m+1"][getattr(prob, "pou", 0)]},
        "lambda": lam.tolist(),
        "lambda_rel_err_vs_oracle": lam_err,
        "local_solve": {"ms": pcg_ms, "items": st["n_items"], "tile_dofs": st["n_tile_dofs"],
                        "it_max": st["it_max"], "it_sum": st["it_sum"],
                        "refine_max": st["refine_max"], "relres_max": st["relres_max"],
                        "bytes_per_tile_dof_iter": per_dof_it, "bytes_per_launch": bytes_launch},
        "roofline": {"kernel": kernel, "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic},
    }
    if getattr(prob, "pou", 0) == 2:
        out["interface_problem"] = {"cg_iterations": st["glue_it"],
                                    "relres": st["glue_relres"]}
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
