"""Write the stored oracle values used by the GPU parity tests and the benchmark.

Calls only the CPU oracle (``oracle/``) on the seeded workloads (``workloads.py``); no
value here comes from the GPU path.  Output: tests/golden/oracle_<name>.json with the
per-level eigenvalues and, for the finest level, eigenvector values at a seeded sample
of interior nodes (each vector with non-negative nodal sum); configuration 4's per-level
eigenvalues for all 256 problems and the finest eigenvectors of four of them at seeded
nodes; and for configuration 5, central differences of the
finest eigenvalue along seeded kappa directions and with respect to 32 seeded single
cells (checks of the reverse sweep).

    python tests/golden/make_golden.py [c1 c2 c3 c5 c2iface c3iface ex62 c2p2 c3p2 c4 c4_vectors c5_fd c5_cells ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import solve  # noqa: E402

CONFIGS = {
    "c1": W.config1,
    "c2": W.config2,
    "c3": W.config3,
    "c5": W.config5,
    "c2iface": lambda: W.config2().with_(pou=2, name="c2_iface"),
    "c3iface": lambda: W.config3().with_(pou=2, name="c3_iface"),
    "ex62": lambda: W.example62(n_refine=5, sub=5, n_eig=6),
    "c2p2": W.config2_p2,
    "c3p2": W.config3_p2,
}


def make(name: str, n_samples: int = 512):
    prob = CONFIGS[name]()
    t0 = time.perf_counter()
    res = solve(prob, keep_levels=False)
    secs = time.perf_counter() - t0
    hier = res.hier
    L = prob.n_refine
    mesh = hier.meshes[L]
    rng = np.random.Generator(np.random.PCG64(1234))
    pick = np.sort(rng.choice(mesh.dof.size, size=min(n_samples, mesh.dof.size), replace=False))
    out = dict(
        name=prob.name, n_refine=L, n_eig=prob.n_eig,
        lam_levels=[l.tolist() for l in res.lam_levels],
        level_seconds=res.seconds,
        total_seconds=secs,
        sample_nodes=mesh.dof[pick].tolist(),
        sample_values=[res.U[pick, i].tolist() for i in range(prob.n_eig)],
        u_l2=[float(np.sqrt(res.U[:, i] @ res.U[:, i])) for i in range(prob.n_eig)],
        u_sum=[float(res.U[:, i].sum()) for i in range(prob.n_eig)],
        source="oracle.solve (CPU FP64), written by tests/golden/make_golden.py",
    )
    path = os.path.join(HERE, f"oracle_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"{name}: {secs:.1f} s -> {path}", flush=True)


def _one_batch_problem(i):
    prob = W.config4()[i]
    res = solve(prob, keep_levels=False)
    return dict(name=prob.name, lam_levels=[l.tolist() for l in res.lam_levels],
                seconds=float(sum(res.seconds)))


def make_batch(workers: int = 6):
    """Configuration 4: all 256 problems, per-level eigenvalues (oracle, process pool)."""
    from multiprocessing import Pool
    n = len(W.config4())
    t0 = time.perf_counter()
    with Pool(workers) as pool:
        out = pool.map(_one_batch_problem, range(n), chunksize=1)
    path = os.path.join(HERE, "oracle_c4.json")
    with open(path, "w") as f:
        json.dump(dict(problems=out, source="oracle.solve (CPU FP64), written by "
                       "tests/golden/make_golden.py from the oracle only"), f)
    print(f"c4: {time.perf_counter() - t0:.1f} s -> {path}", flush=True)


C4_VECTOR_PROBLEMS = (0, 17, 100, 255)


def make_batch_vectors(n_samples: int = 256):
    """Configuration 4: finest eigenvectors of four of the problems at seeded nodes."""
    probs = W.config4()
    t0 = time.perf_counter()
    out = []
    for i in C4_VECTOR_PROBLEMS:
        res = solve(probs[i], keep_levels=False)
        mesh = res.hier.meshes[probs[i].n_refine]
        rng = np.random.Generator(np.random.PCG64(4000 + i))
        pick = np.sort(rng.choice(mesh.dof.size, size=min(n_samples, mesh.dof.size),
                                  replace=False))
        out.append(dict(index=i, name=probs[i].name, lam=res.lam.tolist(),
                        sample_nodes=mesh.dof[pick].tolist(),
                        sample_values=res.U[pick, 0].tolist()))
    path = os.path.join(HERE, "oracle_c4_vectors.json")
    with open(path, "w") as f:
        json.dump(dict(problems=out, source="oracle.solve (CPU FP64), written by "
                       "tests/golden/make_golden.py from the oracle only"), f, indent=1)
    print(f"c4 vectors: {time.perf_counter() - t0:.1f} s -> {path}", flush=True)


def _lam_along(args):
    name, j, t = args
    prob = CONFIGS[name]()
    d = W.kappa_directions(prob.kappa)[j]
    return solve(prob.with_(kappa=prob.kappa + t * d), keep_levels=False).lam[0]


def make_fd(name: str = "c5", t: float = 1e-4, workers: int = 6):
    """Central differences (lambda(kappa + t d) - lambda(kappa - t d)) / (2 t) of the
    oracle's finest eigenvalue along the seeded directions of W.kappa_directions."""
    from multiprocessing import Pool
    nd = len(W.kappa_directions(CONFIGS[name]().kappa))
    jobs = [(name, j, s * t) for j in range(nd) for s in (1.0, -1.0)]
    t0 = time.perf_counter()
    with Pool(min(workers, len(jobs))) as pool:
        lam = pool.map(_lam_along, jobs, chunksize=1)
    fd = [(lam[2 * j] - lam[2 * j + 1]) / (2 * t) for j in range(nd)]
    path = os.path.join(HERE, f"oracle_{name}_fd.json")
    with open(path, "w") as f:
        json.dump(dict(name=CONFIGS[name]().name, t=t, lam_plus=lam[0::2], lam_minus=lam[1::2],
                       directional_fd=fd, directions="workloads.kappa_directions(kappa), seed 501",
                       source="oracle.solve (CPU FP64), written by tests/golden/make_golden.py"),
                  f, indent=1)
    print(f"{name} fd: {time.perf_counter() - t0:.1f} s -> {path}", flush=True)


def _lam_cell(args):
    name, cell, rel = args
    prob = CONFIGS[name]()
    k = prob.kappa.copy()
    k.flat[cell] *= 1.0 + rel
    return solve(prob.with_(kappa=k), keep_levels=False).lam[0]


def make_cell_fd(name: str = "c5", n_cells: int = 32, seed: int = 55,
                 steps=(1e-3, 1e-2), workers: int = 6):
    """Central differences of the oracle's finest eigenvalue with respect to single
    kappa entries (cells drawn with numpy PCG64(seed)), at two relative steps."""
    from multiprocessing import Pool
    prob = CONFIGS[name]()
    rng = np.random.Generator(np.random.PCG64(seed))
    cells = np.sort(rng.choice(prob.kappa.size, size=n_cells, replace=False)).tolist()
    jobs = [(name, c, sg * t) for t in steps for c in cells for sg in (1.0, -1.0)]
    t0 = time.perf_counter()
    with Pool(workers) as pool:
        lam = pool.map(_lam_cell, jobs, chunksize=1)
    fd = {}
    i = 0
    for t in steps:
        vals = []
        for c in cells:
            h = t * prob.kappa.flat[c]
            vals.append((lam[i] - lam[i + 1]) / (2 * h))
            i += 2
        fd[repr(t)] = vals
    path = os.path.join(HERE, f"oracle_{name}_cells.json")
    with open(path, "w") as f:
        json.dump(dict(name=prob.name, seed=seed, cells=cells, steps=list(steps), fd=fd,
                       source="oracle.solve (CPU FP64), written by tests/golden/make_golden.py"),
                  f, indent=1)
    print(f"{name} cell fd: {time.perf_counter() - t0:.1f} s -> {path}", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(CONFIGS) + ["c4", "c4_vectors", "c5_fd", "c5_cells"]):
        if n == "c4":
            make_batch()
        elif n == "c4_vectors":
            make_batch_vectors()
        elif n == "c5_fd":
            make_fd("c5")
        elif n == "c5_cells":
            make_cell_fd("c5")
        else:
            make(n)
