"""Thin ctypes binding of libmlc (argument marshalling only).

Every step of the method runs in the HIP library; this module only converts Python
problem descriptions to the C structs of ``include/mlc.h``, hands PyTorch device
buffers (workspace, outputs) and the current HIP stream to the library, and raises on
error statuses.  If the library is missing it raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# MLC_LIB may point at another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("MLC_LIB") or os.path.join(HERE, "_lib", "libmlc.so")

MLC_OK, MLC_EINVAL, MLC_ENOMEM, MLC_EHIP, MLC_ENOCONV, MLC_ESTATE = range(6)
STATUS_NAMES = ["MLC_OK", "MLC_EINVAL", "MLC_ENOMEM", "MLC_EHIP", "MLC_ENOCONV", "MLC_ESTATE"]

# every entry point declared in include/mlc.h
EXPORTS = [
    "mlc_default_opts", "mlc_workspace_size", "mlc_create", "mlc_coarse_setup",
    "mlc_level_correct", "mlc_run", "mlc_rewind", "mlc_current_level", "mlc_get_eigenpairs",
    "mlc_set_state", "mlc_phase_times", "mlc_destroy", "mlc_status_str", "mlc_last_error",
    "mlc_backward", "mlc_hf_gradient", "mlc_batch_workspace_size", "mlc_batch_create", "mlc_batch_setup", "mlc_batch_step",
    "mlc_batch_run", "mlc_batch_rewind", "mlc_batch_restart", "mlc_batch_current_step", "mlc_batch_get",
    "mlc_batch_step_stats", "mlc_batch_autotune", "mlc_batch_set_blocks",
    "mlc_batch_get_tuning", "mlc_batch_set_tuning",
    "mlc_batch_phase_times", "mlc_batch_destroy", "mlc_batch_last_error", "mlc_solve_static",
]


class ProblemDesc(C.Structure):
    _fields_ = [("domain", C.c_int32), ("n_coarse", C.c_int32), ("n_refine", C.c_int32),
                ("sub_x", C.c_int32), ("sub_y", C.c_int32), ("overlap", C.c_int32),
                ("n_eig", C.c_int32), ("coef_kind", C.c_int32),
                ("kappa", C.POINTER(C.c_double)), ("pou", C.c_int32), ("order", C.c_int32)]


class SolverOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("rtol", C.c_double), ("max_it", C.c_int32),
                ("max_refine", C.c_int32), ("inner_rtol", C.c_double), ("nu", C.c_int32),
                ("omega", C.c_double), ("block", C.c_int32), ("timing", C.c_int32),
                ("record_tape", C.c_int32), ("glue_graph_it", C.c_int32),
                ("smoother", C.c_int32)]


class LevelStats(C.Structure):
    _fields_ = [("level", C.c_int32), ("n_items", C.c_int32), ("h", C.c_double),
                ("n_dofs", C.c_int64), ("n_tile_dofs", C.c_int64), ("it_max", C.c_int32),
                ("refine_max", C.c_int32), ("it_sum", C.c_int64), ("it_dofs", C.c_int64),
                ("relres_max", C.c_double), ("lambda_", C.c_double * 8),
                ("refine_dofs", C.c_int64), ("glue_it", C.c_int32), ("glue_relres", C.c_double)]

    def as_dict(self, q: int) -> dict:
        return dict(level=self.level, n_items=self.n_items, h=self.h, n_dofs=self.n_dofs,
                    n_tile_dofs=self.n_tile_dofs, it_max=self.it_max,
                    refine_max=self.refine_max, it_sum=self.it_sum, it_dofs=self.it_dofs,
                    relres_max=self.relres_max, lam=list(self.lambda_[:q]),
                    refine_dofs=self.refine_dofs, glue_it=self.glue_it,
                    glue_relres=self.glue_relres)


class MLCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 6 else status}: {msg}")


_lib = None


def load_library() -> C.CDLL:
    """Load the built HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libmlc.so not found at {LIB_PATH}; build it with "
                          "`python -m paper_1401_4969_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    lib.mlc_default_opts.argtypes = [C.POINTER(SolverOpts)]
    lib.mlc_workspace_size.argtypes = [C.POINTER(ProblemDesc), C.POINTER(SolverOpts),
                                       C.POINTER(C.c_size_t)]
    lib.mlc_create.argtypes = [C.POINTER(ProblemDesc), C.POINTER(SolverOpts), P, C.c_size_t, P,
                               C.POINTER(P)]
    lib.mlc_coarse_setup.argtypes = [P]
    lib.mlc_level_correct.argtypes = [P, C.POINTER(LevelStats)]
    lib.mlc_run.argtypes = [P]
    lib.mlc_rewind.argtypes = [P]
    lib.mlc_current_level.argtypes = [P, C.POINTER(C.c_int32)]
    lib.mlc_get_eigenpairs.argtypes = [P, C.POINTER(C.c_double), P]
    lib.mlc_set_state.argtypes = [P, C.c_int32, C.POINTER(C.c_double), P]
    lib.mlc_phase_times.argtypes = [P, C.POINTER(C.c_double), C.c_int32]
    lib.mlc_destroy.argtypes = [P]
    lib.mlc_backward.argtypes = [P, C.POINTER(C.c_double), P]
    lib.mlc_hf_gradient.argtypes = [P, P]
    lib.mlc_status_str.argtypes = [C.c_int]
    lib.mlc_status_str.restype = C.c_char_p
    lib.mlc_last_error.argtypes = [P]
    lib.mlc_last_error.restype = C.c_char_p
    lib.mlc_batch_workspace_size.argtypes = [C.c_int32, C.POINTER(ProblemDesc),
                                             C.POINTER(SolverOpts), C.POINTER(C.c_size_t)]
    lib.mlc_batch_create.argtypes = [C.c_int32, C.POINTER(ProblemDesc), C.POINTER(SolverOpts), P,
                                     C.c_size_t, P, C.POINTER(P)]
    lib.mlc_batch_setup.argtypes = [P]
    lib.mlc_batch_step.argtypes = [P, C.c_int32]
    lib.mlc_batch_run.argtypes = [P, C.c_int32]
    lib.mlc_batch_rewind.argtypes = [P]
    lib.mlc_batch_restart.argtypes = [P]
    lib.mlc_batch_current_step.argtypes = [P, C.POINTER(C.c_int32)]
    lib.mlc_batch_get.argtypes = [P, C.c_int32, C.POINTER(C.c_double), P]
    lib.mlc_batch_step_stats.argtypes = [P, C.POINTER(LevelStats)]
    lib.mlc_batch_autotune.argtypes = [P, C.POINTER(C.c_int32), C.c_int32]
    lib.mlc_batch_set_blocks.argtypes = [P, C.POINTER(C.c_int32), C.c_int32]
    lib.mlc_batch_get_tuning.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                         C.POINTER(C.c_double), C.c_int32]
    lib.mlc_batch_set_tuning.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                         C.POINTER(C.c_double), C.c_int32]
    lib.mlc_batch_phase_times.argtypes = [P, C.POINTER(C.c_double), C.c_int32]
    lib.mlc_batch_destroy.argtypes = [P]
    lib.mlc_solve_static.argtypes = [C.POINTER(ProblemDesc), C.POINTER(SolverOpts), P,
                                      C.POINTER(C.c_double), P]
    lib.mlc_batch_last_error.argtypes = [P]
    lib.mlc_batch_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("mlc_status_str", "mlc_last_error", "mlc_batch_last_error"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def default_opts(**kw) -> SolverOpts:
    o = SolverOpts()
    load_library().mlc_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def make_desc(prob) -> Tuple[ProblemDesc, Optional[np.ndarray]]:
    """C descriptor for a ``workloads.Problem``-like object; returns the kappa array that
    must stay alive while the descriptor is used."""
    kap = None
    d = ProblemDesc(int(prob.domain), int(prob.n_coarse), int(prob.n_refine), int(prob.sub_x),
                    int(prob.sub_y), int(prob.overlap), int(prob.n_eig), int(prob.coef_kind),
                    None, int(getattr(prob, "pou", 0)), int(getattr(prob, "order", 1)))
    if prob.coef_kind != 0:
        kap = np.ascontiguousarray(prob.kappa, dtype=np.float64)
        d.kappa = kap.ctypes.data_as(C.POINTER(C.c_double))
    return d, kap


def workspace_size(prob, opts: Optional[SolverOpts] = None) -> int:
    lib = load_library()
    opts = opts or default_opts()
    d, _k = make_desc(prob)
    n = C.c_size_t(0)
    st = lib.mlc_workspace_size(C.byref(d), C.byref(opts), C.byref(n))
    if st != MLC_OK:
        raise MLCError(st, "mlc_workspace_size rejected the problem")
    return int(n.value)


class Solver:
    """One problem on one GPU: owns the torch workspace and the library context."""

    def __init__(self, prob, opts: Optional[SolverOpts] = None, device: str = "cuda:0",
                 stream=None):
        import torch
        self.lib = load_library()
        self.prob = prob
        self.opts = opts or default_opts()
        self.device = torch.device(device)
        self.q = int(prob.n_eig)
        d, self._kap = make_desc(prob)
        self.ws_bytes = workspace_size(prob, self.opts)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = C.c_void_p()
        st = self.lib.mlc_create(C.byref(d), C.byref(self.opts), C.c_void_p(self.ws.data_ptr()),
                                 C.c_size_t(self.ws_bytes), C.c_void_p(self.stream.cuda_stream),
                                 C.byref(self.ctx))
        if st != MLC_OK:
            raise MLCError(st, "mlc_create failed (see stderr)")

    def _check(self, st: int, what: str):
        if st != MLC_OK:
            raise MLCError(st, f"{what}: {self.lib.mlc_last_error(self.ctx).decode()}")

    def coarse_setup(self):
        self._check(self.lib.mlc_coarse_setup(self.ctx), "mlc_coarse_setup")

    def level_correct(self, stats: bool = False) -> Optional[dict]:
        if stats:
            s = LevelStats()
            st = self.lib.mlc_level_correct(self.ctx, C.byref(s))
            if st == MLC_ENOCONV:
                d = s.as_dict(self.q)
                d["enoconv"] = True
                return d
            self._check(st, "mlc_level_correct")
            return s.as_dict(self.q)
        self._check(self.lib.mlc_level_correct(self.ctx, None), "mlc_level_correct")
        return None

    def run(self):
        self._check(self.lib.mlc_run(self.ctx), "mlc_run")

    def rewind(self):
        self._check(self.lib.mlc_rewind(self.ctx), "mlc_rewind")

    @property
    def level(self) -> int:
        v = C.c_int32(0)
        self._check(self.lib.mlc_current_level(self.ctx, C.byref(v)), "mlc_current_level")
        return int(v.value)

    def grid_n(self, level: Optional[int] = None) -> int:
        """Nodes per side of the level's grid vectors (twice the cells' intervals for P2)."""
        lv = self.level if level is None else level
        return (self.prob.n_coarse << (lv + int(getattr(self.prob, "order", 1)) - 1)) + 1

    def eigenpairs(self, with_vectors: bool = True):
        """(lambda numpy[q], u torch[q, n1, n1] float64 on the device or None)."""
        import torch
        lam = np.zeros(self.q)
        u = None
        uptr = None
        if with_vectors:
            n1 = self.grid_n()
            u = torch.empty((self.q, n1, n1), dtype=torch.float64, device=self.device)
            uptr = C.c_void_p(u.data_ptr())
        self._check(self.lib.mlc_get_eigenpairs(self.ctx, lam.ctypes.data_as(C.POINTER(C.c_double)),
                                                uptr), "mlc_get_eigenpairs")
        return lam, u

    def set_state(self, level: int, lam: np.ndarray, u):
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        self._check(self.lib.mlc_set_state(self.ctx, int(level),
                                           lam.ctypes.data_as(C.POINTER(C.c_double)),
                                           C.c_void_p(u.data_ptr())), "mlc_set_state")

    def phase_times(self) -> List[float]:
        ms = (C.c_double * 2)()
        self._check(self.lib.mlc_phase_times(self.ctx, ms, 2), "mlc_phase_times")
        return [ms[0], ms[1]]

    def _kappa_shape(self):
        p = self.prob
        if p.coef_kind == 2:
            n = p.n_coarse << p.n_refine
            return (n, n)
        return (p.n_coarse, p.n_coarse)

    def backward(self, lambda_bar: float = 1.0):
        """lambda_bar * d lambda_1 / d kappa (torch float64 on the device, kappa's layout)."""
        import torch
        out = torch.empty(self._kappa_shape(), dtype=torch.float64, device=self.device)
        lb = C.c_double(lambda_bar)
        self._check(self.lib.mlc_backward(self.ctx, C.byref(lb), C.c_void_p(out.data_ptr())),
                    "mlc_backward")
        return out

    def hf_gradient(self):
        import torch
        out = torch.empty(self._kappa_shape(), dtype=torch.float64, device=self.device)
        self._check(self.lib.mlc_hf_gradient(self.ctx, C.c_void_p(out.data_ptr())),
                    "mlc_hf_gradient")
        return out

    def close(self):
        if self.ctx:
            self.lib.mlc_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(prob, opts: Optional[SolverOpts] = None, device: str = "cuda:0", stats: bool = True):
    """Algorithm 4.2 end to end on the GPU: returns (lambda, u, per-level lambdas, stats)."""
    s = Solver(prob, opts, device)
    s.coarse_setup()
    lam0, _ = s.eigenpairs(with_vectors=False)
    levels = [lam0]
    st = []
    for _ in range(prob.n_refine):
        d = s.level_correct(stats=stats)
        if stats:
            st.append(d)
            levels.append(np.array(d["lam"]))
    lam, u = s.eigenpairs()
    if not stats:
        levels.append(lam)
    s.close()
    return lam, u, levels, st


def solve_static(prob, opts: Optional[SolverOpts] = None, device: str = "cuda:0",
                 with_vectors: bool = True):
    """mlc_solve_static: the whole solve in the library's static device scratch (no device
    allocation by the library; the output vectors here are torch's)."""
    import torch
    lib = load_library()
    opts = opts or default_opts()
    d, _k = make_desc(prob)
    q = int(prob.n_eig)
    lam = np.zeros(q)
    u = None
    if with_vectors:
        n1 = (prob.n_coarse << (prob.n_refine + int(getattr(prob, "order", 1)) - 1)) + 1
        u = torch.empty((q, n1, n1), dtype=torch.float64, device=device)
    stream = torch.cuda.current_stream(torch.device(device))
    st = lib.mlc_solve_static(C.byref(d), C.byref(opts), C.c_void_p(stream.cuda_stream),
                              lam.ctypes.data_as(C.POINTER(C.c_double)),
                              C.c_void_p(u.data_ptr()) if u is not None else None)
    if st != MLC_OK:
        raise MLCError(st, "mlc_solve_static failed (see stderr)")
    return lam, u


def _problem_with_kappa(prob, kappa: np.ndarray):
    """A Problem-like record equal to ``prob`` with ``kappa`` replaced."""
    from types import SimpleNamespace
    f = {k: getattr(prob, k) for k in ("domain", "n_coarse", "n_refine", "sub_x", "sub_y",
                                       "overlap", "n_eig", "coef_kind")}
    f["pou"] = getattr(prob, "pou", 0)
    f["order"] = getattr(prob, "order", 1)
    return SimpleNamespace(kappa=kappa, **f)


_autograd_cls = None


def _multilevel_eigen_cls():
    global _autograd_cls
    if _autograd_cls is not None:
        return _autograd_cls
    import torch

    class MultilevelEigen(torch.autograd.Function):
        """lambda_1 of the multilevel correction as a function of the coefficient kappa
        (per coarse cell or per finest cell, float64); the backward pass is the library's
        reverse sweep (mlc_backward).  ``prob`` supplies everything but kappa."""

        @staticmethod
        def forward(ctx, kappa, prob, opts=None):
            if int(prob.n_eig) != 1 or int(prob.coef_kind) not in (1, 2):
                raise ValueError("MultilevelEigen needs n_eig = 1 and coef_kind 1 or 2")
            k = np.ascontiguousarray(kappa.detach().to("cpu", torch.float64).numpy())
            p = _problem_with_kappa(prob, k)
            o = SolverOpts.from_buffer_copy(opts if opts is not None else default_opts())
            o.record_tape = 1 if ctx.needs_input_grad[0] else 0
            dev = kappa.device if kappa.is_cuda else torch.device("cuda:0")
            s = Solver(p, o, device=str(dev))
            s.coarse_setup()
            s.run()
            lam, _ = s.eigenpairs(with_vectors=False)
            if o.record_tape:
                ctx.solver = s
            else:
                s.close()
            ctx.kappa_device = kappa.device
            return torch.tensor(lam[0], dtype=torch.float64, device=kappa.device)

        @staticmethod
        def backward(ctx, grad_lam):
            s = ctx.solver
            g = s.backward(float(grad_lam))
            s.close()
            ctx.solver = None
            return g.to(ctx.kappa_device), None, None

    _autograd_cls = MultilevelEigen
    return _autograd_cls


def __getattr__(name):
    if name == "MultilevelEigen":
        return _multilevel_eigen_cls()
    raise AttributeError(name)


def eigenvalue(kappa, prob, opts: Optional[SolverOpts] = None):
    """Differentiable lambda_1(kappa): ``MultilevelEigen.apply(kappa, prob, opts)``."""
    return _multilevel_eigen_cls().apply(kappa, prob, opts)


def batch_workspace_size(probs, opts: Optional[SolverOpts] = None) -> int:
    lib = load_library()
    opts = opts or default_opts()
    descs, _keep = _desc_array(probs)
    n = C.c_size_t(0)
    st = lib.mlc_batch_workspace_size(len(probs), descs, C.byref(opts), C.byref(n))
    if st != MLC_OK:
        raise MLCError(st, "mlc_batch_workspace_size rejected the batch")
    return int(n.value)


def _desc_array(probs):
    arr = (ProblemDesc * len(probs))()
    keep = []
    for i, p in enumerate(probs):
        d, k = make_desc(p)
        arr[i] = d
        keep.append(k)
    return arr, keep


class BatchSolver:
    """Many independent problems on one GPU: one launch per kernel and level step."""

    def __init__(self, probs, opts: Optional[SolverOpts] = None, device: str = "cuda:0",
                 stream=None):
        import torch
        self.lib = load_library()
        self.probs = list(probs)
        self.opts = opts or default_opts()
        self.device = torch.device(device)
        self.q = int(self.probs[0].n_eig)
        self._descs, self._keep = _desc_array(self.probs)
        self.ws_bytes = batch_workspace_size(self.probs, self.opts)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.b = C.c_void_p()
        st = self.lib.mlc_batch_create(len(self.probs), self._descs, C.byref(self.opts),
                                       C.c_void_p(self.ws.data_ptr()), C.c_size_t(self.ws_bytes),
                                       C.c_void_p(self.stream.cuda_stream), C.byref(self.b))
        if st != MLC_OK:
            raise MLCError(st, "mlc_batch_create failed (see stderr)")

    def _check(self, st: int, what: str):
        if st != MLC_OK:
            raise MLCError(st, f"{what}: {self.lib.mlc_batch_last_error(self.b).decode()}")

    @property
    def n_steps(self) -> int:
        return max(p.n_refine for p in self.probs)

    def setup(self):
        self._check(self.lib.mlc_batch_setup(self.b), "mlc_batch_setup")

    def step(self, use_graph: bool = False):
        self._check(self.lib.mlc_batch_step(self.b, int(use_graph)), "mlc_batch_step")

    def run(self, use_graph: bool = False):
        self._check(self.lib.mlc_batch_run(self.b, int(use_graph)), "mlc_batch_run")

    def rewind(self):
        self._check(self.lib.mlc_batch_rewind(self.b), "mlc_batch_rewind")

    def restart(self):
        self._check(self.lib.mlc_batch_restart(self.b), "mlc_batch_restart")

    @property
    def current_step(self) -> int:
        v = C.c_int32(0)
        self._check(self.lib.mlc_batch_current_step(self.b, C.byref(v)), "mlc_batch_current_step")
        return int(v.value)

    def stats(self) -> dict:
        s = LevelStats()
        st = self.lib.mlc_batch_step_stats(self.b, C.byref(s))
        d = s.as_dict(self.q)
        if st == MLC_ENOCONV:
            d["enoconv"] = True
            return d
        self._check(st, "mlc_batch_step_stats")
        return d

    def get(self, i: int, with_vectors: bool = True):
        import torch
        lam = np.zeros(self.q)
        u = None
        uptr = None
        if with_vectors:
            p = self.probs[i]
            lvl = min(self.current_step, p.n_refine)
            n1 = (p.n_coarse << (lvl + int(getattr(p, "order", 1)) - 1)) + 1
            u = torch.empty((self.q, n1, n1), dtype=torch.float64, device=self.device)
            uptr = C.c_void_p(u.data_ptr())
        self._check(self.lib.mlc_batch_get(self.b, int(i), lam.ctypes.data_as(C.POINTER(C.c_double)),
                                           uptr), "mlc_batch_get")
        return lam, u

    def autotune(self) -> List[int]:
        out = (C.c_int32 * self.n_steps)()
        self._check(self.lib.mlc_batch_autotune(self.b, out, self.n_steps), "mlc_batch_autotune")
        return list(out)

    def set_blocks(self, blocks: List[int]):
        arr = (C.c_int32 * len(blocks))(*blocks)
        self._check(self.lib.mlc_batch_set_blocks(self.b, arr, len(blocks)), "mlc_batch_set_blocks")

    def tuning(self) -> dict:
        """Per-step local-solve settings: lists of blocks, nu and inner_rtol."""
        n = self.n_steps
        bl, nu, tol = (C.c_int32 * n)(), (C.c_int32 * n)(), (C.c_double * n)()
        self._check(self.lib.mlc_batch_get_tuning(self.b, bl, nu, tol, n), "mlc_batch_get_tuning")
        return {"blocks": list(bl), "nu": list(nu), "inner_rtol": list(tol)}

    def set_tuning(self, tuning: dict):
        n = len(tuning["blocks"])
        bl = (C.c_int32 * n)(*tuning["blocks"])
        nu = (C.c_int32 * n)(*tuning["nu"])
        tol = (C.c_double * n)(*tuning["inner_rtol"])
        self._check(self.lib.mlc_batch_set_tuning(self.b, bl, nu, tol, n), "mlc_batch_set_tuning")

    def phase_times(self) -> List[float]:
        ms = (C.c_double * 2)()
        self._check(self.lib.mlc_batch_phase_times(self.b, ms, 2), "mlc_batch_phase_times")
        return [ms[0], ms[1]]

    def close(self):
        if self.b:
            self.lib.mlc_batch_destroy(self.b)
            self.b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
