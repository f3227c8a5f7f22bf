"""Thin Python binding of liblyapsmw.so (argument marshalling only).

Every step of the method runs in the HIP library; this module converts
numpy / torch arguments to pointers and sizes.  PyTorch is used for device
memory and streams.  There is no fallback: if the library is missing or no
GPU is present, every call raises.

Entry points (names as in include/lyapsmw.h): seed_factor, lyap_seed_apply,
smw_solve_batch, trace_EX, engine_*.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblyapsmw.so")

OK, E_INVAL, E_NOMEM, E_UNSTABLE, E_NOCONV, E_BREAKDOWN, E_DEVICE, E_UNSUPPORTED, E_NONFINITE = range(9)
BASIS = {"auto": 0, "eig": 1, "schur": 2}
PREC = {"fp64": 0, "fp32_ir": 1, "bf16_ir": 2, "fp32": 3}


class LyapError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        super().__init__("%s failed: status %d (%s) %s" % (where, status, _status_str(status), detail))


class SeedOpts(C.Structure):
    _fields_ = [("basis", C.c_int32), ("E_is_diag", C.c_int32), ("max_eig_cond", C.c_double),
                ("tsvd_rank", C.c_int32), ("schur_dense", C.c_int32), ("seed_refine", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("prec", C.c_int32), ("max_iter", C.c_int32), ("restart", C.c_int32),
                ("use_precond", C.c_int32), ("recycle_k", C.c_int32), ("max_refine", C.c_int32),
                ("tol", C.c_double), ("inner_tol", C.c_double)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("cycles", C.c_int32),
                ("refinements", C.c_int32), ("rel_residual", C.c_double), ("trace", C.c_double),
                ("err_est", C.c_double)]


class SeedInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("r", C.c_int64), ("s", C.c_int64), ("npairs", C.c_int64),
                ("ld", C.c_int64), ("basis", C.c_int32), ("tsvd_rank", C.c_int32),
                ("cond_est", C.c_double), ("min_lam_sum", C.c_double),
                ("max_re_lambda", C.c_double), ("t0", C.c_double),
                ("t0_unrefined", C.c_double), ("eps_seed", C.c_double), ("seed_refine", C.c_int32),
                ("factor_seconds", C.c_double), ("device_bytes", C.c_size_t)]


class Profile(C.Structure):
    _fields_ = [("gemm64_ms", C.c_double), ("gemm64_flops", C.c_double),
                ("gemmlo_ms", C.c_double), ("gemmlo_flops", C.c_double),
                ("krylov_ms", C.c_double), ("gemm64_launches", C.c_int64),
                ("gemmlo_launches", C.c_int64), ("krylov_launches", C.c_int64),
                ("steps", C.c_int64), ("slot_steps", C.c_int64), ("graph_steps", C.c_int64),
                ("tuned_bk", C.c_int64), ("tuned_grid_min", C.c_int64), ("tuned_xcd_off", C.c_int64)]


class EkResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("level", C.c_int32), ("dim", C.c_int32),
                ("iters", C.c_int32), ("delta", C.c_double), ("trace", C.c_double)]


class EkInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("r", C.c_int64), ("level", C.c_int64), ("dim", C.c_int64),
                ("blocks", C.c_int64), ("basis_cols", C.c_int64), ("exhausted", C.c_int32),
                ("proj_basis", C.c_int32), ("proj_cond", C.c_double),
                ("basis_seconds", C.c_double), ("level_seconds", C.c_double),
                ("solve_seconds", C.c_double), ("delta_seconds", C.c_double),
                ("batches", C.c_int64)]


EK_RESULT_DTYPE = np.dtype([("status", np.int32), ("level", np.int32), ("dim", np.int32),
                            ("iters", np.int32), ("delta", np.float64), ("trace", np.float64)])

RESULT_DTYPE = np.dtype([("status", np.int32), ("iters", np.int32), ("cycles", np.int32),
                         ("refinements", np.int32), ("rel_residual", np.float64),
                         ("trace", np.float64), ("err_est", np.float64)])

_lib = None

# exported symbols of include/lyapsmw.h (checked by the CPU tests)
EXPORTS = ["seed_factor", "seed_info", "seed_release", "seed_device_bytes", "lyap_seed_apply",
           "lyap_seed_apply_noalloc",
           "smw_workspace_bytes", "smw_solve_batch", "trace_EX", "engine_create",
           "engine_device_bytes", "engine_destroy", "engine_submit", "engine_run",
           "engine_harvest", "engine_launch", "engine_status", "lyap_status_string", "lyap_last_error", "lyap_profile_enable",
           "lyap_profile_read", "lyap_calib_copy", "lyap_real_schur", "seed_full_X", "smw_solve_shifted",
           "seed_x0v", "ek_create",
           "ek_set_level", "ek_solve", "ek_sweep", "ek_info", "ek_release", "seed_unstable_count"]


def load(path: str = LIB_PATH):
    """Load the library (no GPU needed to load it)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("liblyapsmw.so not built (%s); run __graft_entry__.build()" % path)
    # the host LAPACK the library resolves at run time lives in libtorch_cpu
    import torch  # noqa: F401
    lib = C.CDLL(path, mode=C.RTLD_GLOBAL)
    vp, i64, i32, dp = C.c_void_p, C.c_int64, C.c_int32, C.POINTER(C.c_double)
    lib.seed_factor.argtypes = [i64, i64, i64, vp, vp, vp, vp, vp, C.POINTER(SeedOpts), vp,
                                C.POINTER(vp)]
    lib.seed_info.argtypes = [vp, C.POINTER(SeedInfo)]
    lib.seed_release.argtypes = [vp]
    lib.seed_device_bytes.argtypes = [vp]
    lib.seed_device_bytes.restype = C.c_size_t
    lib.lyap_seed_apply.argtypes = [vp, i64, vp, vp, i32, vp]
    lib.lyap_seed_apply_noalloc.argtypes = [vp, i64, vp, vp, i32, vp]
    lib.smw_workspace_bytes.argtypes = [vp, i64, C.POINTER(SolveOpts)]
    lib.smw_workspace_bytes.restype = C.c_size_t
    lib.smw_solve_batch.argtypes = [vp, i64, vp, C.POINTER(SolveOpts), vp, C.POINTER(Result), vp,
                                    C.c_size_t, vp]
    lib.trace_EX.argtypes = [vp, i64, vp, vp, vp]
    lib.engine_create.argtypes = [vp, i64, C.POINTER(SolveOpts), vp, C.POINTER(vp)]
    lib.engine_device_bytes.argtypes = [vp, i64, C.POINTER(SolveOpts)]
    lib.engine_device_bytes.restype = C.c_size_t
    lib.engine_destroy.argtypes = [vp]
    lib.engine_submit.argtypes = [vp, i64, vp, vp]
    lib.engine_run.argtypes = [vp, i64, i32, C.POINTER(i64)]
    lib.engine_harvest.argtypes = [vp, i64, vp, C.POINTER(Result), C.POINTER(i64)]
    lib.engine_launch.argtypes = [vp, i64]
    lib.engine_status.argtypes = [vp, C.POINTER(i64), C.POINTER(i64)]
    lib.lyap_status_string.argtypes = [i32]
    lib.lyap_status_string.restype = C.c_char_p
    lib.lyap_profile_enable.argtypes = [i32]
    lib.lyap_profile_enable.restype = None
    lib.lyap_profile_read.argtypes = [C.POINTER(Profile)]
    lib.lyap_calib_copy.argtypes = [vp, vp, C.c_size_t, vp]
    lib.lyap_real_schur.argtypes = [i64, vp, vp, vp]
    lib.lyap_real_schur.restype = C.c_int
    lib.seed_x0v.argtypes = [vp, vp]
    lib.seed_full_X.argtypes = [vp, i64, vp, vp, vp]
    lib.smw_solve_shifted.argtypes = [vp, i64, vp, C.POINTER(SolveOpts), vp, C.POINTER(Result), vp]
    lib.ek_create.argtypes = [i64, i64, vp, vp, vp, vp, C.c_double, vp, i32, vp, C.POINTER(vp)]
    lib.ek_set_level.argtypes = [vp, i32, C.POINTER(SeedOpts)]
    lib.ek_solve.argtypes = [vp, i64, vp, C.POINTER(SolveOpts), vp, vp, vp, C.POINTER(Result)]
    lib.ek_sweep.argtypes = [vp, i64, vp, C.POINTER(SolveOpts), C.POINTER(SeedOpts), C.c_double,
                             i32, i32, i32, C.POINTER(EkResult)]
    lib.ek_info.argtypes = [vp, C.POINTER(EkInfo)]
    lib.ek_release.argtypes = [vp]
    lib.lyap_last_error.argtypes = []
    lib.lyap_last_error.restype = C.c_char_p
    for name in ("seed_factor", "seed_info", "seed_release", "lyap_seed_apply",
                 "lyap_seed_apply_noalloc", "smw_solve_batch",
                 "trace_EX", "engine_create", "engine_destroy", "engine_submit", "engine_run",
                 "engine_harvest", "engine_launch", "engine_status", "lyap_profile_read",
                 "lyap_calib_copy", "seed_full_X", "smw_solve_shifted", "seed_x0v", "ek_create", "ek_set_level", "ek_solve",
                 "ek_sweep", "ek_info", "ek_release", "seed_unstable_count"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _status_str(st):
    try:
        return load().lyap_status_string(st).decode()
    except Exception:
        return "?"


def _check(st, where):
    if st != OK:
        detail = ""
        try:
            detail = load().lyap_last_error().decode()
        except Exception:
            pass
        raise LyapError(st, where, detail)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("lyapsmw needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _host(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError("expected shape %s, got %s" % (shape, a.shape))
    return a


def _dev_ptr(t, dtype_name="float64", shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("expected a CUDA tensor")
    if str(t.dtype) != "torch." + dtype_name:
        raise TypeError("expected %s, got %s" % (dtype_name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (shape, tuple(t.shape)))
    return C.c_void_p(t.data_ptr())


def _precond_mode(v) -> int:
    """True/1: all of eq:prec the seed holds; 2: block-diagonal part only; False/0: none."""
    if isinstance(v, bool):
        return 1 if v else 0
    return int(v)


def solve_opts(prec="fp64", tol=1e-12, max_iter=600, restart=None, use_precond=True,
               max_refine=30, inner_tol=1e-4, recycle_k=0) -> SolveOpts:
    """restart None: the library's default cycle (64, or 40 with recycle_k > 0)."""
    return SolveOpts(PREC[prec] if isinstance(prec, str) else int(prec), int(max_iter),
                     0 if restart is None else int(restart), _precond_mode(use_precond),
                     int(recycle_k), int(max_refine), float(tol), float(inner_tol))


class Seed:
    """seed_factor: offline stage for one (A0, U, V, B, E)."""

    def __init__(self, A0, U, V, B, E, basis="auto", max_eig_cond=0.0, stream=None,
                 tsvd_rank=0, schur_dense=True, seed_refine=0):
        lib = load()
        _torch()
        A0 = _host(A0)
        n = A0.shape[0]
        U = _host(U)
        V = _host(V)
        B = _host(B)
        E = _host(E)
        if A0.shape != (n, n) or U.ndim != 2 or U.shape[0] != n or V.shape != U.shape \
                or B.ndim != 2 or B.shape[0] != n:
            raise ValueError("inconsistent shapes")
        r, s = U.shape[1], B.shape[1]
        diag = 1 if E.ndim == 1 else 0
        if (diag and E.shape != (n,)) or (not diag and E.shape != (n, n)):
            raise ValueError("E must be (n,) or (n, n)")
        self._keep = (A0, U, V, B, E)
        opts = SeedOpts(BASIS[basis], diag, float(max_eig_cond), int(tsvd_rank),
                        0 if schur_dense else -1, int(seed_refine))
        h = C.c_void_p()
        st = lib.seed_factor(n, r, s, A0.ctypes.data, U.ctypes.data, V.ctypes.data, B.ctypes.data,
                             E.ctypes.data, C.byref(opts), _stream(stream), C.byref(h))
        _check(st, "seed_factor")
        self.h = h
        self.n, self.r, self.s = n, r, s

    @classmethod
    def from_problem(cls, pr, **kw):
        return cls(pr.A0, pr.U, pr.V, pr.B, pr.E, **kw)

    def device_bytes(self) -> int:
        return int(load().seed_device_bytes(self.h))

    def info(self) -> dict:
        inf = SeedInfo()
        _check(load().seed_info(self.h, C.byref(inf)), "seed_info")
        return {k: getattr(inf, k) for k, _ in SeedInfo._fields_}

    def release(self):
        if getattr(self, "h", None):
            load().seed_release(self.h)   # the seed's engine may use the workspace until here
            self.h = None
        self._ws = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    # ---- the seed Lyapunov solve with a low-rank right-hand side ----
    def apply(self, Y, prec="fp64", stream=None):
        torch = _torch()
        batch = Y.shape[0]
        _dev_ptr(Y, shape=(batch, self.r, self.n))
        G = torch.empty_like(Y)
        st = load().lyap_seed_apply(self.h, batch, _dev_ptr(Y), _dev_ptr(G), PREC[prec],
                                    _stream(stream))
        _check(st, "lyap_seed_apply")
        return G

    def apply_noalloc(self, Y, G, prec="fp64", stream=None):
        """lyap_seed_apply_noalloc into the caller's G (no device allocation)."""
        batch = Y.shape[0]
        _dev_ptr(Y, shape=(batch, self.r, self.n))
        _dev_ptr(G, shape=(batch, self.r, self.n))
        st = load().lyap_seed_apply_noalloc(self.h, batch, _dev_ptr(Y), _dev_ptr(G), PREC[prec],
                                            _stream(stream))
        _check(st, "lyap_seed_apply_noalloc")
        return G

    # ---- online stage ----
    def workspace_bytes(self, P, opts: Optional[SolveOpts] = None) -> int:
        opts = opts or solve_opts()
        nbytes = int(load().smw_workspace_bytes(self.h, P, C.byref(opts)))
        if nbytes == 0:
            raise LyapError(1, "smw_workspace_bytes", last_error())
        return nbytes

    def solve(self, d, opts: Optional[SolveOpts] = None, stream=None):
        """smw_solve_batch for d (P x r, CUDA float64).  Returns (Y, results)."""
        torch = _torch()
        opts = opts or solve_opts()
        P = d.shape[0]
        _dev_ptr(d, shape=(P, self.r))
        Y = torch.empty((P, self.r, self.n), dtype=torch.float64, device=d.device)
        nbytes = self.workspace_bytes(P, opts)
        # one workspace kept per seed: the library keeps its engine (graphs over
        # this memory) for the next call with the same P, options and workspace
        ws = getattr(self, "_ws", None)
        if ws is None or ws.numel() < nbytes or ws.device != d.device:
            self._ws = None
            ws = self._ws = torch.empty(nbytes, dtype=torch.uint8, device=d.device)
        res = (Result * P)()
        st = load().smw_solve_batch(self.h, P, _dev_ptr(d), C.byref(opts), _dev_ptr(Y), res,
                                    C.c_void_p(ws.data_ptr()), nbytes, _stream(stream))
        _check(st, "smw_solve_batch")
        out = np.frombuffer(bytes(res), dtype=RESULT_DTYPE).copy()
        return Y, out

    def solve_shifted(self, d, tol=1e-12, max_steps=600, want_Y=False, stream=None):
        """r = 1: one Arnoldi process for all parameters (host d, length P).
        Returns (Y or None, results)."""
        torch = _torch()
        d = _host(np.ravel(d))
        P = d.shape[0]
        Y = torch.empty((P, self.n), dtype=torch.float64, device="cuda") if want_Y else None
        opts = solve_opts(tol=tol, max_iter=max_steps)
        res = (Result * P)()
        st = load().smw_solve_shifted(self.h, P, d.ctypes.data, C.byref(opts),
                                      _dev_ptr(Y) if want_Y else None, res, _stream(stream))
        _check(st, "smw_solve_shifted")
        return Y, np.frombuffer(bytes(res), dtype=RESULT_DTYPE).copy()

    def unstable_count(self, d, stream=None):
        """Stability filter: for device d (P x r), the number of eigenvalues of
        A(p) in the open right half-plane and a flag (nonzero: the frequency
        grid cannot vouch for the count), both device int32 tensors of length P."""
        torch = _torch()
        P = d.shape[0]
        _dev_ptr(d, shape=(P, self.r))
        cnt = torch.empty(P, dtype=torch.int32, device=d.device)
        flag = torch.empty(P, dtype=torch.int32, device=d.device)
        _check(load().seed_unstable_count(self.h, P, _dev_ptr(d), _dev_ptr(cnt, "int32"),
                                          _dev_ptr(flag, "int32"), _stream(stream)),
               "seed_unstable_count")
        return cnt, flag

    def full_X(self, Y=None, stream=None):
        """X(p) (P x n x n) for the solutions Y of solve(); X0 when Y is None."""
        torch = _torch()
        if Y is None:
            X = torch.empty((1, self.n, self.n), dtype=torch.float64, device="cuda")
            _check(load().seed_full_X(self.h, 1, None, _dev_ptr(X), _stream(stream)), "seed_full_X")
            return X
        P = Y.shape[0]
        _dev_ptr(Y, shape=(P, self.r, self.n))
        X = torch.empty((P, self.n, self.n), dtype=torch.float64, device=Y.device)
        _check(load().seed_full_X(self.h, P, _dev_ptr(Y), _dev_ptr(X), _stream(stream)),
               "seed_full_X")
        return X

    def trace(self, Y, stream=None):
        torch = _torch()
        P = Y.shape[0]
        _dev_ptr(Y, shape=(P, self.r, self.n))
        t = torch.empty(P, dtype=torch.float64, device=Y.device)
        _check(load().trace_EX(self.h, P, _dev_ptr(Y), _dev_ptr(t), _stream(stream)), "trace_EX")
        return t


def seed_x0v(seed: "Seed") -> np.ndarray:
    """X0 V (n x r) of a factored seed: the first half of P for the projection framework."""
    out = np.zeros((seed.n, seed.r), dtype=np.float64)
    _check(load().seed_x0v(seed.h, out.ctypes.data), "seed_x0v")
    return out


class EKSpace:
    """Projection framework: one extended Krylov space EK_m(A0, [X0 V, U]) for all parameters."""

    def __init__(self, A0, U, V, X0V, t0, E, stream=None):
        lib = load()
        _torch()
        A0 = _host(A0)
        n = A0.shape[0]
        U, V, X0V, E = _host(U), _host(V), _host(X0V), _host(E)
        if A0.shape != (n, n) or U.ndim != 2 or U.shape[0] != n or V.shape != U.shape \
                or X0V.shape != U.shape:
            raise ValueError("inconsistent shapes")
        diag = 1 if E.ndim == 1 else 0
        if (diag and E.shape != (n,)) or (not diag and E.shape != (n, n)):
            raise ValueError("E must be (n,) or (n, n)")
        self.n, self.r = n, U.shape[1]
        self._stream = stream
        h = C.c_void_p()
        st = lib.ek_create(n, self.r, A0.ctypes.data, U.ctypes.data, V.ctypes.data, X0V.ctypes.data,
                           float(t0), E.ctypes.data, diag, _stream(stream), C.byref(h))
        _check(st, "ek_create")
        self.h = h

    @classmethod
    def from_seed(cls, seed: "Seed", A0, U, V, E, stream=None):
        """X0 V and t0 taken from a factored seed of the same (A0, U, V, B, E)."""
        return cls(A0, U, V, seed_x0v(seed), seed.info()["t0"], E, stream=stream)

    def set_level(self, m: int, basis="auto", max_eig_cond=0.0, tsvd_rank=0):
        o = SeedOpts(BASIS[basis], 0, float(max_eig_cond), int(tsvd_rank), 0, 0)
        _check(load().ek_set_level(self.h, int(m), C.byref(o)), "ek_set_level")
        return self.info()

    def solve(self, d, opts: Optional[SolveOpts] = None):
        """Projected solves at the current level for d (P x r, CUDA float64).
        Returns (W, delta, norms, results)."""
        torch = _torch()
        opts = opts or solve_opts()
        P = d.shape[0]
        _dev_ptr(d, shape=(P, self.r))
        dim = self.info()["dim"]
        W = torch.empty((P, self.r, dim), dtype=torch.float64, device=d.device)
        delta = torch.empty(P, dtype=torch.float64, device=d.device)
        norms = torch.empty((P, 2), dtype=torch.float64, device=d.device)
        res = (Result * P)()
        st = load().ek_solve(self.h, P, _dev_ptr(d), C.byref(opts), _dev_ptr(W), _dev_ptr(delta),
                             _dev_ptr(norms), res)
        _check(st, "ek_solve")
        return W, delta, norms, np.frombuffer(bytes(res), dtype=RESULT_DTYPE).copy()

    def sweep(self, d, eps: float, m_max: int, check_every: int = 1,
              opts: Optional[SolveOpts] = None, basis="auto", max_eig_cond=0.0, tsvd_rank=0,
              m_start: int = 1):
        """Algorithm EKSM_opt over host parameters d (P x r), from level m_start."""
        d = _host(d)
        P = d.shape[0]
        if d.shape != (P, self.r):
            raise ValueError("d must be P x r")
        opts = opts or solve_opts()
        po = SeedOpts(BASIS[basis], 0, float(max_eig_cond), int(tsvd_rank), 0, 0)
        out = (EkResult * P)()
        st = load().ek_sweep(self.h, P, d.ctypes.data, C.byref(opts), C.byref(po), float(eps),
                             int(m_start), int(m_max), int(check_every), out)
        _check(st, "ek_sweep")
        return np.frombuffer(bytes(out), dtype=EK_RESULT_DTYPE).copy()

    def info(self) -> dict:
        inf = EkInfo()
        _check(load().ek_info(self.h, C.byref(inf)), "ek_info")
        return {k: getattr(inf, k) for k, _ in EkInfo._fields_}

    def close(self):
        if getattr(self, "h", None):
            load().ek_release(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Engine:
    """Continuous-batching engine bound to one seed."""

    def __init__(self, seed: Seed, slots: int, opts: Optional[SolveOpts] = None, stream=None):
        lib = load()
        self.seed = seed
        self.opts = opts or solve_opts()
        h = C.c_void_p()
        _check(lib.engine_create(seed.h, int(slots), C.byref(self.opts), _stream(stream),
                                 C.byref(h)), "engine_create")
        self.h = h
        self.slots = slots
        self._queued = 0    # parameters submitted
        self._returned = 0  # results handed out by harvest

    def submit(self, d, tags=None):
        d = _host(d)
        if d.ndim != 2 or d.shape[1] != self.seed.r:
            raise ValueError("d must be (count, r)")
        tg = None
        if tags is not None:
            tg = np.ascontiguousarray(tags, dtype=np.int64)
        _check(load().engine_submit(self.h, d.shape[0], d.ctypes.data,
                                    tg.ctypes.data if tg is not None else None), "engine_submit")
        self._queued += d.shape[0]

    def run(self, max_steps=1 << 30, poll_every=8) -> int:
        busy = C.c_int64()
        _check(load().engine_run(self.h, int(max_steps), int(poll_every), C.byref(busy)),
               "engine_run")
        return busy.value

    def launch(self, steps: int):
        """Enqueue steps without waiting (engines on different streams overlap)."""
        _check(load().engine_launch(self.h, int(steps)), "engine_launch")

    def status(self):
        sub, done = C.c_int64(), C.c_int64()
        _check(load().engine_status(self.h, C.byref(sub), C.byref(done)), "engine_status")
        return sub.value, done.value

    @staticmethod
    def device_bytes(seed: "Seed", slots: int, opts: Optional[SolveOpts] = None) -> int:
        opts = opts or solve_opts()
        return int(load().engine_device_bytes(seed.h, int(slots), C.byref(opts)))

    def harvest(self, max_out=None):
        """Results of parameters finished since the last harvest (tags, records)."""
        cap = int(max_out) if max_out is not None else max(1, self._queued - self._returned)
        tags = np.zeros(cap, dtype=np.int64)
        res = (Result * cap)()
        n = C.c_int64()
        _check(load().engine_harvest(self.h, cap, tags.ctypes.data, res, C.byref(n)),
               "engine_harvest")
        k = n.value
        self._returned += k
        out = np.frombuffer(bytes(res), dtype=RESULT_DTYPE)[:k].copy()
        return tags[:k].copy(), out

    def close(self):
        if getattr(self, "h", None):
            load().engine_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def last_error() -> str:
    """The library's most recent error or diagnostic message."""
    return load().lyap_last_error().decode()


def profile_enable(on=True):
    """False/0: off; True/1: events around the Cauchy GEMMs; 2: also the Krylov kernel."""
    level = (1 if on else 0) if isinstance(on, bool) else int(on)
    load().lyap_profile_enable(level)


def profile_read() -> dict:
    p = Profile()
    _check(load().lyap_profile_read(C.byref(p)), "lyap_profile_read")
    return {k: getattr(p, k) for k, _ in Profile._fields_}


def calib_copy(src, dst, stream=None):
    """Plain device copy (byte-counter calibration); src, dst CUDA tensors of equal size."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("size mismatch")
    _check(load().lyap_calib_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes,
                                  _stream(stream)), "lyap_calib_copy")


def real_schur(A):
    """Host real Schur form of the library (A = Z T Z^T); no GPU needed."""
    A = _host(A)
    n = A.shape[0]
    T = np.zeros((n, n))
    Z = np.zeros((n, n))
    _check(load().lyap_real_schur(n, A.ctypes.data, T.ctypes.data, Z.ctypes.data), "lyap_real_schur")
    return T, Z
