"""ctypes binding of libcr (include/cr.h): argument marshalling only.

Every numerical step runs in the HIP library; this module converts arrays, fills the option and
report structs and raises on error codes.  Host inputs are numpy arrays; device inputs are
contiguous float64 torch tensors on a ROCm device (PyTorch supplies memory and the stream).
The library must be built (``python -m paper_1608_02227_amd.build``); loading fails loudly if it
is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("CR_LIB_PATH") or os.path.join(_HERE, "libcr.so")

CR_OK, CR_EINVAL, CR_ENOMEM, CR_ENOCONV, CR_ENUMERIC, CR_EDEVICE, CR_EAGAIN, CR_ENOTFOUND = 0, -1, -2, -3, -4, -5, -6, -7
CR_ECANCELED = -8
PRECISIONS = {"fp64": 0, "mixed_fp32": 1, "mixed_bf16": 2}


class CROptions(C.Structure):
    _fields_ = [
        ("precision", C.c_int32),
        ("check_every", C.c_int32),
        ("max_iters", C.c_int64),
        ("time_budget_s", C.c_double),
        ("L", C.c_double),
        ("power_max_iters", C.c_int32),
        ("power_rtol", C.c_double),
        ("momentum", C.c_int32),
        ("certificate", C.c_int32),
        ("device", C.c_int32),
        ("stream", C.c_void_p),
        ("stall_checks", C.c_int32),
        ("step_rule", C.c_int32),
        ("upsilon", C.c_double),
        ("restart", C.c_int32),
        ("stop_rule", C.c_int32),
        ("check_rule", C.c_int32),
        ("reform_fp64", C.c_int32),
        ("center", C.c_int32),
        ("keep_lambda", C.c_int32),
        ("block_size", C.c_int32),
        ("reserved2", C.c_int32),
        ("lambda0", C.c_void_p),
    ]


class CRReport(C.Structure):
    _fields_ = [
        ("status", C.c_int32),
        ("precision", C.c_int32),
        ("iters", C.c_int64),
        ("iters_low", C.c_int64),
        ("seconds", C.c_double),
        ("preprocess_seconds", C.c_double),
        ("L", C.c_double),
        ("sigma2", C.c_double),
        ("power_iters", C.c_int32),
        ("checks", C.c_int32),
        ("kkt", C.c_double),
        ("nat_res_max", C.c_double),
        ("stat_y", C.c_double),
        ("stat_xi", C.c_double),
        ("max_viol", C.c_double),
        ("infeas_rms", C.c_double),
        ("dual_gap_paper", C.c_double),
        ("comp_sum", C.c_double),
        ("primal_obj", C.c_double),
        ("dual_obj", C.c_double),
        ("scale", C.c_double),
        ("cert_primal", C.c_double),
        ("cert_gap", C.c_double),
        ("y_err_bound", C.c_double),
        ("step_ms_low", C.c_double),
        ("step_ms_fp64", C.c_double),
        ("step_samples_low", C.c_double),
        ("step_samples_fp64", C.c_double),
        ("step_final", C.c_double),
        ("trials", C.c_double),
        ("restarts", C.c_double),
        ("adv_passes", C.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}



class CRContParams(C.Structure):
    _fields_ = [("eps0", C.c_double), ("beta", C.c_double), ("kappa_gamma", C.c_double),
                ("kappa_delta", C.c_double), ("T", C.c_int32), ("reserved", C.c_int32)]


class CRContStep(C.Structure):
    _fields_ = [("gamma", C.c_double), ("delta", C.c_double), ("iters", C.c_int64), ("status", C.c_int32),
                ("reserved", C.c_int32), ("cert_gap", C.c_double), ("kkt", C.c_double), ("xi_norm", C.c_double),
                ("seconds", C.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class CRError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"libcr error {code} ({strerror(code)}){': ' + what if what else ''}")


_lib = None
_P = C.POINTER


def load() -> C.CDLL:
    """Load libcr.so from the package directory (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch ships its own HIP runtime under the same soname (libamdhip64.so.7).  Whichever copy
    # is loaded first serves the whole process, so torch is imported before libcr: both then share
    # torch's runtime and device pointers and streams pass freely between them.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1608_02227_amd.build`")
    lib = C.CDLL(LIB_PATH)
    d, i64, i32, vp = C.c_double, C.c_int64, C.c_int32, C.c_void_p
    sig = {
        "cr_default_options": (None, [_P(CROptions)]),
        "cr_strerror": (C.c_char_p, [C.c_int]),
        "cr_device_check": (C.c_int, [C.c_int]),
        "cr_fit": (C.c_int, [i64, i64, vp, vp, d, d, _P(CROptions), vp, vp, vp, _P(CRReport)]),
        "cr_fit_device": (C.c_int, [i64, i64, vp, vp, d, d, _P(CROptions), vp, vp, vp, _P(CRReport)]),
        "cr_fit_device_noalloc": (C.c_int, [i64, i64, vp, vp, d, d, _P(CROptions), vp, vp, vp, _P(CRReport)]),
        "cr_noalloc_scratch_bytes": (C.c_size_t, []),
        "cr_noalloc_required_bytes": (C.c_size_t, [i64, i64, _P(CROptions)]),
        "cr_solver_create": (C.c_int, [i64, i64, vp, vp, d, _P(CROptions), vp, _P(vp)]),
        "cr_solver_destroy": (C.c_int, [vp]),
        "cr_solver_lipschitz": (C.c_int, [vp, _P(d), _P(d), _P(i32)]),
        "cr_solver_set_L": (C.c_int, [vp, d]),
        "cr_solver_set_delta": (C.c_int, [vp, d]),
        "cr_fit_continuation": (C.c_int, [i64, i64, vp, vp, _P(CRContParams), _P(CROptions), vp, vp, vp,
                                          _P(CRContStep), _P(CRReport)]),
        "cr_solver_iterate": (C.c_int, [vp, i64]),
        "cr_solver_solve": (C.c_int, [vp, d, _P(CRReport)]),
        "cr_solver_promote": (C.c_int, [vp]),
        "cr_solver_iterations": (i64, [vp]),
        "cr_solver_get_lambda": (C.c_int, [vp, vp]),
        "cr_solver_get_lambda_rows": (C.c_int, [vp, i64, i64, vp]),
        "cr_solver_get_primal": (C.c_int, [vp, vp, vp]),
        "cr_solver_block_iters": (C.c_int, [vp, _P(i32), i64, _P(i64)]),
        "cr_solver_report": (C.c_int, [vp, _P(CRReport)]),
        "cr_op_residual": (C.c_int, [i64, i64, vp, vp, vp, vp, C.c_int]),
        "cr_op_adjoint": (C.c_int, [i64, i64, vp, vp, vp, vp, C.c_int]),
        "cr_ctx_create": (C.c_int, [C.c_int, C.c_size_t, i32, _P(vp)]),
        "cr_ctx_destroy": (C.c_int, [vp]),
        "cr_submit": (C.c_int, [vp, i64, i64, vp, vp, d, d, _P(CROptions), _P(i64)]),
        "cr_poll": (C.c_int, [vp, i64, vp, vp, vp, _P(CRReport), _P(d)]),
        "cr_wait": (C.c_int, [vp, i64, vp, vp, vp, _P(CRReport), _P(d)]),
        "cr_ctx_stats": (C.c_int, [vp, _P(i64), _P(i64), _P(i64), _P(C.c_size_t)]),
        "cr_ctx_group_stats": (C.c_int, [vp, _P(d), _P(d), _P(d)]),
        "cr_ctx_set_grouping": (C.c_int, [vp, i64]),
        "cr_fit_state_bytes": (C.c_size_t, [i64, i64, i32]),
        "cr_pass_geometry": (C.c_int, [i64, i64, C.c_int, _P(i32), _P(i32), _P(i32), _P(i32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols() -> list[str]:
    return [name for name in dir(load()) if name.startswith("cr_")]


def strerror(code: int) -> str:
    try:
        return load().cr_strerror(code).decode()
    except ImportError:
        return "library not loaded"


def _check(code: int, what: str = "", allow=(CR_OK,)) -> int:
    if code not in allow:
        raise CRError(code, what)
    return code


@dataclass
class Options:
    precision: str = "fp64"
    check_every: int = 50
    max_iters: int = 2_000_000
    time_budget_s: float = 0.0
    L: float = 0.0
    power_max_iters: int = 300
    power_rtol: float = 0.0         # 0: 1e-8 (constant step) / 1e-2 (adaptive step)
    momentum: bool = True
    certificate: bool = True
    device: int = 0
    stream: int | None = None
    stall_checks: int = 100
    step_rule: str = "adaptive"     # "adaptive" (PAPG_A) or "constant" (PAPG_C, step 1/L)
    upsilon: float = 2.0
    restart: bool = True            # adaptive step: gradient momentum restart (not in the paper)
    stop: str = "kkt"               # "kkt": report.kkt <= tol; "gap": certified gap <= tol
    checks: str = "predict"         # "predict": next test at the extrapolated crossing of tol,
                                    # within [check_every / 5, check_every]; "fixed": every check_every
    reform_fp64: bool = False       # FP64 adaptive step: re-forming trial pass (24 B/pair) instead of
                                    # storing both candidates (32 B/pair, one FP64 contraction fewer)
    center: bool = True             # mixed modes: work in the frame x - mean(x) (results unchanged)
    keep_lambda: bool = False       # Server: keep each request's final multipliers for wait / poll
    block_size: int = 0             # > 1: K-block partial dualization with blocks of this many points
                                    # (FP64, constant step; Step 1 by an on-device interior-point method)

    def to_c(self) -> CROptions:
        o = CROptions()
        load().cr_default_options(C.byref(o))
        o.precision = PRECISIONS[self.precision]
        o.check_every = self.check_every
        o.max_iters = self.max_iters
        o.time_budget_s = self.time_budget_s
        o.L = self.L
        o.power_max_iters = self.power_max_iters
        o.power_rtol = self.power_rtol
        o.momentum = 1 if self.momentum else 0
        o.certificate = 1 if self.certificate else 0
        o.device = self.device
        o.stream = self.stream
        o.stall_checks = self.stall_checks
        o.step_rule = {"constant": 0, "adaptive": 1}[self.step_rule]
        o.upsilon = self.upsilon
        o.restart = 1 if self.restart else 0
        o.stop_rule = {"kkt": 0, "gap": 1}[self.stop]
        o.check_rule = {"fixed": 0, "predict": 1}[self.checks]
        o.reform_fp64 = 1 if self.reform_fp64 else 0
        o.center = 1 if self.center else 0
        o.keep_lambda = 1 if self.keep_lambda else 0
        o.block_size = self.block_size
        return o


def _host(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _is_torch_device(t) -> bool:
    return type(t).__module__.startswith("torch") and getattr(t, "is_cuda", False)


@dataclass
class FitResult:
    y: object
    xi: object
    lam: object | None
    report: dict
    status: int = CR_OK
    extra: dict = field(default_factory=dict)


def fit(x, ybar, delta: float, tol: float, options: Options | None = None, return_lambda: bool = False,
        allow_noconv: bool = True, no_alloc: bool = False, lambda0=None) -> FitResult:
    """One complete fit (cr_fit / cr_fit_device).  Device tensors in -> device tensors out.

    ``no_alloc`` (device tensors only) calls cr_fit_device_noalloc: the fit runs in the library's
    fixed scratch array instead of allocating device memory (outputs are still the caller's).
    ``lambda0`` (N x N, same kind as ``x``) is a warm start for the multipliers."""
    lib = load()
    opt = options or Options()
    rep = CRReport()
    allow = (CR_OK, CR_ENOCONV) if allow_noconv else (CR_OK,)
    if no_alloc and not _is_torch_device(x):
        raise ValueError("no_alloc needs device tensors (cr_fit_device_noalloc)")
    if _is_torch_device(x):
        import torch
        x = x.contiguous().to(torch.float64)
        ybar = ybar.contiguous().to(torch.float64)
        N, n = x.shape
        y = torch.empty(N, dtype=torch.float64, device=x.device)
        xi = torch.empty((N, n), dtype=torch.float64, device=x.device)
        lam = torch.empty((N, N), dtype=torch.float64, device=x.device) if return_lambda else None
        if opt.stream is None:
            opt = Options(**{**opt.__dict__, "stream": torch.cuda.current_stream(x.device).cuda_stream,
                             "device": x.device.index or 0})
        co = opt.to_c()
        if lambda0 is not None:
            if not _is_torch_device(lambda0) or tuple(lambda0.shape) != (N, N):
                raise ValueError("lambda0 must be an N x N device tensor like x")
            lambda0 = lambda0.contiguous().to(torch.float64)
            co.lambda0 = lambda0.data_ptr()
        entry = lib.cr_fit_device_noalloc if no_alloc else lib.cr_fit_device
        code = entry(N, n, C.c_void_p(x.data_ptr()), C.c_void_p(ybar.data_ptr()), delta, tol,
                     C.byref(co), C.c_void_p(y.data_ptr()), C.c_void_p(xi.data_ptr()),
                     C.c_void_p(lam.data_ptr()) if lam is not None else None, C.byref(rep))
    else:
        x = _host(x)
        N, n = x.shape
        ybar = _host(ybar, (N,))
        y = np.empty(N)
        xi = np.empty((N, n))
        lam = np.empty((N, N)) if return_lambda else None
        co = opt.to_c()
        if lambda0 is not None:
            lambda0 = _host(lambda0, (N, N))
            co.lambda0 = lambda0.ctypes.data
        code = lib.cr_fit(N, n, _ptr(x), _ptr(ybar), delta, tol, C.byref(co), _ptr(y), _ptr(xi),
                          _ptr(lam) if lam is not None else None, C.byref(rep))
    _check(code, "cr_fit", allow)
    return FitResult(y, xi, lam, rep.as_dict(), code)


def noalloc_scratch_bytes() -> int:
    return int(load().cr_noalloc_scratch_bytes())


def noalloc_required_bytes(N: int, n: int, options: Options | None = None) -> int:
    co = (options or Options()).to_c()
    return int(load().cr_noalloc_required_bytes(N, n, C.byref(co)))


def fit_continuation(x, ybar, eps0: float, beta: float, kappa_gamma: float, kappa_delta: float, T: int,
                     options: Options | None = None, return_lambda: bool = False,
                     allow_noconv: bool = True) -> FitResult:
    """Continuation to the unregularized estimator (cr_fit_continuation); host arrays.

    extra["steps"] lists one record per outer iteration t (gamma, delta, iters, status, cert_gap,
    kkt, xi_norm, seconds).
    """
    lib = load()
    opt = options or Options()
    x = _host(x)
    N, n = x.shape
    ybar = _host(ybar, (N,))
    y = np.empty(N)
    xi = np.empty((N, n))
    lam = np.empty((N, N)) if return_lambda else None
    cp = CRContParams(eps0, beta, kappa_gamma, kappa_delta, T, 0)
    steps = (CRContStep * T)()
    rep = CRReport()
    co = opt.to_c()
    code = lib.cr_fit_continuation(N, n, _ptr(x), _ptr(ybar), C.byref(cp), C.byref(co), _ptr(y), _ptr(xi),
                                   _ptr(lam) if lam is not None else None, steps, C.byref(rep))
    _check(code, "cr_fit_continuation", (CR_OK, CR_ENOCONV) if allow_noconv else (CR_OK,))
    return FitResult(y, xi, lam, rep.as_dict(), code, {"steps": [st.as_dict() for st in steps]})


class Solver:
    """Step-level access to one fit whose state stays on the device (cr_solver_*)."""

    def __init__(self, x, ybar, delta: float, options: Options | None = None, lambda0=None):
        lib = load()
        self.x = _host(x)
        self.N, self.n = self.x.shape
        self.ybar = _host(ybar, (self.N,))
        self.delta = delta
        self._opt = (options or Options()).to_c()
        lam0 = _host(lambda0, (self.N, self.N)) if lambda0 is not None else None
        h = C.c_void_p()
        _check(lib.cr_solver_create(self.N, self.n, _ptr(self.x), _ptr(self.ybar), delta, C.byref(self._opt),
                                    _ptr(lam0) if lam0 is not None else None, C.byref(h)), "cr_solver_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().cr_solver_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def lipschitz(self) -> tuple[float, float, int]:
        L, s2, it = C.c_double(), C.c_double(), C.c_int32()
        _check(load().cr_solver_lipschitz(self._h, C.byref(L), C.byref(s2), C.byref(it)), "lipschitz")
        return L.value, s2.value, it.value

    def set_L(self, L: float):
        _check(load().cr_solver_set_L(self._h, L), "set_L")

    def set_delta(self, delta: float):
        """New Tikhonov weight; lam is kept as the warm start (one continuation step)."""
        _check(load().cr_solver_set_delta(self._h, delta), "set_delta")
        self.delta = delta

    def iterate(self, iters: int):
        _check(load().cr_solver_iterate(self._h, iters), "iterate")

    def solve(self, tol: float) -> tuple[int, dict]:
        rep = CRReport()
        code = load().cr_solver_solve(self._h, tol, C.byref(rep))
        _check(code, "solve", (CR_OK, CR_ENOCONV))
        return code, rep.as_dict()

    def promote(self):
        _check(load().cr_solver_promote(self._h), "promote")

    @property
    def iterations(self) -> int:
        return int(load().cr_solver_iterations(self._h))

    def lam(self) -> np.ndarray:
        out = np.empty((self.N, self.N))
        _check(load().cr_solver_get_lambda(self._h, _ptr(out)), "get_lambda")
        return out

    def lam_rows(self, row0: int, nrows: int) -> np.ndarray:
        out = np.empty((nrows, self.N))
        _check(load().cr_solver_get_lambda_rows(self._h, row0, nrows, _ptr(out)), "get_lambda_rows")
        return out

    def block_iters(self) -> np.ndarray | None:
        """Interior-point iterations of each block's QP in the most recent Step 1 (K-block mode),
        else None."""
        nb = C.c_int64()
        _check(load().cr_solver_block_iters(self._h, None, 0, C.byref(nb)), "block_iters")
        if nb.value == 0:
            return None
        out = np.zeros(nb.value, dtype=np.int32)
        _check(load().cr_solver_block_iters(self._h, out.ctypes.data_as(C.POINTER(C.c_int32)), nb.value, C.byref(nb)),
               "block_iters")
        return out

    def primal(self) -> tuple[np.ndarray, np.ndarray]:
        y = np.empty(self.N)
        xi = np.empty((self.N, self.n))
        _check(load().cr_solver_get_primal(self._h, _ptr(y), _ptr(xi)), "get_primal")
        return y, xi

    def report(self) -> dict:
        rep = CRReport()
        _check(load().cr_solver_report(self._h, C.byref(rep)), "report", (CR_OK, CR_ENUMERIC))
        return rep.as_dict()


def op_residual(x, y, xi, device: int = 0):
    """s = C eta on device tensors (N x n, N, N x n) -> N x N device tensor."""
    import torch
    N, n = x.shape
    s = torch.empty((N, N), dtype=torch.float64, device=x.device)
    torch.cuda.synchronize(x.device)
    _check(load().cr_op_residual(N, n, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                 C.c_void_p(xi.data_ptr()), C.c_void_p(s.data_ptr()), device), "op_residual")
    return s


def op_adjoint(x, lam, device: int = 0):
    """(u, w) = C^T lam on device tensors -> (N, N x n) device tensors."""
    import torch
    N, n = x.shape
    u = torch.empty(N, dtype=torch.float64, device=x.device)
    w = torch.empty((N, n), dtype=torch.float64, device=x.device)
    torch.cuda.synchronize(x.device)
    _check(load().cr_op_adjoint(N, n, C.c_void_p(x.data_ptr()), C.c_void_p(lam.data_ptr()), C.c_void_p(u.data_ptr()),
                                C.c_void_p(w.data_ptr()), device), "op_adjoint")
    return u, w


def pass_geometry(N: int, n: int, device: int = 0) -> dict:
    """Tiling of the pair sweep (cr_pass_geometry): padded rows, chunks, columns per chunk, workgroups."""
    r, c, cc, wg = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(load().cr_pass_geometry(N, n, device, C.byref(r), C.byref(c), C.byref(cc), C.byref(wg)), "geometry")
    return {"rows": r.value, "chunks": c.value, "chunk_cols": cc.value, "workgroups": wg.value}


def state_bytes(N: int, n: int, precision: str = "fp64") -> int:
    """Device bytes a serving context reserves for one fit (cr_fit_state_bytes)."""
    return int(load().cr_fit_state_bytes(N, n, PRECISIONS[precision]))


class Server:
    """Continuous-batching fit server (cr_ctx_*): submit returns at once; wait/poll collect."""

    def __init__(self, device: int = 0, byte_budget: int = 0, max_slots: int = 4, group_max_n: int = 0):
        h = C.c_void_p()
        _check(load().cr_ctx_create(device, byte_budget, max_slots, C.byref(h)), "cr_ctx_create")
        self._h = h
        self._shapes = {}
        if group_max_n:
            self.set_grouping(group_max_n)

    def set_grouping(self, max_n: int):
        """Grouped iterations for fits with N <= max_n admitted from now on (0: off)."""
        _check(load().cr_ctx_set_grouping(self._h, max_n), "cr_ctx_set_grouping")

    def close(self):
        if getattr(self, "_h", None):
            load().cr_ctx_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def submit(self, x, ybar, delta: float, tol: float, options: Options | None = None, lambda0=None) -> int:
        """Queues a fit; ``lambda0`` (N x N, host) is an optional warm start, copied at submission."""
        x = _host(x)
        N, n = x.shape
        ybar = _host(ybar, (N,))
        rid = C.c_int64()
        opt = options or Options()
        co = opt.to_c()
        if lambda0 is not None:
            lambda0 = _host(lambda0, (N, N))
            co.lambda0 = lambda0.ctypes.data
        _check(load().cr_submit(self._h, N, n, _ptr(x), _ptr(ybar), delta, tol, C.byref(co), C.byref(rid)),
               "cr_submit")
        self._shapes[rid.value] = (N, n, bool(opt.keep_lambda))
        return rid.value

    def _collect(self, fn, rid):
        N, n, keep = self._shapes[rid]
        y = np.empty(N)
        xi = np.empty((N, n))
        lam = np.empty((N, N)) if keep else None
        rep = CRReport()
        lat = C.c_double()
        code = fn(self._h, rid, _ptr(y), _ptr(xi), _ptr(lam) if keep else None, C.byref(rep), C.byref(lat))
        if code == CR_EAGAIN:
            return None
        _check(code, "collect", (CR_OK, CR_ENOCONV))
        del self._shapes[rid]
        return FitResult(y, xi, lam, rep.as_dict(), code, {"latency_s": lat.value})

    def wait(self, rid: int) -> FitResult:
        return self._collect(load().cr_wait, rid)

    def poll(self, rid: int) -> FitResult | None:
        return self._collect(load().cr_poll, rid)

    def stats(self) -> dict:
        q, r, f, b = C.c_int64(), C.c_int64(), C.c_int64(), C.c_size_t()
        _check(load().cr_ctx_stats(self._h, C.byref(q), C.byref(r), C.byref(f), C.byref(b)), "stats")
        return {"queued": q.value, "running": r.value, "finished": f.value, "resident_bytes": b.value}

    def group_stats(self) -> dict:
        """Grouped iterations so far: rounds launched, grouped pass launches, fit rounds carried."""
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        _check(load().cr_ctx_group_stats(self._h, C.byref(a), C.byref(b), C.byref(c)), "group_stats")
        return {"rounds": a.value, "pass_launches": b.value, "fit_rounds": c.value}
