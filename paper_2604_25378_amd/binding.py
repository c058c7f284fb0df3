"""ctypes binding of libyand (argument marshalling only).

PyTorch supplies device memory and the current stream; every step of the
method runs in the library's HIP kernels.  The binding raises if libyand.so is
missing or no GPU is visible: there is no CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libyand.so")

YAND_OK = 0
YAND_WARN_MAXITER = 1
YAND_WARN_STALL = 2
ERRORS = {
    -1: "YAND_ERR_ARG", -2: "YAND_ERR_NONFINITE", -3: "YAND_ERR_HIP",
    -4: "YAND_ERR_OOM", -5: "YAND_ERR_INDEFINITE", -6: "YAND_ERR_UNBOUNDED",
    -7: "YAND_ERR_TOO_LARGE",
}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2}
SOLVERS = {"direct": 0, "pcg": 1}
SETS = {"budget": 0, "simplex": 1}
LINESEARCH = {"exact": 0, "armijo": 1}
TRACE = {"exact": 0, "probe": 1}


class YandError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {ERRORS.get(code, code)}")
        self.code = code


class yand_opts(C.Structure):
    _fields_ = [("solver", C.c_int), ("feasible_set", C.c_int),
                ("eps", C.c_double), ("max_iter", C.c_int),
                ("max_elapsed", C.c_double), ("regularization", C.c_double),
                ("krylov_tol", C.c_double), ("krylov_maxit", C.c_int),
                ("tau", C.c_double), ("stall_recovery", C.c_int),
                ("restart_max_iter", C.c_int), ("eta", C.c_double),
                ("linesearch", C.c_int), ("dense_fp64", C.c_int),
                ("trace_mode", C.c_int), ("probes", C.c_int),
                ("probe_seed", C.c_uint64)]


class yand_info(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", C.c_int),
                ("restarts", C.c_int), ("cg_iters", C.c_int),
                ("f", C.c_double), ("gnorm", C.c_double),
                ("elapsed", C.c_double), ("lambda_used", C.c_double),
                ("oracle_passes", C.c_int64), ("hvp_passes", C.c_int64),
                ("third_passes", C.c_int64), ("ls_passes", C.c_int64),
                ("dense_traces", C.c_int64), ("kkt", C.c_double),
                ("projected_steps", C.c_int),
                ("phase_iterations", C.c_int * 3),
                ("probe_traces", C.c_int64), ("probe_cg_iters", C.c_int64),
                ("thin_traces", C.c_int64)]


class yand_mlp_opts(C.Structure):
    _fields_ = [("hidden", C.c_int), ("layers", C.c_int), ("epochs", C.c_int),
                ("lr", C.c_double), ("seed", C.c_uint64)]


WS_FEATURES = 11

_D = C.POINTER(C.c_double)
_lib = None


def load(path: str = LIB_PATH):
    """Load libyand.so and declare its signatures (no GPU needed to load)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"libyand.so not found at {path}; build it with "
            "`python -m paper_2604_25378_amd.build`")
    lib = C.CDLL(path)
    vp = C.c_void_p
    sig = {
        "yand_default_opts": (None, [C.POINTER(yand_opts)]),
        "yand_large_opts": (None, [C.POINTER(yand_opts)]),
        "yand_create": (C.c_int, [vp, C.c_int64, C.c_int64, C.c_int64, C.c_int,
                                  vp, C.POINTER(vp)]),
        "yand_destroy": (C.c_int, [vp]),
        "yand_get_mu": (C.c_int, [vp, vp]),
        "yand_eval": (C.c_int, [vp, _D, vp, _D, vp, _D]),
        "yand_hvp": (C.c_int, [vp, _D, vp, vp, vp]),
        "yand_linesearch_coeffs": (C.c_int, [vp, _D, vp, vp, _D]),
        "yand_select_step": (C.c_int, [vp, _D, C.c_double, _D]),
        "yand_affine_normal": (C.c_int, [vp, _D, _D, vp, C.POINTER(yand_opts),
                                         vp, _D]),
        "yand_mvsk_solve": (C.c_int, [vp, _D, _D, vp, C.POINTER(yand_opts),
                                      vp, C.POINTER(yand_info)]),
        "yand_mvsk_solve_R": (C.c_int, [vp, C.c_int64, C.c_int64, C.c_double,
                                        C.c_double, C.c_double, C.c_double,
                                        _D, vp]),
        "yand_mvsk_solve_R_noalloc": (C.c_int, [vp, C.c_int64, C.c_int64,
                                                C.c_double, C.c_double,
                                                C.c_double, C.c_double, _D,
                                                vp]),
        "yand_is_certified_convex": (C.c_int, [_D]),
        "yand_shape": (C.c_int, [vp, C.POINTER(C.c_int64),
                                 C.POINTER(C.c_int64), C.POINTER(C.c_int)]),
        "yand_frontier_solve": (C.c_int, [vp, C.c_int64, _D, _D, vp,
                                          C.POINTER(yand_opts), vp,
                                          C.POINTER(yand_info)]),
        "yand_batch_solve": (C.c_int, [C.c_int64, C.POINTER(vp), _D, _D,
                                       C.POINTER(vp), C.POINTER(yand_opts),
                                       C.POINTER(vp), C.POINTER(yand_info),
                                       C.c_int, C.c_int]),
        "yand_default_mlp_opts": (None, [C.POINTER(yand_mlp_opts)]),
        "yand_mlp_create": (C.c_int, [C.c_int64, C.c_int64, C.c_int, C.c_int,
                                      C.c_uint64, vp, C.POINTER(vp)]),
        "yand_mlp_destroy": (C.c_int, [vp]),
        "yand_mlp_num_params": (C.c_int64, [vp]),
        "yand_mlp_get_params": (C.c_int, [vp, vp]),
        "yand_mlp_set_params": (C.c_int, [vp, vp]),
        "yand_mlp_forward": (C.c_int, [vp, C.c_int64, vp, vp]),
        "yand_mlp_loss_grad": (C.c_int, [vp, C.c_int64, vp, vp, vp, _D]),
        "yand_mlp_adam_step": (C.c_int, [vp, vp, C.c_double]),
        "yand_reduced_coords": (C.c_int, [C.c_int64, C.c_int64, vp, vp, vp]),
        "yand_from_reduced": (C.c_int, [C.c_int64, C.c_int64, vp, vp, vp]),
        "yand_warmstart_features": (C.c_int, [vp, C.c_int64, _D, _D, _D]),
        "yand_warmstart_train": (C.c_int, [vp, C.c_int64, _D, _D, vp,
                                           C.POINTER(yand_mlp_opts),
                                           C.POINTER(vp), _D]),
        "yand_warmstart_predict": (C.c_int, [vp, vp, C.c_int64, _D, _D, vp,
                                             C.POINTER(C.c_int), _D]),
        "yand_profile_enable": (C.c_int, [vp, C.c_int]),
        "yand_project_simplex": (C.c_int, [vp, C.c_int64, C.c_double, vp]),
        "yand_kkt_residual": (C.c_int, [vp, _D, vp, C.c_double, _D]),
        "yand_return_floor": (C.c_int, [vp, _D, C.c_double,
                                        C.POINTER(yand_opts), C.c_int, _D, _D,
                                        _D, vp, C.POINTER(yand_info),
                                        C.POINTER(C.c_int)]),
        "yand_autotune": (C.c_int, [vp, _D]),
        "yand_tuning": (C.c_int, [vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "yand_profile_read": (C.c_int, [vp, C.c_int, C.c_char_p, C.c_int, _D,
                                        C.POINTER(C.c_int64)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _c4(c):
    arr = (C.c_double * 4)(*[float(v) for v in c])
    return arr


def _check(rc: int, where: str, warn_ok: bool = False):
    if rc < 0 or (rc > 0 and not warn_ok):
        raise YandError(rc, where)
    return rc


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libyand needs a visible GPU (no CPU fallback)")
    return torch


def _dev(t, n=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t, dtype=np.float64))
    t = t.to(device="cuda", dtype=torch.float64).contiguous()
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return t


def default_opts(**kw) -> yand_opts:
    o = yand_opts()
    lib = load()
    if kw.pop("large", False):
        lib.yand_large_opts(C.byref(o))
    else:
        lib.yand_default_opts(C.byref(o))
    for k, v in kw.items():
        if k == "solver":
            v = SOLVERS[v] if isinstance(v, str) else v
        if k == "feasible_set":
            v = SETS[v] if isinstance(v, str) else v
        if k == "linesearch":
            v = LINESEARCH[v] if isinstance(v, str) else v
        if k == "trace_mode":
            v = TRACE[v] if isinstance(v, str) else v
        setattr(o, k, v)
    return o


def project_simplex(y, tau: float = 0.0):
    """Euclidean projection of y onto Delta(tau) on the GPU."""
    torch = _torch()
    y = _dev(y)
    out = torch.empty_like(y)
    _check(load().yand_project_simplex(C.c_void_p(y.data_ptr()), y.numel(),
                                       float(tau), C.c_void_p(out.data_ptr())),
           "yand_project_simplex")
    return out


def is_certified_convex(c) -> bool:
    return bool(load().yand_is_certified_convex(_c4(c)))


@dataclass
class SolveInfo:
    status: int
    iterations: int
    restarts: int
    cg_iters: int
    f: float
    gnorm: float
    elapsed: float
    lambda_used: float
    oracle_passes: int
    hvp_passes: int
    third_passes: int
    ls_passes: int
    dense_traces: int
    kkt: float
    projected_steps: int
    phase_iterations: tuple
    probe_traces: int
    probe_cg_iters: int
    thin_traces: int


def _info(i) -> SolveInfo:
    d = {k: getattr(i, k) for k, _ in yand_info._fields_}
    d["phase_iterations"] = tuple(d["phase_iterations"])
    return SolveInfo(**d)


class Context:
    """A libyand context owning the centered matrix A at one precision."""

    def __init__(self, R, precision: str = "fp64", stream=None):
        torch = _torch()
        lib = load()
        R = _dev(R)
        if R.dim() != 2:
            raise ValueError("R must be T x n")
        self.T, self.n = R.shape
        self.precision = precision
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        rc = lib.yand_create(C.c_void_p(R.data_ptr()), self.T, self.n, self.n,
                             PRECISIONS[precision],
                             C.c_void_p(self._stream.cuda_stream), C.byref(h))
        _check(rc, "yand_create")
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.yand_destroy(self._h)
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

    def mu(self):
        torch = _torch()
        out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        _check(self._lib.yand_get_mu(self._h, C.c_void_p(out.data_ptr())),
               "yand_get_mu")
        return out

    def eval(self, c, w, grad: bool = True):
        torch = _torch()
        w = _dev(w, self.n)
        f = C.c_double()
        mom = (C.c_double * 4)()
        g = torch.empty(self.n, dtype=torch.float64, device="cuda") if grad else None
        rc = self._lib.yand_eval(self._h, _c4(c), C.c_void_p(w.data_ptr()),
                                 C.byref(f),
                                 C.c_void_p(g.data_ptr()) if grad else None, mom)
        _check(rc, "yand_eval")
        return f.value, g, np.array(mom[:])

    def hvp(self, c, w, v):
        torch = _torch()
        w, v = _dev(w, self.n), _dev(v, self.n)
        out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        rc = self._lib.yand_hvp(self._h, _c4(c), C.c_void_p(w.data_ptr()),
                                C.c_void_p(v.data_ptr()),
                                C.c_void_p(out.data_ptr()))
        _check(rc, "yand_hvp")
        return out

    def linesearch_coeffs(self, c, w, d):
        w, d = _dev(w, self.n), _dev(d, self.n)
        coef = (C.c_double * 5)()
        rc = self._lib.yand_linesearch_coeffs(self._h, _c4(c),
                                              C.c_void_p(w.data_ptr()),
                                              C.c_void_p(d.data_ptr()), coef)
        _check(rc, "yand_linesearch_coeffs")
        return np.array(coef[:])

    def select_step(self, coef, alpha_max=math.inf):
        arr = (C.c_double * 5)(*[float(v) for v in coef])
        al = C.c_double()
        rc = self._lib.yand_select_step(self._h, arr, float(alpha_max),
                                        C.byref(al))
        _check(rc, "yand_select_step")
        return al.value

    def kkt_residual(self, c, w, tau: float = 0.0) -> float:
        w = _dev(w, self.n)
        k = C.c_double()
        _check(self._lib.yand_kkt_residual(self._h, _c4(c),
                                           C.c_void_p(w.data_ptr()),
                                           float(tau), C.byref(k)),
               "yand_kkt_residual")
        return k.value

    def affine_normal(self, c, w, target=None, opts: yand_opts | None = None):
        torch = _torch()
        w = _dev(w, self.n)
        d = torch.empty(self.n, dtype=torch.float64, device="cuda")
        gn = C.c_double()
        tg = C.byref(C.c_double(float(target))) if target is not None else None
        rc = self._lib.yand_affine_normal(self._h, _c4(c), tg,
                                          C.c_void_p(w.data_ptr()),
                                          C.byref(opts) if opts else None,
                                          C.c_void_p(d.data_ptr()), C.byref(gn))
        _check(rc, "yand_affine_normal")
        return d, gn.value

    def solve(self, c, target=None, w0=None, opts: yand_opts | None = None,
              raise_on_warning: bool = False):
        torch = _torch()
        out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        w0d = _dev(w0, self.n) if w0 is not None else None
        info = yand_info()
        tg = C.byref(C.c_double(float(target))) if target is not None else None
        rc = self._lib.yand_mvsk_solve(
            self._h, _c4(c), tg,
            C.c_void_p(w0d.data_ptr()) if w0d is not None else None,
            C.byref(opts) if opts else None, C.c_void_p(out.data_ptr()),
            C.byref(info))
        _check(rc, "yand_mvsk_solve", warn_ok=not raise_on_warning)
        return out, _info(info)

    def return_floor(self, profile, q: float, opts: yand_opts | None = None,
                     max_rounds: int = 40):
        """Return-floor protocol: (c, w, floor, ret, info, solves) of the
        long-only solve whose mean return is closest to the q-th percentile
        of the asset means, with c2..c4 normalised from profile (p2, p3, p4).
        """
        torch = _torch()
        out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        prof = (C.c_double * 3)(*[float(v) for v in profile])
        c = (C.c_double * 4)()
        fl, ret, ns = C.c_double(), C.c_double(), C.c_int()
        info = yand_info()
        rc = self._lib.yand_return_floor(
            self._h, prof, float(q), C.byref(opts) if opts else None,
            int(max_rounds), c, C.byref(fl), C.byref(ret),
            C.c_void_p(out.data_ptr()), C.byref(info), C.byref(ns))
        _check(rc, "yand_return_floor", warn_ok=True)
        si = _info(info)
        return list(c), out, fl.value, ret.value, si, ns.value

    def frontier(self, C4, targets=None, opts: yand_opts | None = None,
                 W0=None):
        """Batched solve of B instances on this context's A (direct or PCG).

        C4: B x 4 preference vectors; targets: B return targets or None;
        W0: B x n starting weights (device) or None.
        Returns (W (B x n device tensor), [SolveInfo])."""
        torch = _torch()
        C4 = np.ascontiguousarray(np.asarray(C4, dtype=np.float64).reshape(-1, 4))
        B = C4.shape[0]
        W = torch.empty((B, self.n), dtype=torch.float64, device="cuda")
        W0d = _dev(W0, B * self.n) if W0 is not None else None
        infos = (yand_info * B)()
        tg = None
        if targets is not None:
            tga = np.ascontiguousarray(np.asarray(targets, dtype=np.float64))
            if tga.shape[0] != B:
                raise ValueError("targets must have one entry per instance")
            tg = tga.ctypes.data_as(_D)
        rc = self._lib.yand_frontier_solve(
            self._h, B, C4.ctypes.data_as(_D), tg,
            C.c_void_p(W0d.data_ptr()) if W0d is not None else None,
            C.byref(opts) if opts else None, C.c_void_p(W.data_ptr()), infos)
        _check(rc, "yand_frontier_solve", warn_ok=True)
        return W, [_info(i)
                   for i in infos]

    PASS_KINDS = ("oracle", "value", "hvp", "line", "dot", "third")

    TUNING_INTS = 15  # YAND_TUNING_INTS

    def autotune(self):
        """Time candidate launch shapes on this context and keep the fastest.

        Returns {"pass_groups": {kind: workgroups}, "chol_group": blocks,
        "pass_rows": {kind: rows per block}, "chol_step_tm": width,
        "chol_band": width, "ms": {kind or "potrf_trtri": best mean ms}}
        (0 = the built-in default)."""
        nt = self.TUNING_INTS
        rep = (C.c_double * (nt + 7))()
        _check(self._lib.yand_autotune(self._h, rep), "yand_autotune")
        r = list(rep)
        return {"pass_groups": {k: int(r[i]) for i, k in enumerate(self.PASS_KINDS)},
                "chol_group": int(r[6]),
                "pass_rows": {k: int(r[7 + i]) for i, k in enumerate(self.PASS_KINDS)},
                "chol_step_tm": int(r[13]),
                "chol_band": int(r[14]),
                "ms": {**{k: r[nt + i] for i, k in enumerate(self.PASS_KINDS)},
                       "potrf_trtri": r[nt + 6]}}

    def tuning(self, set=None):
        """Current launch-shape record (TUNING_INTS ints; 0 = default);
        optionally set it first."""
        nt = self.TUNING_INTS
        get = (C.c_int * nt)()
        if set is not None:
            if len(set) != nt:
                raise ValueError(f"a launch-shape record has {nt} entries")
            sv = (C.c_int * nt)(*[int(v) for v in set])
        else:
            sv = None
        _check(self._lib.yand_tuning(self._h, sv, get), "yand_tuning")
        return list(get)

    def profile(self, enable: bool = True):
        _check(self._lib.yand_profile_enable(self._h, int(enable)),
               "yand_profile_enable")

    def profile_read(self):
        k = self._lib.yand_profile_read(self._h, -1, None, 0, None, None)
        out = {}
        for i in range(k):
            name = C.create_string_buffer(64)
            ms = C.c_double()
            cnt = C.c_int64()
            self._lib.yand_profile_read(self._h, i, name, 64, C.byref(ms),
                                        C.byref(cnt))
            out[name.value.decode()] = (ms.value, cnt.value)
        return out


def batch_solve(contexts, C4, targets=None, opts: yand_opts | None = None,
                max_lanes: int = 64, use_graph: bool = True, W0=None,
                grouped: bool = True):
    """Batched solve where instance b runs on contexts[b] (uneven universes).
    grouped=False keeps lanes of one context on separate streams instead of
    grouped lockstep launches.

    Returns ([w_b device tensors], [SolveInfo])."""
    torch = _torch()
    lib = load()
    C4 = np.ascontiguousarray(np.asarray(C4, dtype=np.float64).reshape(-1, 4))
    B = C4.shape[0]
    if len(contexts) != B:
        raise ValueError("one context per instance")
    outs = [torch.empty(cx.n, dtype=torch.float64, device="cuda")
            for cx in contexts]
    ctx_arr = (C.c_void_p * B)(*[cx._h.value for cx in contexts])
    out_arr = (C.c_void_p * B)(*[o.data_ptr() for o in outs])
    infos = (yand_info * B)()
    tg = None
    if targets is not None:
        tga = np.ascontiguousarray(np.asarray(targets, dtype=np.float64))
        tg = tga.ctypes.data_as(_D)
    w0_arr = None
    if W0 is not None:
        starts = [_dev(w, cx.n) if w is not None else None
                  for w, cx in zip(W0, contexts)]
        w0_arr = (C.c_void_p * B)(*[w.data_ptr() if w is not None else None
                                    for w in starts])
    rc = lib.yand_batch_solve(B, ctx_arr, C4.ctypes.data_as(_D), tg, w0_arr,
                              C.byref(opts) if opts else None, out_arr, infos,
                              int(max_lanes),
                              int(bool(use_graph)) | (0 if grouped else 2))
    _check(rc, "yand_batch_solve", warn_ok=True)
    return outs, [_info(i)
                  for i in infos]


def solve_R(R, c, target=None):
    """Stateless solve (FP64 storage, direct solver, budget set)."""
    torch = _torch()
    lib = load()
    R = _dev(R)
    T, n = R.shape
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    tg = C.byref(C.c_double(float(target))) if target is not None else None
    rc = lib.yand_mvsk_solve_R(C.c_void_p(R.data_ptr()), T, n, *map(float, c),
                               tg, C.c_void_p(out.data_ptr()))
    _check(rc, "yand_mvsk_solve_R", warn_ok=True)
    return out


def solve_R_noalloc(R, c, target=None, out=None):
    """yand_mvsk_solve_R_noalloc: the stateless solve with every workspace
    taken from the library's fixed device array.  R (T x n) and out (n) are
    the caller's device buffers; out is allocated here only when None."""
    torch = _torch()
    lib = load()
    R = _dev(R)
    T, n = R.shape
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device="cuda")
    tg = C.byref(C.c_double(float(target))) if target is not None else None
    rc = lib.yand_mvsk_solve_R_noalloc(C.c_void_p(R.data_ptr()), T, n,
                                       *map(float, c), tg,
                                       C.c_void_p(out.data_ptr()))
    _check(rc, "yand_mvsk_solve_R_noalloc", warn_ok=True)
    return out


# ------------------------------------------------------------ warm start --

def default_mlp_opts(**kw) -> yand_mlp_opts:
    o = yand_mlp_opts()
    load().yand_default_mlp_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _f32(t, n=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t, dtype=np.float32))
    t = t.to(device="cuda", dtype=torch.float32).contiguous()
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return t


class Mlp:
    """Handle of a libyand FP32 network (weights, Adam state, activations)."""

    def __init__(self, handle=None, in_dim=None, out_dim=None, hidden=512,
                 layers=4, seed=0, stream=None):
        torch = _torch()
        self._lib = load()
        if handle is None:
            st = stream if stream is not None else torch.cuda.current_stream()
            handle = C.c_void_p()
            _check(self._lib.yand_mlp_create(int(in_dim), int(out_dim),
                                             int(hidden), int(layers),
                                             int(seed), C.c_void_p(st.cuda_stream),
                                             C.byref(handle)),
                   "yand_mlp_create")
        self._h = handle
        self.in_dim, self.out_dim = in_dim, out_dim
        self.hidden, self.layers = hidden, layers

    def close(self):
        if getattr(self, "_h", None):
            self._lib.yand_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_params(self) -> int:
        return int(self._lib.yand_mlp_num_params(self._h))

    def get_params(self):
        torch = _torch()
        out = torch.empty(self.num_params, dtype=torch.float32, device="cuda")
        _check(self._lib.yand_mlp_get_params(self._h, C.c_void_p(out.data_ptr())),
               "yand_mlp_get_params")
        return out

    def set_params(self, p):
        p = _f32(p, self.num_params)
        _check(self._lib.yand_mlp_set_params(self._h, C.c_void_p(p.data_ptr())),
               "yand_mlp_set_params")

    def forward(self, X):
        torch = _torch()
        X = _f32(X)
        N = X.shape[0]
        out = torch.empty((N, self.out_dim), dtype=torch.float32, device="cuda")
        _check(self._lib.yand_mlp_forward(self._h, N, C.c_void_p(X.data_ptr()),
                                          C.c_void_p(out.data_ptr())),
               "yand_mlp_forward")
        return out

    def loss_grad(self, X, Y):
        torch = _torch()
        X, Y = _f32(X), _f32(Y)
        g = torch.empty(self.num_params, dtype=torch.float32, device="cuda")
        loss = C.c_double()
        _check(self._lib.yand_mlp_loss_grad(self._h, X.shape[0],
                                            C.c_void_p(X.data_ptr()),
                                            C.c_void_p(Y.data_ptr()),
                                            C.c_void_p(g.data_ptr()),
                                            C.byref(loss)),
               "yand_mlp_loss_grad")
        return loss.value, g

    def adam_step(self, lr, grad=None):
        gp = None
        if grad is not None:
            grad = _f32(grad, self.num_params)
            gp = C.c_void_p(grad.data_ptr())
        _check(self._lib.yand_mlp_adam_step(self._h, gp, float(lr)),
               "yand_mlp_adam_step")


def reduced_coords(W, n):
    """Y = U^T (W - 1/n) row by row (device FP64, N x (n-1))."""
    torch = _torch()
    W = _dev(W).reshape(-1, n)
    Y = torch.empty((W.shape[0], n - 1), dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    _check(load().yand_reduced_coords(W.shape[0], n, C.c_void_p(W.data_ptr()),
                                      C.c_void_p(Y.data_ptr()), C.c_void_p(st)),
           "yand_reduced_coords")
    return Y


def from_reduced(Y, n):
    """W = 1/n + U Y row by row (device FP64, N x n)."""
    torch = _torch()
    Y = _dev(Y).reshape(-1, n - 1)
    W = torch.empty((Y.shape[0], n), dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    _check(load().yand_from_reduced(Y.shape[0], n, C.c_void_p(Y.data_ptr()),
                                    C.c_void_p(W.data_ptr()), C.c_void_p(st)),
           "yand_from_reduced")
    return W


def _c4_targets(C4, targets):
    C4 = np.ascontiguousarray(np.asarray(C4, dtype=np.float64).reshape(-1, 4))
    tg = None
    tga = None
    if targets is not None:
        tga = np.ascontiguousarray(np.asarray(targets, dtype=np.float64))
        if tga.shape[0] != C4.shape[0]:
            raise ValueError("targets must have one entry per instance")
        tg = tga.ctypes.data_as(_D)
    return C4, tga, tg


def warmstart_features(ctx: Context, C4, targets=None):
    C4, tga, tg = _c4_targets(C4, targets)
    F = np.zeros((C4.shape[0], WS_FEATURES))
    _check(ctx._lib.yand_warmstart_features(ctx._h, C4.shape[0],
                                            C4.ctypes.data_as(_D), tg,
                                            F.ctypes.data_as(_D)),
           "yand_warmstart_features")
    return F


def warmstart_train(ctx: Context, C4, targets, W_solved,
                    opts: yand_mlp_opts | None = None):
    """Train the warm-start network on solved instances; returns (Mlp, loss)."""
    C4, tga, tg = _c4_targets(C4, targets)
    W = _dev(W_solved, C4.shape[0] * ctx.n)
    h = C.c_void_p()
    loss = C.c_double()
    _check(ctx._lib.yand_warmstart_train(ctx._h, C4.shape[0],
                                         C4.ctypes.data_as(_D), tg,
                                         C.c_void_p(W.data_ptr()),
                                         C.byref(opts) if opts else None,
                                         C.byref(h), C.byref(loss)),
           "yand_warmstart_train")
    o = opts or default_mlp_opts()
    return Mlp(handle=h, in_dim=WS_FEATURES, out_dim=ctx.n - 1,
               hidden=o.hidden, layers=o.layers), loss.value


def warmstart_predict(ctx: Context, mlp: Mlp, C4, targets=None):
    """Warm starts (B x n device), used_mlp (B bool), gnorms (B x 2)."""
    torch = _torch()
    C4, tga, tg = _c4_targets(C4, targets)
    B = C4.shape[0]
    W0 = torch.empty((B, ctx.n), dtype=torch.float64, device="cuda")
    used = (C.c_int * B)()
    gn = np.zeros((B, 2))
    _check(ctx._lib.yand_warmstart_predict(ctx._h, mlp._h, B,
                                           C4.ctypes.data_as(_D), tg,
                                           C.c_void_p(W0.data_ptr()), used,
                                           gn.ctypes.data_as(_D)),
           "yand_warmstart_predict")
    return W0, np.array(used[:], dtype=bool), gn
