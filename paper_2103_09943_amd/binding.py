"""Thin ctypes binding of libllp (include/llp.h).

Argument marshalling only: every step of the solve runs in the HIP library.  Tensors are torch CUDA (HIP)
tensors used as device memory; the current torch stream is passed through.  If the library has not been
built, every entry point raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libllp.so")

# llp_status values
OK, NOT_CONVERGED = 0, 1
E_ARG, E_SHAPE, E_UNSUPPORTED, E_HIP, E_OOM, E_BREAKDOWN, E_NONFINITE = -1, -2, -3, -4, -5, -6, -7


class Shape(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("h", ctypes.c_int), ("w", ctypes.c_int), ("c", ctypes.c_int),
                ("n", ctypes.c_int)]


class Params(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int), ("lam", ctypes.c_float), ("eps", ctypes.c_float),
                ("max_iters", ctypes.c_int), ("tol", ctypes.c_float), ("init_mode", ctypes.c_int),
                ("precond", ctypes.c_int)]


class Report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("true_rel_residual", ctypes.c_double), ("objective", ctypes.c_double), ("init", ctypes.c_int),
                ("out_rel_residual", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelTimes(ctypes.Structure):
    _fields_ = [("apply_ms", ctypes.c_double), ("apply_launches", ctypes.c_longlong),
                ("dir_ms", ctypes.c_double), ("dir_launches", ctypes.c_longlong),
                ("pc_rows_ms", ctypes.c_double), ("pc_rows_launches", ctypes.c_longlong),
                ("pc_cols_ms", ctypes.c_double), ("pc_cols_launches", ctypes.c_longlong),
                ("pc_rows_inv_ms", ctypes.c_double), ("pc_rows_inv_launches", ctypes.c_longlong),
                ("ref_ms", ctypes.c_double), ("ref_passes", ctypes.c_longlong)]


class TuneResult(ctypes.Structure):
    _fields_ = [("fast", ctypes.c_int), ("dir_rows", ctypes.c_int), ("apply_variant", ctypes.c_int),
                ("seg_rows", ctypes.c_int), ("us_per_iter", ctypes.c_double), ("default_us_per_iter", ctypes.c_double),
                ("candidates", ctypes.c_int)]


class KernelEstParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("l", ctypes.c_int), ("lam_w", ctypes.c_double), ("alpha1", ctypes.c_double),
                ("alpha2", ctypes.c_double), ("mu1", ctypes.c_double), ("mu2", ctypes.c_double),
                ("mu3", ctypes.c_double), ("rho", ctypes.c_double), ("t_max", ctypes.c_int), ("th", ctypes.c_double)]


class KernelEstReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("change", ctypes.c_double)]


class LlpError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {status_str(status)} ({status})")
        self.status = status


_lib = None
_vp = ctypes.c_void_p
_SIGS = {
    "llp_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int]),
    "llp_destroy": (None, [_vp]),
    "llp_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "llp_validate": (ctypes.c_int, [ctypes.POINTER(Shape), ctypes.POINTER(Params)]),
    "llp_pansharpen": (ctypes.c_int, [_vp, ctypes.POINTER(Shape), ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp,
                                      ctypes.POINTER(Report), _vp]),
    "llp_pan_stats": (ctypes.c_int, [_vp, ctypes.POINTER(Shape), ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp]),
    "llp_rhs": (ctypes.c_int, [_vp, ctypes.POINTER(Shape), _vp, _vp, _vp, _vp]),
    "llp_apply_A": (ctypes.c_int, [_vp, ctypes.POINTER(Shape), ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp]),
    "llp_apply_data": (ctypes.c_int, [_vp, ctypes.POINTER(Shape), ctypes.POINTER(Params), _vp, _vp, _vp, _vp]),
    "llp_apply_llp": (ctypes.c_int, [_vp, ctypes.POINTER(Shape), ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp]),
    "llp_precond_apply": (ctypes.c_int, [_vp, ctypes.POINTER(Shape), ctypes.POINTER(Params), _vp, _vp, _vp, _vp,
                                         _vp]),
    "llp_apply_data_fourier": (ctypes.c_int, [_vp, ctypes.POINTER(Shape), ctypes.POINTER(Params), _vp, _vp, _vp,
                                              _vp]),
    "llp_polish": (ctypes.c_int, [_vp, ctypes.POINTER(Shape), ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp, _vp]),
    "llp_apply_A_noalloc": (ctypes.c_int, [ctypes.POINTER(Shape), ctypes.POINTER(Params), _vp, _vp, _vp, _vp, _vp]),
    "llp_apply_prior": (ctypes.c_int, [_vp, ctypes.POINTER(Shape), ctypes.POINTER(Params), ctypes.c_int, _vp, _vp,
                                       _vp, _vp, ctypes.c_int, _vp]),
    "llp_prior_pansharpen": (ctypes.c_int, [_vp, ctypes.POINTER(Shape), ctypes.POINTER(Params), ctypes.c_int, _vp,
                                            _vp, _vp, _vp, _vp, ctypes.POINTER(Report), _vp]),
    "llp_estimate_kernel": (ctypes.c_int, [_vp, ctypes.POINTER(KernelEstParams), ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp,
                                           ctypes.POINTER(KernelEstReport), _vp]),
    "llp_set_profiling": (ctypes.c_int, [_vp, ctypes.c_int]),
    "llp_get_kernel_times": (ctypes.c_int, [_vp, ctypes.POINTER(KernelTimes), ctypes.c_int]),
    "llp_objective": (ctypes.c_int, [_vp, ctypes.POINTER(Shape), ctypes.POINTER(Params), _vp, _vp, _vp, _vp,
                                     ctypes.POINTER(ctypes.c_double), _vp]),
    "llp_autotune": (ctypes.c_int, [_vp, ctypes.POINTER(Shape), ctypes.POINTER(Params), _vp, _vp, _vp, _vp,
                                    ctypes.c_int, _vp, _vp]),
    "llp_autotune_batch": (ctypes.c_int, [_vp, ctypes.POINTER(Shape), ctypes.POINTER(Params), _vp, _vp, _vp,
                                          ctypes.c_int, ctypes.c_int, _vp, _vp]),
    "llp_tune_save": (ctypes.c_int, [_vp, ctypes.c_char_p]),
    "llp_tune_load": (ctypes.c_int, [_vp, ctypes.c_char_p]),
    "llp_tune_clear": (ctypes.c_int, [_vp]),
    "llp_tune_count": (ctypes.c_int, [_vp]),
    "llp_cnn_set_weights": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int]),
    "llp_cnn_get_weights": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int]),
    "llp_cnn_warm_start": (ctypes.c_int, [_vp, ctypes.POINTER(Shape), _vp, _vp, _vp, _vp, _vp]),
    "llp_cnn_loss_grad": (ctypes.c_int, [_vp, ctypes.POINTER(Shape), _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_float), _vp]),
    "llp_cnn_train_step": (ctypes.c_int, [_vp, ctypes.POINTER(Shape), _vp, _vp, _vp, ctypes.c_float,
                                          ctypes.POINTER(ctypes.c_double), _vp]),
    "llp_pansharpen_batch": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(Shape), ctypes.POINTER(Params),
                                            ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                            ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(Report),
                                            ctypes.c_int, _vp]),
}

BATCH_NO_GRAPH = 1
BATCH_SERIAL = 2
BATCH_AUTOTUNE = 4
CNN_PARAMS = 28641
INIT_ZERO, INIT_USER, INIT_NET, INIT_NET_REJECTED = 0, 1, 2, 3
PRIORS = {"llp": 0, "lgc": 1, "lpp": 2, "lpf": 3, "hpf": 4}  # llp_prior


def lib() -> ctypes.CDLL:
    """The loaded library.  Raises if libllp.so is missing (build it with paper_2103_09943_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2103_09943_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_str(status: int) -> str:
    return lib().llp_status_str(int(status)).decode()


def validate(shape: Shape, params: Optional[Params]) -> int:
    """Host-only validation (llp_validate); returns the status code."""
    return lib().llp_validate(ctypes.byref(shape), ctypes.byref(params) if params is not None else None)


def _check(status: int, where: str, allow=(OK,)):
    if status not in allow:
        raise LlpError(status, where)
    return status


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError("expected a contiguous float32 CUDA tensor")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def apply_A_noalloc(z, pan, kernel, *, c: int, r: int, lam: float, eps: float, out=None, stream=None):
    """A z with llp_apply_A_noalloc (no context, no device allocation by the library).  `out` may be given so
    that nothing is allocated on this side either."""
    import torch
    N, H, W = z.shape
    shp = Shape(N, H // c, W // c, c, kernel.shape[0])
    prm = Params(int(r), float(lam), float(eps), 0, 0.0, 0)
    if out is None:
        out = torch.empty_like(z)
    _check(lib().llp_apply_A_noalloc(ctypes.byref(shp), ctypes.byref(prm), _ptr(pan), _ptr(kernel), _ptr(z),
                                     _ptr(out), _stream(stream)), "llp_apply_A_noalloc")
    return out


def shape_of(lrms, pan, kernel) -> Shape:
    N, h, w = lrms.shape
    H, W = pan.shape
    if H % h or W % w or H // h != W // w:
        raise ValueError("PAN size must be c times the LRMS size in both directions")
    n = kernel.shape[0]
    if kernel.shape != (n, n):
        raise ValueError("kernel must be square")
    return Shape(N, h, w, H // h, n)


class Context:
    """Owns an llp_ctx (device workspaces).  Not thread-safe."""

    def __init__(self, device: int = 0):
        h = _vp()
        _check(lib().llp_create(ctypes.byref(h), int(device)), "llp_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.llp_destroy(self._h)
        self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def pansharpen(self, lrms, pan, kernel, *, r: int, lam: float, eps: float, max_iters: int, tol: float = 0.0,
                   init=None, out=None, report: bool = True, stream=None, allow_not_converged: bool = True,
                   precond: int = 0):
        """Solve eq. (Z_ini_matting) for every band.  Returns (hrms, list of report dicts or None, status)."""
        import torch
        shp = shape_of(lrms, pan, kernel)
        H, W = pan.shape
        if out is None:
            out = torch.empty((shp.N, H, W), dtype=torch.float32, device=lrms.device)
        mode = 2 if isinstance(init, str) and init == "cnn" else (1 if init is not None else 0)
        if mode == 2:
            init = None
        prm = Params(int(r), float(lam), float(eps), int(max_iters), float(tol), mode, int(precond))
        reps = (Report * shp.N)() if report else None
        st = lib().llp_pansharpen(self._h, ctypes.byref(shp), ctypes.byref(prm), _ptr(lrms), _ptr(pan), _ptr(kernel),
                                  _ptr(init), _ptr(out), reps, _stream(stream))
        allow = (OK, NOT_CONVERGED) if allow_not_converged else (OK,)
        _check(st, "llp_pansharpen", allow)
        return out, ([rp.as_dict() for rp in reps] if report else None), st

    def pansharpen_batch(self, scenes, *, r: int, lam: float, eps: float, max_iters: int, tol: float = 0.0,
                         inits=None, outs=None, report: bool = True, flags: int = 0, stream=None,
                         allow_not_converged: bool = True, precond: int = 0):
        """Solve every band of several scenes together (llp_pansharpen_batch).  `scenes` is a sequence of
        (lrms, pan, kernel) device tensors.  Returns (list of hrms, list of per-scene report lists or None,
        status)."""
        import torch
        S = len(scenes)
        shapes = (Shape * max(S, 1))()
        for i, (X, Y, u) in enumerate(scenes):
            shapes[i] = shape_of(X, Y, u)
        if outs is None:
            outs = [torch.empty((X.shape[0], Y.shape[0], Y.shape[1]), dtype=torch.float32, device=X.device)
                    for X, Y, u in scenes]
        arr = lambda ts: (_vp * max(S, 1))(*[_ptr(t) for t in ts])  # noqa: E731
        mode = 2 if isinstance(inits, str) and inits == "cnn" else (1 if inits is not None else 0)
        if mode == 2:
            inits = None
        prm = Params(int(r), float(lam), float(eps), int(max_iters), float(tol), mode, int(precond))
        nb = sum(shapes[i].N for i in range(S))
        reps = (Report * max(nb, 1))() if report else None
        st = lib().llp_pansharpen_batch(self._h, S, shapes, ctypes.byref(prm), arr([s[0] for s in scenes]),
                                        arr([s[1] for s in scenes]), arr([s[2] for s in scenes]),
                                        arr(inits) if inits is not None else None, arr(outs), reps, int(flags),
                                        _stream(stream))
        allow = (OK, NOT_CONVERGED) if allow_not_converged else (OK,)
        _check(st, "llp_pansharpen_batch", allow)
        out_reps = None
        if report:
            out_reps, k = [], 0
            for i in range(S):
                out_reps.append([reps[k + c].as_dict() for c in range(shapes[i].N)])
                k += shapes[i].N
        return outs, out_reps, st

    def autotune(self, lrms, pan, kernel, *, r: int, lam: float, eps: float, iters: int = 8, scratch=None,
                 stream=None) -> dict:
        """Time every launch configuration on this scene (llp_autotune) and keep the fastest for its class."""
        shp = shape_of(lrms, pan, kernel)
        prm = Params(int(r), float(lam), float(eps), int(iters), 0.0, 0)
        res = TuneResult()
        _check(lib().llp_autotune(self._h, ctypes.byref(shp), ctypes.byref(prm), _ptr(lrms), _ptr(pan),
                                  _ptr(kernel), _ptr(scratch), int(iters), ctypes.byref(res), _stream(stream)),
               "llp_autotune")
        return {k: getattr(res, k) for k, _ in res._fields_}

    def autotune_batch(self, lrms, pan, kernel, *, r: int, lam: float, eps: float, iters: int = 8, copies: int = 0,
                       stream=None) -> dict:
        """Time every specialised launch configuration on a batch of copies of this scene
        (llp_autotune_batch) and keep the fastest as its class's batched entry."""
        shp = shape_of(lrms, pan, kernel)
        prm = Params(int(r), float(lam), float(eps), int(iters), 0.0, 0)
        res = TuneResult()
        _check(lib().llp_autotune_batch(self._h, ctypes.byref(shp), ctypes.byref(prm), _ptr(lrms), _ptr(pan),
                                        _ptr(kernel), int(copies), int(iters), ctypes.byref(res),
                                        _stream(stream)), "llp_autotune_batch")
        return {k: getattr(res, k) for k, _ in res._fields_}

    # ---- warm-start network
    def cnn_set_weights(self, params):
        """Load the network's parameters (CNN_PARAMS float32 values, per layer W then b)."""
        import numpy as np
        a = np.ascontiguousarray(params, dtype=np.float32)
        if a.size != CNN_PARAMS:
            raise ValueError(f"expected {CNN_PARAMS} parameters, got {a.size}")
        _check(lib().llp_cnn_set_weights(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size),
               "llp_cnn_set_weights")

    def cnn_get_weights(self):
        import numpy as np
        a = np.empty(CNN_PARAMS, dtype=np.float32)
        _check(lib().llp_cnn_get_weights(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size),
               "llp_cnn_get_weights")
        return a

    def cnn_warm_start(self, lrms, pan, c: int, *, z0=True, net_out=False, stream=None):
        """The network's estimate z0 and/or its raw output, each [N][H][W] (None where not asked for)."""
        import torch
        N, h, w = lrms.shape
        shp = Shape(N, h, w, c, 1)
        H, W = pan.shape
        z = torch.empty((N, H, W), dtype=torch.float32, device=lrms.device) if z0 else None
        o = torch.empty((N, H, W), dtype=torch.float32, device=lrms.device) if net_out else None
        _check(lib().llp_cnn_warm_start(self._h, ctypes.byref(shp), _ptr(lrms), _ptr(pan), _ptr(z), _ptr(o),
                                        _stream(stream)), "llp_cnn_warm_start")
        return z, o

    def cnn_loss_grad(self, lrms, pan, target, c: int, stream=None):
        """(loss, gradient as a CNN_PARAMS float32 array) of one scene against the target HRMS."""
        import numpy as np
        N, h, w = lrms.shape
        shp = Shape(N, h, w, c, 1)
        loss = ctypes.c_double()
        g = np.empty(CNN_PARAMS, dtype=np.float32)
        _check(lib().llp_cnn_loss_grad(self._h, ctypes.byref(shp), _ptr(lrms), _ptr(pan), _ptr(target),
                                       ctypes.byref(loss), g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                       _stream(stream)), "llp_cnn_loss_grad")
        return loss.value, g

    def cnn_train_step(self, lrms, pan, target, c: int, lr: float, want_loss: bool = True, stream=None):
        N, h, w = lrms.shape
        shp = Shape(N, h, w, c, 1)
        loss = ctypes.c_double()
        _check(lib().llp_cnn_train_step(self._h, ctypes.byref(shp), _ptr(lrms), _ptr(pan), _ptr(target), float(lr),
                                        ctypes.byref(loss) if want_loss else None, _stream(stream)),
               "llp_cnn_train_step")
        return loss.value if want_loss else None

    def tune_save(self, path: str):
        _check(lib().llp_tune_save(self._h, os.fsencode(path)), "llp_tune_save")

    def tune_load(self, path: str):
        _check(lib().llp_tune_load(self._h, os.fsencode(path)), "llp_tune_load")

    def tune_clear(self):
        _check(lib().llp_tune_clear(self._h), "llp_tune_clear")

    def tune_count(self) -> int:
        return lib().llp_tune_count(self._h)

    def pan_stats(self, pan, *, N: int, c: int, n: int, r: int, eps: float, stream=None):
        import torch
        H, W = pan.shape
        shp = Shape(N, H // c, W // c, c, n)
        prm = Params(int(r), 0.0, float(eps), 0, 0.0, 0)
        G, mu, d = (torch.empty((H, W), dtype=torch.float32, device=pan.device) for _ in range(3))
        _check(lib().llp_pan_stats(self._h, ctypes.byref(shp), ctypes.byref(prm), _ptr(pan), _ptr(G), _ptr(mu),
                                   _ptr(d), _stream(stream)), "llp_pan_stats")
        return G, mu, d

    def rhs(self, lrms, kernel, c: int, stream=None):
        import torch
        N, h, w = lrms.shape
        shp = Shape(N, h, w, c, kernel.shape[0])
        b = torch.empty((N, h * c, w * c), dtype=torch.float32, device=lrms.device)
        _check(lib().llp_rhs(self._h, ctypes.byref(shp), _ptr(lrms), _ptr(kernel), _ptr(b), _stream(stream)),
               "llp_rhs")
        return b

    def apply_A(self, z, pan, kernel, *, c: int, r: int, lam: float, eps: float, stream=None):
        import torch
        N, H, W = z.shape
        shp = Shape(N, H // c, W // c, c, kernel.shape[0])
        prm = Params(int(r), float(lam), float(eps), 0, 0.0, 0)
        out = torch.empty_like(z)
        _check(lib().llp_apply_A(self._h, ctypes.byref(shp), ctypes.byref(prm), _ptr(pan), _ptr(kernel), _ptr(z),
                                 _ptr(out), _stream(stream)), "llp_apply_A")
        return out

    def polish(self, z0, lrms, pan, kernel, *, r: int, lam: float, eps: float, stream=None):
        """A, C step and FFT Z step of Algorithm Fast Pansharpening on z0 (llp_polish); returns the new HRMS."""
        import torch
        N, H, W = z0.shape
        c = H // lrms.shape[1]
        shp = Shape(N, H // c, W // c, c, kernel.shape[0])
        prm = Params(int(r), float(lam), float(eps), 0, 0.0, 0)
        out = torch.empty_like(z0)
        _check(lib().llp_polish(self._h, ctypes.byref(shp), ctypes.byref(prm), _ptr(lrms), _ptr(pan), _ptr(kernel),
                                _ptr(z0), _ptr(out), _stream(stream)), "llp_polish")
        return out

    def prior_pansharpen(self, prior: str, lrms, pan, kernel, *, r: int, lam: float, eps: float, max_iters: int,
                         tol: float = 0.0, init=None, out=None, report: bool = True, stream=None,
                         allow_not_converged: bool = True):
        """Solve every band under one of the compared priors (llp_prior_pansharpen).  Returns (hrms, reports,
        status)."""
        import torch
        shp = shape_of(lrms, pan, kernel)
        H, W = pan.shape
        if out is None:
            out = torch.empty((shp.N, H, W), dtype=torch.float32, device=lrms.device)
        prm = Params(int(r), float(lam), float(eps), int(max_iters), float(tol), 1 if init is not None else 0, 0)
        reps = (Report * shp.N)() if report else None
        st = lib().llp_prior_pansharpen(self._h, ctypes.byref(shp), ctypes.byref(prm), PRIORS[prior], _ptr(lrms),
                                        _ptr(pan), _ptr(kernel), _ptr(init), _ptr(out), reps, _stream(stream))
        allow = (OK, NOT_CONVERGED) if allow_not_converged else (OK,)
        _check(st, "llp_prior_pansharpen", allow)
        return out, ([rp.as_dict() for rp in reps] if report else None), st

    def apply_prior(self, prior: str, z, pan, kernel, *, c: int, r: int, lam: float, eps: float,
                    data_term: bool = False, stream=None):
        """lambda sum_d F_d^T M_d F_d z (+ B^T D^T D B z) under one of the compared priors (llp_apply_prior)."""
        import torch
        N, H, W = z.shape
        shp = Shape(N, H // c, W // c, c, kernel.shape[0])
        prm = Params(int(r), float(lam), float(eps), 0, 0.0, 0)
        out = torch.empty_like(z)
        _check(lib().llp_apply_prior(self._h, ctypes.byref(shp), ctypes.byref(prm), PRIORS[prior], _ptr(pan),
                                     _ptr(kernel), _ptr(z), _ptr(out), int(bool(data_term)), _stream(stream)),
               "llp_apply_prior")
        return out

    def estimate_kernel(self, lrms, pan, c: int, *, n: int, l: int = 1, lam_w: float = 10.0, alpha1: float = 1.0,
                        alpha2: float = 0.006, mu1: float = 100.0, mu2: float = 100.0, mu3: float = 100.0,
                        rho: float = 0.5, t_max: int = 10000, th: float = 1e-5, stream=None):
        """Algorithm Blur Kernel Estimation (llp_estimate_kernel).  Returns (kernel [n][n] float32, omega [Np]
        float64, report dict)."""
        import torch
        Np, h, w = lrms.shape
        prm = KernelEstParams(int(n), int(l), float(lam_w), float(alpha1), float(alpha2), float(mu1), float(mu2),
                              float(mu3), float(rho), int(t_max), float(th))
        out = torch.empty((n, n), dtype=torch.float32, device=lrms.device)
        om = torch.empty((Np,), dtype=torch.float64, device=lrms.device)
        rep = KernelEstReport()
        _check(lib().llp_estimate_kernel(self._h, ctypes.byref(prm), int(Np), int(h), int(w), int(c), _ptr(lrms),
                                         _ptr(pan), _ptr(out), om.data_ptr(), ctypes.byref(rep), _stream(stream)),
               "llp_estimate_kernel")
        return out, om, {"iters": rep.iters, "change": rep.change}

    def apply_data(self, z, kernel, *, c: int, r: int, stream=None):
        """B^T D^T D B z (llp_apply_data)."""
        import torch
        N, H, W = z.shape
        shp = Shape(N, H // c, W // c, c, kernel.shape[0])
        prm = Params(int(r), 0.0, 0.0, 0, 0.0, 0)
        out = torch.empty_like(z)
        _check(lib().llp_apply_data(self._h, ctypes.byref(shp), ctypes.byref(prm), _ptr(kernel), _ptr(z), _ptr(out),
                                    _stream(stream)), "llp_apply_data")
        return out

    def apply_llp(self, z, pan, kernel, *, c: int, r: int, lam: float, eps: float, stream=None):
        """lambda L^T M_LY L z (llp_apply_llp)."""
        import torch
        N, H, W = z.shape
        shp = Shape(N, H // c, W // c, c, kernel.shape[0])
        prm = Params(int(r), float(lam), float(eps), 0, 0.0, 0)
        out = torch.empty_like(z)
        _check(lib().llp_apply_llp(self._h, ctypes.byref(shp), ctypes.byref(prm), _ptr(pan), _ptr(kernel), _ptr(z),
                                   _ptr(out), _stream(stream)), "llp_apply_llp")
        return out

    def precond_apply(self, rr, pan, kernel, *, c: int, r: int, lam: float, eps: float, stream=None):
        """P^{-1} r (llp_precond_apply)."""
        import torch
        N, H, W = rr.shape
        shp = Shape(N, H // c, W // c, c, kernel.shape[0])
        prm = Params(int(r), float(lam), float(eps), 0, 0.0, 0, 1)
        out = torch.empty_like(rr)
        _check(lib().llp_precond_apply(self._h, ctypes.byref(shp), ctypes.byref(prm), _ptr(pan), _ptr(kernel),
                                       _ptr(rr), _ptr(out), _stream(stream)), "llp_precond_apply")
        return out

    def apply_data_fourier(self, z, kernel, *, c: int, stream=None):
        """B^T D^T D B z in the Fourier domain (llp_apply_data_fourier)."""
        import torch
        N, H, W = z.shape
        shp = Shape(N, H // c, W // c, c, kernel.shape[0])
        prm = Params(1, 0.0, 0.0, 0, 0.0, 0)
        out = torch.empty_like(z)
        _check(lib().llp_apply_data_fourier(self._h, ctypes.byref(shp), ctypes.byref(prm), _ptr(kernel), _ptr(z),
                                            _ptr(out), _stream(stream)), "llp_apply_data_fourier")
        return out

    def objective(self, z, lrms, pan, kernel, *, r: int, lam: float, eps: float, stream=None):
        shp = shape_of(lrms, pan, kernel)
        prm = Params(int(r), float(lam), float(eps), 0, 0.0, 0)
        obj = (ctypes.c_double * shp.N)()
        _check(lib().llp_objective(self._h, ctypes.byref(shp), ctypes.byref(prm), _ptr(lrms), _ptr(pan),
                                   _ptr(kernel), _ptr(z), obj, _stream(stream)), "llp_objective")
        return list(obj)

    def set_profiling(self, enable: bool):
        _check(lib().llp_set_profiling(self._h, 1 if enable else 0), "llp_set_profiling")

    def kernel_times(self, reset: bool = True) -> dict:
        t = KernelTimes()
        _check(lib().llp_get_kernel_times(self._h, ctypes.byref(t), 1 if reset else 0), "llp_get_kernel_times")
        return {k: getattr(t, k) for k, _ in t._fields_}
