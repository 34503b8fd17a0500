"""Python binding of liblagp (include/lagp.h): local approximate GP
prediction with greedy ALC local designs on MI355X.

The functions named ``lagp_*`` mirror the C entry points one to one and only
marshal arguments: torch tensors on the GPU pass their data pointers and the
current HIP stream.  Every step of the computation runs in the library's HIP
kernels.  Importing this module fails if the library has not been built
(``python paper_1303_0383_amd/build.py`` or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblagp.so")

LAGP_OK, LAGP_E_INVAL, LAGP_E_NOMEM, LAGP_E_NODEVICE, LAGP_E_HIP, LAGP_E_BUDGET, LAGP_E_NOTPD = 0, -1, -2, -3, -4, -5, -6
LAGP_LOC_OK, LAGP_LOC_NOTPD, LAGP_LOC_NOTCAND, LAGP_LOC_NOCAND = 0, 1, 2, 3
LAGP_PREC_FP64, LAGP_PREC_SCORE_FP32, LAGP_PREC_SCORE_BF16 = 0, 1, 2
LAGP_PTR_HOST, LAGP_STRICT = 1, 2
LAGP_BATCH_SEL, LAGP_BATCH_STATUS = 1, 2
PHASES = ("knn", "design", "mle", "predict")   # LAGP_PHASE_* order

# torch first: its bundled HIP runtime is then the one the library binds to.
# Loading the library first would map a second HIP runtime into the process.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                      "(python paper_1303_0383_amd/build.py)")

_lib = C.CDLL(LIB_PATH)


class lagp_params(C.Structure):
    _fields_ = [("n0", C.c_int32), ("n", C.c_int32), ("ncand", C.c_int32), ("d", C.c_double),
                ("g", C.c_double), ("precision", C.c_int32), ("flags", C.c_uint32)]


class lagp_options(C.Structure):
    _fields_ = [("d_per", C.c_void_p), ("start", C.c_void_p), ("start_stride", C.c_int64),
                ("start_n", C.c_void_p), ("vratio", C.c_double)]


class lagp_mle_params(C.Structure):
    _fields_ = [("tmin", C.c_double), ("tmax", C.c_double), ("maxit", C.c_int32), ("tol", C.c_double)]


_P = C.c_void_p
_lib.lagp_design_create.argtypes = [_P, _P, C.c_int64, C.c_int32, C.c_uint32, _P, C.POINTER(_P)]
_lib.lagp_design_destroy.argtypes = [_P]
_lib.lagp_design_destroy.restype = None
_lib.lagp_knn.argtypes = [_P, _P, C.c_int64, C.c_int32, _P, C.c_int64, _P]
_lib.lagp_predict.argtypes = [_P, _P, C.c_int64, C.POINTER(lagp_params), _P, _P, _P, _P, _P, _P, _P,
                              C.c_int64, _P, _P]
_lib.lagp_predict_ex.argtypes = [_P, _P, C.c_int64, C.POINTER(lagp_params), C.POINTER(lagp_options), _P, _P, _P, _P,
                                _P, _P, _P, C.c_int64, _P, _P]
_lib.lagp_predict_mspe.argtypes = [_P, _P, C.c_int64, C.POINTER(lagp_params), _P, _P, _P, _P, _P, _P, _P, C.c_int64,
                                  _P, _P]
_lib.lagp_predict_theta.argtypes = [_P, _P, C.c_int64, C.POINTER(lagp_params), _P, _P, _P, _P, _P, _P, _P, _P,
                                   C.c_int64, _P, _P]
_lib.lagp_predict_alc2.argtypes = [_P, _P, C.c_int64, C.POINTER(lagp_params), C.POINTER(lagp_mle_params), _P, _P, _P,
                                  _P, _P, _P, _P, _P, C.c_int64, _P, _P, _P, _P]
_lib.lagp_mle.argtypes = [_P, C.c_int64, _P, C.c_int64, _P, C.c_int32, _P, C.c_double, C.c_double,
                         C.POINTER(lagp_mle_params), _P, _P, _P, _P]
_lib.lagp_predict_designs.argtypes = [_P, _P, C.c_int64, _P, C.c_int64, _P, C.c_int32, C.c_double, _P, C.c_double,
                                      _P, _P, _P, _P, _P, _P]
_lib.lagp_predict_noalloc.argtypes = [_P, _P, C.c_int64, C.POINTER(lagp_params), _P, _P, _P, _P, _P, C.c_int64,
                                      _P, _P]
_lib.lagp_noalloc_scratch_bytes.restype = C.c_size_t
_lib.lagp_workspace_bytes.argtypes = [_P, C.c_int64, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]
_lib.lagp_timing_enable.argtypes = [_P, C.c_int]
_lib.lagp_phase_times.argtypes = [_P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
_lib.lagp_batch_create.argtypes = [_P, C.c_int64, C.POINTER(lagp_params), _P, _P, C.c_uint32, C.POINTER(_P)]
_lib.lagp_batch_enqueue.argtypes = [_P, _P, _P, _P, _P, _P, _P, C.c_int64, _P, _P]
_lib.lagp_batch_launch_graph.argtypes = [_P, _P, _P, _P, _P, _P, _P, C.c_int64, _P, _P]
_lib.lagp_batch_info.argtypes = [_P, C.POINTER(C.c_int32), C.POINTER(C.c_size_t)]
_lib.lagp_batch_destroy.argtypes = [_P]
_lib.lagp_batch_destroy.restype = None
_lib.lagp_design_set_variant.argtypes = [_P, C.c_int32, C.c_int32]
_lib.lagp_design_set_variant_ex.argtypes = [_P, C.c_int32, C.c_int32, C.c_int32]
_lib.lagp_server_create.argtypes = [_P, C.c_size_t, C.POINTER(_P)]
_lib.lagp_server_create_ex.argtypes = [_P, C.c_size_t, C.c_int32, C.c_int32, C.POINTER(_P)]
_lib.lagp_server_submit.argtypes = [_P, _P, C.c_int32, C.POINTER(lagp_params), _P, _P, C.POINTER(C.c_uint64)]
_lib.lagp_server_poll.argtypes = [_P, C.c_uint64, C.c_int32, _P, _P, _P, _P, _P, C.c_int64, _P, _P]
_lib.lagp_server_stats.argtypes = [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_double)]
_lib.lagp_server_destroy.argtypes = [_P]
_lib.lagp_server_destroy.restype = None
_lib.lagp_monotonic_seconds.restype = C.c_double
_lib.lagp_last_error.restype = C.c_char_p
for _f in ("lagp_design_create", "lagp_knn", "lagp_predict", "lagp_workspace_bytes", "lagp_device_count",
           "lagp_version", "lagp_timing_enable", "lagp_phase_times", "lagp_predict_designs", "lagp_batch_create",
           "lagp_batch_enqueue", "lagp_batch_launch_graph", "lagp_batch_info", "lagp_design_set_variant",
           "lagp_design_set_variant_ex",
           "lagp_server_create", "lagp_server_create_ex", "lagp_server_submit", "lagp_server_poll",
           "lagp_server_stats", "lagp_predict_theta", "lagp_predict_alc2", "lagp_mle", "lagp_predict_ex", "lagp_predict_mspe", "lagp_predict_noalloc"):
    getattr(_lib, _f).restype = C.c_int


class LagpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lagp error {code}: {msg}")
        self.code = code


def _check(rc: int) -> int:
    if rc != LAGP_OK:
        raise LagpError(rc, lagp_last_error())
    return rc


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is not None:
        return int(stream)
    import torch
    return torch.cuda.current_stream().cuda_stream


# ----------------------------------------------------------- C entry points
def lagp_version() -> int:
    return _lib.lagp_version()


def lagp_device_count() -> int:
    return _lib.lagp_device_count()


def lagp_last_error() -> str:
    return _lib.lagp_last_error().decode()


def lagp_design_create(X, y, stream=None):
    """Copy the design (X: N x p float64, y: N) to the device.

    X, y may be CUDA tensors or host numpy arrays / CPU tensors."""
    import torch
    host = isinstance(X, np.ndarray) or (hasattr(X, "is_cuda") and not X.is_cuda)
    if host:
        X = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
        y = np.ascontiguousarray(np.asarray(y, dtype=np.float64))
        flags = LAGP_PTR_HOST
        s = None if not torch.cuda.is_available() else _stream(stream)
    else:
        X = X.contiguous()
        y = y.contiguous()
        flags = 0
        s = _stream(stream)
    N, p = X.shape
    out = _P()
    _check(_lib.lagp_design_create(_ptr(X), _ptr(y), N, p, flags, s, C.byref(out)))
    return out


def lagp_design_destroy(design) -> None:
    _lib.lagp_design_destroy(design)


def lagp_knn(design, XX, T: int, M: int, idx, idx_stride: int, stream=None) -> None:
    _check(_lib.lagp_knn(design, _ptr(XX), T, M, _ptr(idx), idx_stride, _stream(stream)))


def lagp_predict(design, XX, T: int, params: lagp_params, n_per, ncand_per, mean, s2, df, var, sel,
                 sel_stride: int, status, stream=None) -> None:
    _check(_lib.lagp_predict(design, _ptr(XX), T, C.byref(params), _ptr(n_per), _ptr(ncand_per), _ptr(mean),
                             _ptr(s2), _ptr(df), _ptr(var), _ptr(sel), sel_stride, _ptr(status),
                             _stream(stream)))


def lagp_predict_noalloc(design, XX, T: int, params: lagp_params, mean, s2, df, var, sel, sel_stride: int, status,
                         stream=None) -> None:
    _check(_lib.lagp_predict_noalloc(design, _ptr(XX), T, C.byref(params), _ptr(mean), _ptr(s2), _ptr(df), _ptr(var),
                                     _ptr(sel), sel_stride, _ptr(status), _stream(stream)))


def lagp_noalloc_scratch_bytes() -> int:
    return int(_lib.lagp_noalloc_scratch_bytes())


def lagp_predict_ex(design, XX, T: int, params: lagp_params, opts, n_per, ncand_per, mean, s2, df, var, sel,
                    sel_stride: int, status, stream=None) -> None:
    _check(_lib.lagp_predict_ex(design, _ptr(XX), T, C.byref(params), None if opts is None else C.byref(opts),
                                _ptr(n_per), _ptr(ncand_per), _ptr(mean), _ptr(s2), _ptr(df), _ptr(var), _ptr(sel),
                                sel_stride, _ptr(status), _stream(stream)))


def lagp_predict_mspe(design, XX, T: int, params: lagp_params, n_per, ncand_per, mean, s2, df, var, sel,
                      sel_stride: int, status, stream=None) -> None:
    _check(_lib.lagp_predict_mspe(design, _ptr(XX), T, C.byref(params), _ptr(n_per), _ptr(ncand_per), _ptr(mean),
                                  _ptr(s2), _ptr(df), _ptr(var), _ptr(sel), sel_stride, _ptr(status),
                                  _stream(stream)))


def lagp_predict_theta(design, XX, T: int, params: lagp_params, d_per, n_per, ncand_per, mean, s2, df, var, sel,
                       sel_stride: int, status, stream=None) -> None:
    _check(_lib.lagp_predict_theta(design, _ptr(XX), T, C.byref(params), _ptr(d_per), _ptr(n_per), _ptr(ncand_per),
                                   _ptr(mean), _ptr(s2), _ptr(df), _ptr(var), _ptr(sel), sel_stride, _ptr(status),
                                   _stream(stream)))


def lagp_predict_alc2(design, XX, T: int, params: lagp_params, mle: lagp_mle_params, d_per, n_per, ncand_per, mean,
                      s2, df, var, sel, sel_stride: int, status, d1, d2, stream=None) -> None:
    _check(_lib.lagp_predict_alc2(design, _ptr(XX), T, C.byref(params), C.byref(mle), _ptr(d_per), _ptr(n_per),
                                  _ptr(ncand_per), _ptr(mean), _ptr(s2), _ptr(df), _ptr(var), _ptr(sel), sel_stride,
                                  _ptr(status), _ptr(d1), _ptr(d2), _stream(stream)))


def lagp_mle(design, T: int, sel, sel_stride: int, n_per, n: int, d0_per, d0: float, g: float,
             mle: lagp_mle_params, d_hat, iters, status, stream=None) -> None:
    _check(_lib.lagp_mle(design, T, _ptr(sel), sel_stride, _ptr(n_per), n, _ptr(d0_per), d0, g, C.byref(mle),
                         _ptr(d_hat), _ptr(iters), _ptr(status), _stream(stream)))


def lagp_predict_designs(design, XX, T: int, sel, sel_stride: int, n_per, n: int, d: float, d_per, g: float, mean,
                         s2, df, var, status, stream=None) -> None:
    _check(_lib.lagp_predict_designs(design, _ptr(XX), T, _ptr(sel), sel_stride, _ptr(n_per), n, d, _ptr(d_per), g,
                                     _ptr(mean), _ptr(s2), _ptr(df), _ptr(var), _ptr(status), _stream(stream)))


def lagp_workspace_bytes(design, T: int, nmax: int, ncand_max: int) -> int:
    out = C.c_size_t()
    _check(_lib.lagp_workspace_bytes(design, T, nmax, ncand_max, C.byref(out)))
    return int(out.value)


def lagp_batch_create(design, T: int, params: lagp_params, n_per=None, ncand_per=None, flags: int = 0):
    """n_per / ncand_per: host int32 arrays of length T (or None)."""
    hn = None if n_per is None else np.ascontiguousarray(np.asarray(n_per, dtype=np.int32))
    hm = None if ncand_per is None else np.ascontiguousarray(np.asarray(ncand_per, dtype=np.int32))
    out = _P()
    _check(_lib.lagp_batch_create(design, T, C.byref(params), _ptr(hn), _ptr(hm), flags, C.byref(out)))
    return out


def lagp_batch_enqueue(batch, XX, mean, s2, df, var, sel, sel_stride: int, status, stream=None) -> None:
    _check(_lib.lagp_batch_enqueue(batch, _ptr(XX), _ptr(mean), _ptr(s2), _ptr(df), _ptr(var), _ptr(sel),
                                   sel_stride, _ptr(status), _stream(stream)))


def lagp_batch_launch_graph(batch, XX, mean, s2, df, var, sel, sel_stride: int, status, stream=None) -> None:
    _check(_lib.lagp_batch_launch_graph(batch, _ptr(XX), _ptr(mean), _ptr(s2), _ptr(df), _ptr(var), _ptr(sel),
                                        sel_stride, _ptr(status), _stream(stream)))


def lagp_batch_info(batch):
    """(buckets, workspace_bytes)."""
    b, w = C.c_int32(), C.c_size_t()
    _check(_lib.lagp_batch_info(batch, C.byref(b), C.byref(w)))
    return b.value, int(w.value)


def lagp_batch_destroy(batch) -> None:
    _lib.lagp_batch_destroy(batch)


def lagp_design_set_variant(design, threads: int, coords: int) -> None:
    _check(_lib.lagp_design_set_variant(design, threads, coords))


def lagp_design_set_variant_ex(design, threads: int, coords: int, lds_rows_pct: int) -> None:
    _check(_lib.lagp_design_set_variant_ex(design, threads, coords, lds_rows_pct))


def lagp_server_create(design, hbm_budget_bytes: int):
    out = _P()
    _check(_lib.lagp_server_create(design, hbm_budget_bytes, C.byref(out)))
    return out


def lagp_server_create_ex(design, hbm_budget_bytes: int, slots: int = 0, piece_locations: int = 0):
    out = _P()
    _check(_lib.lagp_server_create_ex(design, hbm_budget_bytes, slots, piece_locations, C.byref(out)))
    return out


def lagp_server_submit(server, XX, T: int, params: lagp_params, n_per=None, ncand_per=None) -> int:
    """XX, n_per, ncand_per: host arrays."""
    XX = np.ascontiguousarray(np.asarray(XX, dtype=np.float64))
    hn = None if n_per is None else np.ascontiguousarray(np.asarray(n_per, dtype=np.int32))
    hm = None if ncand_per is None else np.ascontiguousarray(np.asarray(ncand_per, dtype=np.int32))
    ticket = C.c_uint64()
    _check(_lib.lagp_server_submit(server, _ptr(XX), T, C.byref(params), _ptr(hn), _ptr(hm), C.byref(ticket)))
    return int(ticket.value)


def lagp_server_poll(server, ticket: int, wait_ms: int, mean, s2, df, var, sel, sel_stride: int, status, times):
    """Host numpy outputs (each may be None); returns 1 when done, 0 while pending."""
    rc = _lib.lagp_server_poll(server, ticket, wait_ms, _ptr(mean), _ptr(s2), _ptr(df), _ptr(var), _ptr(sel),
                               sel_stride, _ptr(status), _ptr(times))
    if rc < 0:
        _check(rc)
    return rc


def lagp_server_stats(server):
    """(batches, locations, requests, busy_seconds)."""
    b, l, r, s = C.c_int64(), C.c_int64(), C.c_int64(), C.c_double()
    _check(_lib.lagp_server_stats(server, C.byref(b), C.byref(l), C.byref(r), C.byref(s)))
    return b.value, l.value, r.value, s.value


def lagp_server_destroy(server) -> None:
    _lib.lagp_server_destroy(server)


def lagp_monotonic_seconds() -> float:
    return _lib.lagp_monotonic_seconds()


def lagp_timing_enable(design, enable: bool) -> None:
    _check(_lib.lagp_timing_enable(design, 1 if enable else 0))


def lagp_phase_times(design):
    """(ms, design_launches) summed since the last call: ms is a dict of the
    phases' device milliseconds (knn, design, mle, predict)."""
    ms = (C.c_double * 4)()
    n = C.c_int64()
    _check(_lib.lagp_phase_times(design, ms, C.byref(n)))
    return dict(zip(PHASES, ms)), n.value


# ------------------------------------------------------- tensor conveniences
@dataclass
class Prediction:
    mean: "torch.Tensor"
    s2: "torch.Tensor"
    df: "torch.Tensor"
    var: "torch.Tensor"
    sel: "torch.Tensor"
    status: "torch.Tensor"
    theta1: Optional["torch.Tensor"] = None   # two-stage scheme: local MLE from the first designs
    theta2: Optional["torch.Tensor"] = None   # ... and from the second designs


# Newton controls of the local lengthscale search (the paper leaves them open).
MLE_MAXIT = 100
MLE_TOL = 1e-10


def _outputs(T: int, nmax: int, dev) -> Prediction:
    import torch
    return Prediction(mean=torch.empty(T, dtype=torch.float64, device=dev),
                      s2=torch.empty(T, dtype=torch.float64, device=dev),
                      df=torch.empty(T, dtype=torch.int32, device=dev),
                      var=torch.empty(T, dtype=torch.float64, device=dev),
                      sel=torch.empty((T, max(nmax, 1)), dtype=torch.int32, device=dev),
                      status=torch.empty(T, dtype=torch.int8, device=dev))


class Design:
    """Owns a lagp_design; frees it on close() or garbage collection."""

    def __init__(self, X, y, stream=None):
        self.N, self.p = int(X.shape[0]), int(X.shape[1])
        self._h = lagp_design_create(X, y, stream)

    def close(self):
        if getattr(self, "_h", None):
            lagp_design_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def knn(self, XX, M: int, stream=None):
        import torch
        XX = XX.contiguous()
        idx = torch.empty((XX.shape[0], M), dtype=torch.int32, device=XX.device)
        lagp_knn(self._h, XX, XX.shape[0], M, idx, M, stream)
        return idx

    def predict_designs(self, XX, sel, d: float, g: float, n_per=None, d_per=None, stream=None) -> Prediction:
        """Prediction from given local designs (sel: T x n int32 design indices);
        d_per (device float64[T]) gives each location its own lengthscale."""
        XX = XX.contiguous()
        sel = sel.contiguous()
        T, n = sel.shape
        out = _outputs(T, 0, XX.device)
        out.sel = sel
        lagp_predict_designs(self._h, XX, T, sel, n, n_per, n, d, d_per, g, out.mean, out.s2, out.df, out.var,
                             out.status, stream)
        return out

    def predict_mspe(self, XX, n0: int, n: int, ncand: int, d: float, g: float, n_per=None, ncand_per=None,
                     strict: bool = False, out: Optional[Prediction] = None, stream=None) -> Prediction:
        """Greedy MSPE designs (eq mspe) and prediction."""
        XX = XX.contiguous()
        T = XX.shape[0]
        nmax = int(n_per.max().item()) if (n_per is not None and T) else n
        if out is None:
            out = _outputs(T, nmax, XX.device)
        prm = lagp_params(n0, n, ncand, d, g, LAGP_PREC_FP64, LAGP_STRICT if strict else 0)
        lagp_predict_mspe(self._h, XX, T, prm, n_per, ncand_per, out.mean, out.s2, out.df, out.var, out.sel,
                          out.sel.shape[1], out.status, stream)
        return out

    def mle(self, sel, d0, g: float, tmin: float, tmax: float, n_per=None, maxit: int = MLE_MAXIT,
            tol: float = MLE_TOL, stream=None):
        """Local MLE lengthscale of each design (sel: T x n int32); d0 a float or a
        device float64[T] of starting values.  Returns (theta, iters, status)."""
        import torch
        sel = sel.contiguous()
        T, n = sel.shape
        dev = sel.device
        theta = torch.empty(T, dtype=torch.float64, device=dev)
        iters = torch.empty(T, dtype=torch.int32, device=dev)
        status = torch.empty(T, dtype=torch.int8, device=dev)
        per = d0 if torch.is_tensor(d0) else None
        lagp_mle(self._h, T, sel, n, n_per, n, per, 1.0 if per is not None else float(d0), g,
                 lagp_mle_params(tmin, tmax, maxit, tol), theta, iters, status, stream)
        return theta, iters, status

    def predict_alc2(self, XX, n0: int, n: int, ncand: int, d: float, g: float, tmin: float, tmax: float,
                     maxit: int = MLE_MAXIT, tol: float = MLE_TOL, d_per=None, n_per=None, ncand_per=None,
                     precision: int = LAGP_PREC_FP64, strict: bool = False, out: Optional[Prediction] = None,
                     stream=None) -> Prediction:
        """The two-stage scheme (designs, local MLE, designs again, MLE, prediction)."""
        import torch
        XX = XX.contiguous()
        T = XX.shape[0]
        nmax = int(n_per.max().item()) if (n_per is not None and T) else n
        if out is None:
            out = _outputs(T, nmax, XX.device)
        if out.theta1 is None:
            out.theta1 = torch.empty(T, dtype=torch.float64, device=XX.device)
        if out.theta2 is None:
            out.theta2 = torch.empty(T, dtype=torch.float64, device=XX.device)
        prm = lagp_params(n0, n, ncand, d, g, precision, LAGP_STRICT if strict else 0)
        lagp_predict_alc2(self._h, XX, T, prm, lagp_mle_params(tmin, tmax, maxit, tol), d_per, n_per, ncand_per,
                          out.mean, out.s2, out.df, out.var, out.sel, out.sel.shape[1], out.status, out.theta1,
                          out.theta2, stream)
        return out

    def predict(self, XX, n0: int, n: int, ncand: int, d: float, g: float, n_per=None, ncand_per=None,
                precision: int = LAGP_PREC_FP64, strict: bool = False, out: Optional[Prediction] = None,
                d_per=None, start=None, start_n=None, vratio: float = 0.0, stream=None) -> Prediction:
        """Greedy ALC designs and prediction; d_per (device float64[T]) gives each
        location its own lengthscale; start (device int32 T x k) saved designs to
        augment (their first start_n[t], or n0, entries); vratio > 0 the
        variance-ratio stopping rule (df then holds each design's size)."""
        XX = XX.contiguous()
        T = XX.shape[0]
        nmax = int(n_per.max().item()) if (n_per is not None and T) else n
        if out is None:
            out = _outputs(T, nmax, XX.device)
        prm = lagp_params(n0, n, ncand, d, g, precision, LAGP_STRICT if strict else 0)
        if start is not None or vratio != 0.0:
            st = None if start is None else start.contiguous()
            opts = lagp_options(_ptr(d_per), _ptr(st), 0 if st is None else st.shape[1], _ptr(start_n), vratio)
            lagp_predict_ex(self._h, XX, T, prm, opts, n_per, ncand_per, out.mean, out.s2, out.df, out.var,
                            out.sel, out.sel.shape[1], out.status, stream)
        elif d_per is None:
            lagp_predict(self._h, XX, T, prm, n_per, ncand_per, out.mean, out.s2, out.df, out.var, out.sel,
                         out.sel.shape[1], out.status, stream)
        else:
            lagp_predict_theta(self._h, XX, T, prm, d_per, n_per, ncand_per, out.mean, out.s2, out.df, out.var,
                               out.sel, out.sel.shape[1], out.status, stream)
        return out


class Batch:
    """Owns a lagp_batch: a fixed-shape batch of T locations (per-location
    sizes fixed at creation) that runs as plain launches or one graph launch."""

    def __init__(self, design: Design, T: int, n0: int, n: int, ncand: int, d: float, g: float, n_per=None,
                 ncand_per=None, precision: int = LAGP_PREC_FP64, with_sel: bool = True, with_status: bool = True):
        self.design = design
        self.T = int(T)
        self.nmax = int(np.max(n_per)) if n_per is not None else int(n)
        prm = lagp_params(n0, n, ncand, d, g, precision, 0)
        flags = (LAGP_BATCH_SEL if with_sel else 0) | (LAGP_BATCH_STATUS if with_status else 0)
        self.with_sel, self.with_status = with_sel, with_status
        self._h = lagp_batch_create(design.handle, self.T, prm, n_per, ncand_per, flags)

    def close(self):
        if getattr(self, "_h", None):
            lagp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self):
        return lagp_batch_info(self._h)

    def outputs(self, device) -> Prediction:
        import torch
        T = self.T
        return Prediction(mean=torch.empty(T, dtype=torch.float64, device=device),
                          s2=torch.empty(T, dtype=torch.float64, device=device),
                          df=torch.empty(T, dtype=torch.int32, device=device),
                          var=torch.empty(T, dtype=torch.float64, device=device),
                          sel=torch.empty((T, self.nmax), dtype=torch.int32, device=device) if self.with_sel else None,
                          status=torch.empty(T, dtype=torch.int8, device=device) if self.with_status else None)

    def run(self, XX, out: Optional[Prediction] = None, graph: bool = True, stream=None) -> Prediction:
        XX = XX.contiguous()
        out = out if out is not None else self.outputs(XX.device)
        f = lagp_batch_launch_graph if graph else lagp_batch_enqueue
        f(self._h, XX, out.mean, out.s2, out.df, out.var, out.sel, self.nmax if out.sel is None else out.sel.shape[1],
          out.status, stream)
        return out


@dataclass
class Served:
    """Results of one served request (host arrays)."""
    mean: np.ndarray
    s2: np.ndarray
    df: np.ndarray
    var: np.ndarray
    sel: np.ndarray
    status: np.ndarray
    submitted: float
    done: float


class Server:
    """Owns a lagp_server: continuous batching of host-side requests
    (slots: pieces in flight, 0 for the default; piece: locations per piece)."""

    def __init__(self, design: Design, hbm_budget_bytes: int, slots: int = 0, piece: int = 0):
        self.design = design
        self._h = lagp_server_create_ex(design.handle, int(hbm_budget_bytes), int(slots), int(piece))
        self._n = {}

    def close(self):
        if getattr(self, "_h", None):
            lagp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, XX, n0: int, n, ncand, d: float, g: float, precision: int = LAGP_PREC_FP64) -> int:
        """n, ncand: ints or per-location int arrays."""
        XX = np.asarray(XX, dtype=np.float64)
        T = XX.shape[0]
        n_arr = np.broadcast_to(np.asarray(n, dtype=np.int32), (T,))
        m_arr = np.broadcast_to(np.asarray(ncand, dtype=np.int32), (T,))
        prm = lagp_params(n0, int(n_arr.max()), int(m_arr.max()), d, g, precision, 0)
        ticket = lagp_server_submit(self._h, XX, T, prm, n_arr, m_arr)
        self._n[ticket] = (T, int(n_arr.max()))
        return ticket

    def poll(self, ticket: int, wait_ms: int = 0) -> Optional[Served]:
        T, nmax = self._n[ticket]
        out = Served(mean=np.empty(T), s2=np.empty(T), df=np.empty(T, np.int32), var=np.empty(T),
                     sel=np.empty((T, nmax), np.int32), status=np.empty(T, np.int8), submitted=0.0, done=0.0)
        times = np.zeros(2)
        if not lagp_server_poll(self._h, ticket, wait_ms, out.mean, out.s2, out.df, out.var, out.sel, nmax,
                                out.status, times):
            return None
        del self._n[ticket]
        out.submitted, out.done = float(times[0]), float(times[1])
        return out

    def wait(self, ticket: int) -> Served:
        return self.poll(ticket, wait_ms=-1)

    def stats(self):
        return lagp_server_stats(self._h)
