"""ctypes wrapper for the FP64 CPU oracle (``lagp_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg are the only users.  The product path never
imports this package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lagp_oracle.c")
LIB = os.path.join(HERE, "liblagp_oracle.so")

OK, NOTPD, EINVAL, ENOMEM = 0, 1, -1, -2

_lib = None


def compile_source(src: str, out: str) -> str:
    """Compile one oracle source file with gcc (FP64, no FMA contraction, OpenMP)."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        compile_source(SRC, LIB)
    return LIB


def load(path: str):
    """Load an oracle build from ``path`` with argument types configured."""
    L = C.CDLL(path)
    _configure(L)
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = load(LIB)
    return _lib


def _configure(L):
    P = C.c_void_p
    i32, i64, f64 = C.c_int32, C.c_int64, C.c_double
    L.lagp_oracle_knn.argtypes = [P, i64, i32, P, i64, P, P]
    L.lagp_oracle_predict.argtypes = [P, P, i32, P, P, i32, f64, f64, P]
    L.lagp_oracle_alc.argtypes = [P, i32, P, P, i32, P, i64, f64, f64, P, P, P, P]
    L.lagp_oracle_alc_brute.argtypes = [P, i32, P, P, i32, P, i64, f64, f64, P]
    L.lagp_oracle_local.argtypes = [P, P, i64, i32, P, i32, i32, i64, f64, f64, P, P, P, P]
    L.lagp_oracle_mspe.argtypes = [P, P, i32, P, P, i32, P, i32, f64, f64, P, P, P]
    L.lagp_oracle_mspe_local.argtypes = [P, P, i64, i32, P, i32, i32, i64, f64, f64, P, P, P]
    L.lagp_oracle_local_ex.argtypes = [P, P, i64, i32, P, i32, i32, i64, f64, f64, P, P, f64, P, P, P, P]
    L.lagp_oracle_batch.argtypes = [P, P, i64, i32, P, i64, i32, i32, i64, P, P, f64, f64,
                                    P, i64, P, P, i32]
    L.lagp_oracle_loglik.argtypes = [P, P, i32, P, i32, f64, f64, P]
    L.lagp_oracle_mle.argtypes = [P, P, i32, P, i32, f64, f64, f64, f64, i32, f64, P, P]
    L.lagp_oracle_alc2.argtypes = [P, P, i64, i32, P, i32, i32, i64, f64, f64, f64, f64, i32, f64, P, P, P, P]
    for f in (L.lagp_oracle_knn, L.lagp_oracle_predict, L.lagp_oracle_alc,
              L.lagp_oracle_alc_brute, L.lagp_oracle_local, L.lagp_oracle_batch,
              L.lagp_oracle_max_threads, L.lagp_oracle_loglik, L.lagp_oracle_mle, L.lagp_oracle_alc2,
              L.lagp_oracle_local_ex, L.lagp_oracle_mspe, L.lagp_oracle_mspe_local):
        f.restype = C.c_int


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a):
    return None if a is None else a.ctypes.data


def knn(X, x, M, L=None):
    """Indices and squared distances of the M nearest design points of x."""
    X = _f64(X); x = _f64(x)
    idx = np.empty(M, np.int32); d2 = np.empty(M, np.float64)
    rc = (L or lib()).lagp_oracle_knn(_ptr(X), X.shape[0], X.shape[1], _ptr(x), M, _ptr(idx), _ptr(d2))
    if rc != OK:
        raise ValueError(f"oracle knn failed: {rc}")
    return idx, d2


def predict(X, y, x, D, d, g, L=None):
    """{mean, s2, var, v_n(x), psi} from the design indices D (fresh Cholesky)."""
    X = _f64(X); y = _f64(y); x = _f64(x); D = _i32(D)
    out = np.empty(5, np.float64)
    rc = (L or lib()).lagp_oracle_predict(_ptr(X), _ptr(y), X.shape[1], _ptr(x), _ptr(D), len(D), d, g, _ptr(out))
    return rc, out


def alc(X, x, D, cand, d, g, L=None):
    """(alc, v_j(c), cov_j(x,c), v_j(x)) for candidates ``cand`` given design D."""
    X = _f64(X); x = _f64(x); D = _i32(D); cand = _i32(cand)
    a = np.empty(len(cand)); v = np.empty(len(cand)); cv = np.empty(len(cand)); vx = np.empty(1)
    rc = (L or lib()).lagp_oracle_alc(_ptr(X), X.shape[1], _ptr(x), _ptr(D), len(D), _ptr(cand), len(cand),
                               d, g, _ptr(a), _ptr(v), _ptr(cv), _ptr(vx))
    if rc != OK:
        raise ValueError(f"oracle alc failed: {rc}")
    return a, v, cv, float(vx[0])


def alc_brute(X, x, D, cand, d, g, L=None):
    X = _f64(X); x = _f64(x); D = _i32(D); cand = _i32(cand)
    a = np.empty(len(cand))
    rc = (L or lib()).lagp_oracle_alc_brute(_ptr(X), X.shape[1], _ptr(x), _ptr(D), len(D), _ptr(cand),
                                     len(cand), d, g, _ptr(a))
    if rc != OK:
        raise ValueError(f"oracle brute alc failed: {rc}")
    return a


def local(X, y, x, n0, n, M, d, g, replay=None, L=None):
    """Greedy ALC design + prediction at one location.

    Returns (rc, sel[n], out[5] = {mean, s2, var, v_n(x), psi}, diag[n,3])."""
    X = _f64(X); y = _f64(y); x = _f64(x)
    sel = np.empty(n, np.int32); out = np.empty(5); diag = np.empty((n, 3))
    rp = None if replay is None else _i32(replay)
    rc = (L or lib()).lagp_oracle_local(_ptr(X), _ptr(y), X.shape[0], X.shape[1], _ptr(x), n0, n, M, d, g,
                                 _ptr(rp), _ptr(sel), _ptr(out), _ptr(diag))
    if rc < 0:
        raise ValueError(f"oracle local failed: {rc}")
    return rc, sel, out, diag


def local_ex(X, y, x, n0, n, M, d, g, start=None, vratio=0.0, replay=None, L=None):
    """lagp_oracle_local with a saved starting design (n0 = len(start)) and the
    variance-ratio stopping rule.  Returns (rc, sel[n_used], n_used, out[5], diag[n,3])."""
    X = _f64(X); y = _f64(y); x = _f64(x)
    sel = np.empty(n, np.int32); out = np.empty(5); diag = np.empty((n, 3)); nu = np.zeros(1, np.int32)
    st = None if start is None else _i32(start)
    if st is not None:
        n0 = len(st)
    rp = None if replay is None else _i32(replay)
    rc = (L or lib()).lagp_oracle_local_ex(_ptr(X), _ptr(y), X.shape[0], X.shape[1], _ptr(x), n0, n, M, d, g,
                                           _ptr(rp), _ptr(st), vratio, _ptr(sel), _ptr(nu), _ptr(out), _ptr(diag))
    if rc < 0:
        raise ValueError(f"oracle local_ex failed: {rc}")
    return rc, sel[:int(nu[0])], int(nu[0]), out, diag


def mspe(X, y, x, D, cand, d, g, L=None):
    """MSPE criterion J(c) of each candidate for the design D (eq mspe).
    Returns (rc, J, parts[ncand, 5] = {V_j(x|c), dmu_c, dV_c, V_c, G},
    scal = {F_j, dmu_x, psi, q, v_j(x)})."""
    X = _f64(X); y = _f64(y); x = _f64(x); D = _i32(D); cand = _i32(cand)
    J = np.empty(len(cand)); parts = np.empty((len(cand), 5)); scal = np.empty(5)
    rc = (L or lib()).lagp_oracle_mspe(_ptr(X), _ptr(y), X.shape[1], _ptr(x), _ptr(D), len(D), _ptr(cand), len(cand),
                                       d, g, _ptr(J), _ptr(parts), _ptr(scal))
    if rc < 0:
        raise ValueError(f"oracle mspe failed: {rc}")
    return rc, J, parts, scal


def mspe_local(X, y, x, n0, n, M, d, g, L=None):
    """Greedy MSPE design + prediction.  Returns (rc, sel[n], out[5], diag[n, 2])."""
    X = _f64(X); y = _f64(y); x = _f64(x)
    sel = np.empty(n, np.int32); out = np.empty(5); diag = np.empty((n, 2))
    rc = (L or lib()).lagp_oracle_mspe_local(_ptr(X), _ptr(y), X.shape[0], X.shape[1], _ptr(x), n0, n, M, d, g,
                                             _ptr(sel), _ptr(out), _ptr(diag))
    if rc < 0:
        raise ValueError(f"oracle mspe_local failed: {rc}")
    return rc, sel, out, diag


def batch(X, y, XX, n0, n, M, d, g, n_per=None, M_per=None, threads=0, sel_stride=None, L=None):
    """All locations, OpenMP over locations.

    Returns (status[T], sel[T, sel_stride], out[T, 5]); sel_stride defaults to
    the largest design size and entries past a location's n stay -1."""
    X = _f64(X); y = _f64(y); XX = _f64(XX)
    T = XX.shape[0]
    npe = None if n_per is None else _i32(n_per)
    mpe = None if M_per is None else _i32(M_per)
    nmax = int(npe.max()) if (npe is not None and T) else n
    stride = nmax if sel_stride is None else int(sel_stride)
    if stride < nmax:
        raise ValueError("sel_stride below the largest design size")
    sel = np.full((T, stride), -1, np.int32)
    out = np.empty((T, 5)); st = np.empty(T, np.int32)
    rc = (L or lib()).lagp_oracle_batch(_ptr(X), _ptr(y), X.shape[0], X.shape[1], _ptr(XX), T, n0, n, M,
                                 _ptr(npe), _ptr(mpe), d, g, _ptr(sel), stride, _ptr(out), _ptr(st),
                                 int(threads))
    if rc < 0:
        raise ValueError(f"oracle batch failed: {rc}")
    return st, sel, out


# Newton controls shared by the MLE functions (a reading: the paper leaves them open).
MLE_MAXIT = 100
MLE_TOL = 1e-10


def loglik(X, y, D, d, g, L=None):
    """(l, l', l'') of the local design D at lengthscale d (eqs gpk, dl, d2l)."""
    X = _f64(X); y = _f64(y); D = _i32(D)
    out = np.empty(3)
    rc = (L or lib()).lagp_oracle_loglik(_ptr(X), _ptr(y), X.shape[1], _ptr(D), len(D), d, g, _ptr(out))
    if rc < 0:
        raise ValueError(f"oracle loglik failed: {rc}")
    return rc, out


def mle(X, y, D, d0, g, tmin, tmax, maxit=MLE_MAXIT, tol=MLE_TOL, L=None):
    """(rc, theta_hat, iterations) by Newton's method from d0."""
    X = _f64(X); y = _f64(y); D = _i32(D)
    th = np.empty(1); it = np.empty(1, np.int32)
    rc = (L or lib()).lagp_oracle_mle(_ptr(X), _ptr(y), X.shape[1], _ptr(D), len(D), d0, g, tmin, tmax,
                                      maxit, tol, _ptr(th), _ptr(it))
    if rc < 0:
        raise ValueError(f"oracle mle failed: {rc}")
    return rc, float(th[0]), int(it[0])


def alc2(X, y, x, n0, n, M, d0, g, tmin, tmax, maxit=MLE_MAXIT, tol=MLE_TOL, L=None):
    """Two-stage scheme: (rc, sel1, sel2, (theta1, theta2), out[5])."""
    X = _f64(X); y = _f64(y); x = _f64(x)
    s1 = np.empty(n, np.int32); s2 = np.empty(n, np.int32); th = np.empty(2); out = np.empty(5)
    rc = (L or lib()).lagp_oracle_alc2(_ptr(X), _ptr(y), X.shape[0], X.shape[1], _ptr(x), n0, n, M, d0, g,
                                       tmin, tmax, maxit, tol, _ptr(s1), _ptr(s2), _ptr(th), _ptr(out))
    if rc < 0:
        raise ValueError(f"oracle alc2 failed: {rc}")
    return rc, s1, s2, (float(th[0]), float(th[1])), out


def max_threads() -> int:
    return int(lib().lagp_oracle_max_threads())
