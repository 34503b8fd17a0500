"""GPU tests of local lengthscale inference and the two-stage scheme through
the C ABI, against the FP64 oracle.

Tolerances.  The estimate solves l'(theta) = 0; the GPU and the oracle
evaluate l' and l'' with different summation orders, so the estimates differ
by rounding amplified by the conditioning of K: |dtheta| / theta <= 1e-8.
Both searches must converge (the last steps of a converged search are at
the rounding level of l', so the iterate counts may differ by a few).  The
two-stage scheme is checked stage
by stage, each stage fed the GPU's own output of the stage before, so that
every comparison has identical inputs: second designs against the oracle's
designs at the GPU's theta1 (selection rule of the parity tests), theta2
against the oracle's estimate from the GPU's second designs, and the
prediction against the oracle's prediction from those designs at the GPU's
theta2 (1e-9 relative).
"""
import numpy as np
import pytest

import oracle
import workloads
from parity import compare, gpu_predict

pytestmark = pytest.mark.gpu

THETA_TOL = 1e-8


@pytest.fixture(scope="session")
def lagp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_1303_0383_amd as L
    return L


@pytest.fixture(scope="session")
def c0(lagp):
    w = workloads.c0()
    return w, lagp.Design(w.X, w.y)


@pytest.fixture(scope="session")
def c2(lagp):
    w = workloads.c2(n=50, T=256)
    return w, lagp.Design(w.X, w.y)


def _dev(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0")


def _mle_gpu(D, sel, d0, g, tmin, tmax, n_per=None):
    import torch
    th, it, st = D.mle(_dev(sel), d0 if np.isscalar(d0) else _dev(d0), g, tmin, tmax,
                       n_per=None if n_per is None else _dev(n_per))
    torch.cuda.synchronize()
    return th.cpu().numpy(), it.cpu().numpy(), st.cpu().numpy()


def _check_mle(w, sel, d0, th, it, st, tmin, tmax, n_per=None):
    worst = 0.0
    dit = []
    for t in range(sel.shape[0]):
        nt = int(n_per[t]) if n_per is not None else sel.shape[1]
        d0t = float(d0[t]) if np.ndim(d0) else d0
        rc, tho, ito = oracle.mle(w.X, w.y, sel[t, :nt], d0t, w.g, tmin, tmax)
        assert rc == 0 and st[t] == 0, (t, rc, st[t])
        e = abs(th[t] - tho) / tho
        worst = max(worst, e)
        assert e <= THETA_TOL, f"location {t}: theta {th[t]!r} oracle {tho!r} rel {e:.2e}"
        assert 1 <= it[t] < oracle.MLE_MAXIT and ito < oracle.MLE_MAXIT, (t, it[t], ito)
        dit.append(int(it[t]) - ito)
    print(f"iterates GPU - oracle: min {min(dit)}, max {max(dit)}, mean {np.mean(dit):.2f}")
    return worst


def test_mle_matches_oracle_c0(c0, lagp):
    w, D = c0
    tmin, tmax = workloads.mle_range(w.X)
    res = gpu_predict(D, w.XX, w.n0, w.n, w.ncand, w.d, w.g)
    sel = res["sel"][:, :w.n]
    th, it, st = _mle_gpu(D, sel, w.d, w.g, tmin, tmax)
    worst = _check_mle(w, sel, w.d, th, it, st, tmin, tmax)
    print(f"c0 mle: worst rel {worst:.2e}, mean iterations {it.mean():.2f}")


def test_mle_matches_oracle_c2(c2, lagp):
    w, D = c2
    tmin, tmax = workloads.mle_range(w.X)
    XX = w.XX[:64]
    res = gpu_predict(D, XX, w.n0, w.n, w.ncand, w.d, w.g)
    sel = res["sel"][:, :w.n]
    th, it, st = _mle_gpu(D, sel, w.d, w.g, tmin, tmax)
    worst = _check_mle(w, sel, w.d, th, it, st, tmin, tmax)
    print(f"c2 mle: worst rel {worst:.2e}, mean iterations {it.mean():.2f}")


def test_mle_uneven_sizes_and_starts(c2, lagp):
    """Per-location design sizes from 2 to 128 (the largest the LDS layout is
    sized for at p = 8) and per-location starting values, some outside the
    search interval."""
    w, D = c2
    tmin, tmax = workloads.mle_range(w.X)
    T = 40
    r = np.random.default_rng(11)
    n_per = np.concatenate([[2, 3, 128, 127], r.integers(2, 129, T - 4)]).astype(np.int32)
    sel = np.full((T, 128), -7, np.int32)
    for t in range(T):
        sel[t, :n_per[t]] = oracle.knn(w.X, w.XX[t], int(n_per[t]))[0]
    d0 = r.uniform(0.1, 3.0, T)
    d0[:3] = [tmax * 2.0, 0.0, tmin * 0.5]
    th, it, st = _mle_gpu(D, sel, d0, w.g, tmin, tmax, n_per=n_per)
    _check_mle(w, sel, d0, th, it, st, tmin, tmax, n_per=n_per)


def test_mle_designs_above_128_points(lagp):
    """A batch whose largest design has more than 128 points (130 at p = 2,
    about the most the LDS holds) runs the per-column factorisation, the
    Gauss-Jordan inverse and the vector-unit panels for all of its
    locations; sizes from 2 to 130, one of them ending on the upper bound."""
    import types
    r = np.random.default_rng(23)
    X = r.uniform(0, 1, (3000, 2))
    y = np.sin(5 * X[:, 0]) * np.cos(3 * X[:, 1]) + 0.05 * r.standard_normal(3000)
    w = types.SimpleNamespace(X=X, y=y, g=1e-3)
    D = lagp.Design(X, y)
    XX = r.uniform(0.1, 0.9, (12, 2))
    n_per = np.array([130, 129, 2, 17, 64, 65, 100, 128, 130, 129, 77, 3], np.int32)
    sel = np.full((len(XX), 130), -7, np.int32)
    for t in range(len(XX)):
        sel[t, :n_per[t]] = oracle.knn(X, XX[t], int(n_per[t]))[0]
    tmin, tmax = workloads.mle_range(X)
    th, it, st = _mle_gpu(D, sel, 0.1, w.g, tmin, tmax, n_per=n_per)
    _check_mle(w, sel, 0.1, th, it, st, tmin, tmax, n_per=n_per)


def test_mle_boundary_and_failures(lagp):
    """Two-point designs whose likelihood is monotone end on a bound; a design
    with an index outside the data or without a nugget on duplicated points
    fails alone."""
    import torch
    X = np.array([[0.0, 0.0], [0.6, 0.8], [0.6, 0.8], [1.0, 1.0]])
    y = np.array([1.0, 1.0, -1.0, 0.5])
    D = lagp.Design(X, y)
    tmin, tmax = 0.01, 10.0
    sel = np.array([[0, 1], [0, 2], [0, 9], [1, 2]], np.int32)
    for g, expect in ((1e-2, [tmax, tmin, None, None]), (0.0, [tmax, tmin, None, None])):
        th, it, st = _mle_gpu(D, sel, 0.7, g, tmin, tmax)
        for t in (0, 1):
            assert st[t] == 0 and abs(th[t] - expect[t]) <= 1e-6 * expect[t], (g, t, th[t])
            rc, tho, _ = oracle.mle(X, y, sel[t], 0.7, g, tmin, tmax)
            assert abs(th[t] - tho) <= THETA_TOL * tho
        assert st[2] == 1 and np.isnan(th[2])           # index 9 is outside the design
        if g == 0.0:                                    # duplicated point, no nugget: K singular
            assert st[3] == 1 and np.isnan(th[3])
        else:
            assert st[3] == 0
    D.close()


def test_mle_invalid_arguments(c0, lagp):
    import ctypes
    w, D = c0
    sel = _dev(np.zeros((4, 10), np.int32))
    E = lagp.LagpError
    for tmin, tmax, maxit, tol in ((0.0, 1.0, 10, 1e-10), (1.0, 0.5, 10, 1e-10), (0.1, 1.0, 0, 1e-10),
                                   (0.1, 1.0, 10, 0.0)):
        with pytest.raises(E):
            D.mle(sel, 0.5, w.g, tmin, tmax, maxit=maxit, tol=tol)
    with pytest.raises(E):
        D.mle(_dev(np.zeros((4, 1), np.int32)), 0.5, w.g, 0.1, 1.0)       # n < 2
    host = np.zeros((4, 10), np.int32)
    out = _dev(np.zeros(4))
    mp = lagp.lagp_mle_params(0.1, 1.0, 10, 1e-10)
    rc = lagp._lib.lagp_mle(D.handle, 4, host.ctypes.data, 10, None, 10, None, 0.5, w.g, ctypes.byref(mp),
                            out.data_ptr(), None, None, None)
    assert rc == lagp.LAGP_E_INVAL                                       # host array refused


def test_predict_theta_per_location(c0, lagp):
    """Designs at a lengthscale per location against the oracle, and a constant
    d_per against the scalar entry point (bitwise)."""
    import torch
    w, D = c0
    T = 30
    XX = w.XX[:T]
    d_per = np.random.default_rng(5).uniform(0.1, 2.0, T)
    out = D.predict(_dev(XX), w.n0, w.n, w.ncand, w.d, w.g, d_per=_dev(d_per))
    torch.cuda.synchronize()
    res = {k: getattr(out, k).cpu().numpy() for k in ("mean", "s2", "df", "var", "sel", "status")}
    print("d_per vs oracle", compare(w.X, w.y, XX, w.n0, w.n, w.ncand, d_per, w.g, res))
    const = D.predict(_dev(XX), w.n0, w.n, w.ncand, 1.0, w.g, d_per=_dev(np.full(T, w.d)))
    ref = D.predict(_dev(XX), w.n0, w.n, w.ncand, w.d, w.g)
    torch.cuda.synchronize()
    for k in ("mean", "s2", "var", "sel", "status"):
        assert torch.equal(getattr(const, k), getattr(ref, k)), k
    # a lengthscale that is not positive fails its location only
    bad = d_per.copy()
    bad[[2, 5]] = [0.0, np.nan]
    o2 = D.predict(_dev(XX), w.n0, w.n, w.ncand, w.d, w.g, d_per=_dev(bad))
    torch.cuda.synchronize()
    st = o2.status.cpu().numpy()
    assert st[2] == 1 and st[5] == 1 and np.isnan(o2.mean[2].item()) and (o2.sel[2] == -1).all()
    keep = [t for t in range(T) if t not in (2, 5)]
    assert torch.equal(o2.mean[keep], out.mean[keep])


def test_predict_designs_theta_per_location(c0, lagp):
    import torch
    w, D = c0
    T = 20
    res = gpu_predict(D, w.XX[:T], w.n0, w.n, w.ncand, w.d, w.g)
    sel = res["sel"][:, :w.n]
    d_per = np.linspace(0.2, 1.5, T)
    out = D.predict_designs(_dev(w.XX[:T]), _dev(sel), 1.0, w.g, d_per=_dev(d_per))
    torch.cuda.synchronize()
    for t in range(T):
        rc, o = oracle.predict(w.X, w.y, w.XX[t], sel[t], d_per[t], w.g)
        assert abs(out.mean[t].item() - o[0]) <= 1e-9 * max(abs(o[0]), np.std(w.y))
        assert abs(out.s2[t].item() - o[1]) <= 1e-9 * o[1]


def _alc2_stagewise(w, D, XX, lagp, n_per=None, M_per=None):
    """Runs the two-stage scheme and checks each stage against the oracle fed
    the GPU's previous stage.  Returns the GPU outputs."""
    import torch
    tmin, tmax = workloads.mle_range(w.X)
    T = XX.shape[0]
    out = D.predict_alc2(_dev(XX), w.n0, w.n, w.ncand, w.d, w.g, tmin, tmax,
                         n_per=None if n_per is None else _dev(n_per),
                         ncand_per=None if M_per is None else _dev(M_per))
    torch.cuda.synchronize()
    th1 = out.theta1.cpu().numpy()
    th2 = out.theta2.cpu().numpy()
    res = {k: getattr(out, k).cpu().numpy() for k in ("mean", "s2", "df", "var", "sel", "status")}
    assert np.all(res["status"] == 0)
    # stage 1: the designs at theta0 are lagp_predict's; theta1 is their MLE
    first = gpu_predict(D, XX, w.n0, w.n, w.ncand, w.d, w.g, n_per=n_per, M_per=M_per)
    for t in range(T):
        nt = int(n_per[t]) if n_per is not None else w.n
        rc, tho, _ = oracle.mle(w.X, w.y, first["sel"][t, :nt], w.d, w.g, tmin, tmax)
        assert abs(th1[t] - tho) <= THETA_TOL * tho, (t, th1[t], tho)
    # stage 2: designs at the GPU's theta1 (checked as in the parity tests)
    d1 = D.predict(_dev(XX), w.n0, w.n, w.ncand, w.d, w.g, d_per=_dev(th1),
                   n_per=None if n_per is None else _dev(n_per), ncand_per=None if M_per is None else _dev(M_per))
    torch.cuda.synchronize()
    r1 = {k: getattr(d1, k).cpu().numpy() for k in ("mean", "s2", "df", "var", "sel", "status")}
    for t in range(T):   # the pipeline's second designs are lagp_predict_theta's at theta1
        nt = int(n_per[t]) if n_per is not None else w.n
        assert np.array_equal(r1["sel"][t, :nt], res["sel"][t, :nt]), t
    summary = compare(w.X, w.y, XX, w.n0, w.n, w.ncand, th1, w.g, r1, n_per=n_per, M_per=M_per)
    # theta2: the MLE of the second designs started from theta1
    for t in range(T):
        nt = int(n_per[t]) if n_per is not None else w.n
        s2 = res["sel"][t, :nt]
        rc, tho, _ = oracle.mle(w.X, w.y, s2, th1[t], w.g, tmin, tmax)
        assert abs(th2[t] - tho) <= THETA_TOL * tho, (t, th2[t], tho)
        # the prediction: the second designs at the GPU's theta2
        rc, o = oracle.predict(w.X, w.y, XX[t], s2, th2[t], w.g)
        assert abs(res["mean"][t] - o[0]) <= 1e-9 * max(abs(o[0]), np.std(w.y)), t
        assert abs(res["s2"][t] - o[1]) <= 1e-9 * o[1], t
        if nt > 2:
            assert abs(res["var"][t] - o[2]) <= 1e-9 * o[2], t
        assert res["df"][t] == nt
    return res, th1, th2, summary


def test_alc2_stagewise_c0(c0, lagp):
    w, D = c0
    res, th1, th2, summary = _alc2_stagewise(w, D, w.XX, lagp)
    print("alc2 c0: second designs", summary, "theta1 range", th1.min(), th1.max())
    # end to end against the oracle's own two-stage run where no selection
    # was decided by a near-tie: same thetas and predictions
    tmin, tmax = workloads.mle_range(w.X)
    same = 0
    for t in range(0, 100, 7):
        rc, s1, s2, (t1, t2), o = oracle.alc2(w.X, w.y, w.XX[t], w.n0, w.n, w.ncand, w.d, w.g, tmin, tmax)
        if np.array_equal(s2, res["sel"][t, :w.n]):
            same += 1
            assert abs(th2[t] - t2) <= THETA_TOL * t2
            assert abs(res["mean"][t] - o[0]) <= 1e-9 * max(abs(o[0]), np.std(w.y))
    assert same >= 10, same


def test_alc2_stagewise_c2_uneven(c2, lagp):
    w, D = c2
    T = 24
    r = np.random.default_rng(3)
    n_per = r.integers(16, 65, T).astype(np.int32)
    M_per = (256 * r.integers(1, 9, T)).astype(np.int32)
    res, th1, th2, summary = _alc2_stagewise(w, D, w.XX[:T], lagp, n_per=n_per, M_per=M_per)
    print("alc2 c2 uneven:", summary)


def test_alc2_mixed_precision_runs(c2, lagp):
    """The mixed mode applies to both design passes; the estimates and
    predictions come from FP64 kernels on the designs it chose."""
    import torch
    w, D = c2
    tmin, tmax = workloads.mle_range(w.X)
    XX = w.XX[:32]
    out = D.predict_alc2(_dev(XX), w.n0, w.n, w.ncand, w.d, w.g, tmin, tmax, precision=lagp.LAGP_PREC_SCORE_FP32)
    torch.cuda.synchronize()
    st = out.status.cpu().numpy()
    assert np.all(st == 0)
    sel = out.sel.cpu().numpy()
    th1 = out.theta1.cpu().numpy()
    th2 = out.theta2.cpu().numpy()
    for t in range(0, 32, 4):
        rc, tho, _ = oracle.mle(w.X, w.y, sel[t, :w.n], th1[t], w.g, tmin, tmax)
        assert abs(th2[t] - tho) <= THETA_TOL * tho
        rc, o = oracle.predict(w.X, w.y, XX[t], sel[t, :w.n], th2[t], w.g)
        assert abs(out.mean[t].item() - o[0]) <= 1e-9 * max(abs(o[0]), np.std(w.y))


def test_alc2_invalid_arguments(c0, lagp):
    w, D = c0
    E = lagp.LagpError
    XX = _dev(w.XX[:4])
    with pytest.raises(E):
        D.predict_alc2(XX, 1, 1, 10, w.d, w.g, 0.1, 1.0)          # n < 2
    with pytest.raises(E):
        D.predict_alc2(XX, w.n0, w.n, w.ncand, w.d, w.g, 1.0, 0.1)  # tmin >= tmax


def test_alc2_failure_stays_local(lagp):
    """A location whose first design cannot be factorised (duplicated points,
    no nugget) ends with status NOTPD and NaN estimates and outputs; the
    other locations are unaffected."""
    import torch
    r = np.random.default_rng(21)
    X = r.uniform(0, 1, (400, 2))
    X[1] = X[0]                      # an exact duplicate next to the first location
    y = np.sin(4 * X[:, 0]) + X[:, 1]
    XX = np.vstack([X[0] + 1e-4, r.uniform(0.2, 0.8, (5, 2))])
    D = lagp.Design(X, y)
    out = D.predict_alc2(_dev(XX), 3, 12, 60, 0.3, 0.0, 1e-3, 2.0)
    torch.cuda.synchronize()
    st = out.status.cpu().numpy()
    assert st[0] == lagp.LAGP_LOC_NOTPD
    assert np.isnan(out.mean[0].item()) and np.isnan(out.theta1[0].item()) and np.isnan(out.theta2[0].item())
    ok = D.predict_alc2(_dev(XX[1:]), 3, 12, 60, 0.3, 0.0, 1e-3, 2.0)
    torch.cuda.synchronize()
    assert np.all(st[1:] == 0)
    assert torch.equal(out.mean[1:], ok.mean) and torch.equal(out.theta2[1:], ok.theta2)
    D.close()
