"""Pins for the oracle's local lengthscale inference (eq gpk of Section 2,
eqs dl and d2l of SM Section 2, the Newton search of Section 3.2 and the
two-stage scheme of Section 4.2).

Each pin checks the oracle against something other than itself: the log
likelihood evaluated by dense NumPy algebra (slogdet and solves), derivatives
from finite differences of that NumPy likelihood, a brute-force grid search
for the maximum, closed forms on two-point designs, and the consistency of
the two-stage scheme with the one-stage functions.  ``test_planted_*``
rebuilds the oracle with deliberate mistakes and checks that a pin fails.
"""
import os
import re
import tempfile

import numpy as np
import pytest

import oracle
import workloads


def loglik_np(XD, yD, theta, eta):
    """-1/2 log|K| - n/2 log(Y'K^{-1}Y) by dense NumPy algebra (eq gpk, constant dropped)."""
    d2 = ((XD[:, None, :] - XD[None, :, :]) ** 2).sum(-1)
    K = np.exp(-d2 / theta) + eta * np.eye(len(XD))
    sign, logdet = np.linalg.slogdet(K)
    assert sign > 0
    psi = yD @ np.linalg.solve(K, yD)
    return -0.5 * logdet - 0.5 * len(yD) * np.log(psi)


def _cases():
    """(X, y, D, eta): a c0 local design, a 3-D design without nugget-free ties."""
    w = workloads.c0()
    rc, sel, _, _ = oracle.local(w.X, w.y, w.XX[7], w.n0, 24, 300, w.d, w.g)
    assert rc == 0
    r = np.random.default_rng(5)
    X3 = r.uniform(0, 1, (40, 3))
    y3 = np.sin(5 * X3[:, 0]) + X3[:, 1] * X3[:, 2] + 0.05 * r.standard_normal(40)
    return [(w.X, w.y, sel, w.g), (X3, y3, np.arange(0, 40, 2, dtype=np.int32), 1e-3)]


# --------------------------------------------------------------------- pins
def pin_loglik_matches_dense(L=None):
    for X, y, D, g in _cases():
        for th in (0.05, 0.3, 1.7):
            rc, l = oracle.loglik(X, y, D, th, g, L=L)
            ref = loglik_np(X[D], y[D], th, g)
            assert rc == 0 and abs(l[0] - ref) <= 1e-9 * max(1.0, abs(ref)), (th, l[0], ref)


def pin_first_derivative_finite_difference(L=None):
    for X, y, D, g in _cases():
        for th in (0.05, 0.3, 1.7):
            h = 1e-5 * th
            fd = (loglik_np(X[D], y[D], th + h, g) - loglik_np(X[D], y[D], th - h, g)) / (2 * h)
            _, l = oracle.loglik(X, y, D, th, g, L=L)
            assert abs(l[1] - fd) <= 1e-5 * max(1.0, abs(fd)), (th, l[1], fd)


def pin_second_derivative_finite_difference(L=None):
    for X, y, D, g in _cases():
        for th in (0.05, 0.3, 1.7):
            h = 1e-3 * th
            f = [loglik_np(X[D], y[D], th + k * h, g) for k in (-1, 0, 1)]
            fd2 = (f[0] - 2 * f[1] + f[2]) / (h * h)
            _, l = oracle.loglik(X, y, D, th, g, L=L)
            assert abs(l[2] - fd2) <= 1e-3 * max(1.0, abs(fd2)), (th, l[2], fd2)


def pin_mle_is_grid_maximum(L=None):
    tmin, tmax = 1e-3, 20.0
    for X, y, D, g in _cases():
        rc, th, it = oracle.mle(X, y, D, 0.5, g, tmin, tmax, L=L)
        assert rc == 0 and 1 <= it < oracle.MLE_MAXIT
        grid = np.exp(np.linspace(np.log(tmin * 1.01), np.log(tmax * 0.99), 4001))
        vals = np.array([loglik_np(X[D], y[D], t, g) for t in grid])
        best = grid[np.argmax(vals)]
        step = grid[1] / grid[0]
        assert best / step <= th <= best * step, (th, best)
        _, l = oracle.loglik(X, y, D, th, g, L=L)
        assert abs(l[1]) <= 1e-6 * max(1.0, abs(l[2]) * th) and l[2] < 0, l


def pin_two_point_boundaries(L=None):
    # K = [[1+g, rho], [rho, 1+g]], rho = exp(-d^2/theta).  With y = (1, 1),
    # psi = 2/(1+g+rho) and l = 1/2 log(1+g+rho) - 1/2 log(1+g-rho) + const
    # grows with rho, so the maximum is at theta = tmax; with y = (1, -1) the
    # signs swap and it is at tmin.
    X = np.array([[0.0, 0.0], [0.6, 0.8]])
    D = np.array([0, 1], np.int32)
    tmin, tmax = 0.01, 10.0
    for y, bound in ((np.array([1.0, 1.0]), tmax), (np.array([1.0, -1.0]), tmin)):
        rc, th, it = oracle.mle(X, y, D, 0.7, 1e-2, tmin, tmax, L=L)
        assert rc == 0
        assert abs(th - bound) <= 1e-6 * bound + 1e-9, (th, bound)
        rho = np.exp(-1.0 / 0.7)
        _, l = oracle.loglik(X, y, D, 0.7, 1e-2, L=L)
        s = 1.0 if y[1] > 0 else -1.0
        ref = 0.5 * np.log(1.01 + s * rho) - 0.5 * np.log(1.01 - s * rho) - np.log(2.0)
        assert abs(l[0] - ref) <= 1e-12, (l[0], ref)


def pin_two_stage_consistent(L=None):
    w = workloads.c0()
    tmin, tmax = 1e-3, 20.0
    for t in (3, 41):
        rc, s1, s2, (t1, t2), out = oracle.alc2(w.X, w.y, w.XX[t], w.n0, 20, 200, w.d, w.g, tmin, tmax, L=L)
        assert rc == 0
        r1, sel, _, _ = oracle.local(w.X, w.y, w.XX[t], w.n0, 20, 200, w.d, w.g, L=L)
        assert np.array_equal(sel, s1)
        assert oracle.mle(w.X, w.y, s1, w.d, w.g, tmin, tmax, L=L)[1] == t1
        r2, sel2, _, _ = oracle.local(w.X, w.y, w.XX[t], w.n0, 20, 200, t1, w.g, L=L)
        assert np.array_equal(sel2, s2)
        assert oracle.mle(w.X, w.y, s2, t1, w.g, tmin, tmax, L=L)[1] == t2
        rp, o = oracle.predict(w.X, w.y, w.XX[t], s2, t2, w.g, L=L)
        assert np.array_equal(o, out)
        # the second-stage prediction is a textbook GP on its design at theta2
        d2 = ((w.X[s2][:, None, :] - w.X[s2][None, :, :]) ** 2).sum(-1)
        K = np.exp(-d2 / t2) + w.g * np.eye(len(s2))
        k = np.exp(-((w.X[s2] - w.XX[t]) ** 2).sum(-1) / t2)
        assert abs(k @ np.linalg.solve(K, w.y[s2]) - out[0]) <= 1e-8 * max(1.0, abs(out[0]))


PINS = [pin_loglik_matches_dense, pin_first_derivative_finite_difference, pin_second_derivative_finite_difference,
        pin_mle_is_grid_maximum, pin_two_point_boundaries, pin_two_stage_consistent]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin()


def test_mle_invalid_arguments():
    w = workloads.c0()
    D = np.arange(10, dtype=np.int32)
    for args in ((0.5, w.g, 0.0, 1.0), (0.5, w.g, 1.0, 0.5)):
        with pytest.raises(ValueError):
            oracle.mle(w.X, w.y, D, *args)
    with pytest.raises(ValueError):
        oracle.mle(w.X, w.y, D[:1], 0.5, w.g, 1e-3, 1.0)


# ------------------------------------------------------ planted mistakes
MUTATIONS = [
    ("l' drops the trace term", r"out3\[1\] = -0\.5 \* t1 \+", "out3[1] = 0.0 * t1 +"),
    ("l'' middle term sign", r"\(r - 2\.0 \* sq\)", "(r + 2.0 * sq)"),
    ("l'' drops the squared term", r"\+ 0\.5 \* n \* q \* q / \(psi \* psi\);", ";"),
    ("dK/dtheta over theta instead of theta^2", r"Kd\[\(size_t\)a \* n \+ b\] = k \* d2 / \(theta \* theta\);",
     "Kd[(size_t)a * n + b] = k * d2 / theta;"),
    ("Newton step sign", r"\? -l\[1\] / l\[2\]", "? l[1] / l[2]"),
    ("log-likelihood uses psi^n/2 with the wrong sign", r"- 0\.5 \* n \* log\(psi\);", "+ 0.5 * n * log(psi);"),
    ("second stage starts from theta0", r"lagp_oracle_local\(X, y, N, p, x, n0, n, M, thetas\[0\]",
     "lagp_oracle_local(X, y, N, p, x, n0, n, M, theta0"),
]


@pytest.mark.parametrize("desc,pat,rep", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(desc, pat, rep, oracle_lib):
    src = open(oracle.SRC).read()
    mutated, count = re.subn(pat, rep, src)
    assert count >= 1, f"mutation pattern not found: {desc}"
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mutant.c")
        open(path, "w").write(mutated)
        lib = oracle.load(oracle.compile_source(path, os.path.join(d, "libmutant.so")))
        failed = []
        for pin in PINS:
            try:
                pin(L=lib)
            except (AssertionError, ValueError):
                failed.append(pin.__name__)
        assert failed, f"no pin catches: {desc}"
