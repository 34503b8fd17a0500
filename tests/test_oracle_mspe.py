"""Pins for the oracle's MSPE criterion (eq mspe of Section 3.1, with the
derivative expressions of Section 3.1 and SM Section 2) and its greedy
design.

Each part of J(c) is checked against a definition evaluated independently
by dense NumPy algebra: the predictive mean and variance of the candidate
and of x at theta +- h (central differences for their theta-derivatives),
the Fisher information as minus a second difference of the NumPy log
likelihood, and the reduced variance V_j(x|c) by a dense solve with c added
to the design.  The greedy choice is the argmin of that NumPy J.
``test_planted_*`` rebuilds the oracle with deliberate mistakes.
"""
import os
import re
import tempfile

import numpy as np
import pytest

import oracle
import workloads


def _dense(X, y, D, z, th, g):
    """mu(z), V(z) = psi v(z)/(j-2) and psi for the design rows D at lengthscale th."""
    mu, v, psi = _dense_v(X, y, D, z, th, g)
    return mu, psi * v / (len(D) - 2), psi


def _dense_v(X, y, D, z, th, g):
    """mu(z), v(z) = 1 + g - k'K^{-1}k and psi by dense solves."""
    XD = X[D]
    K = np.exp(-((XD[:, None, :] - XD[None, :, :]) ** 2).sum(-1) / th) + g * np.eye(len(D))
    k = np.exp(-((XD - z) ** 2).sum(-1) / th)
    Y = y[D]
    return k @ np.linalg.solve(K, Y), 1.0 + g - k @ np.linalg.solve(K, k), Y @ np.linalg.solve(K, Y)


def _loglik(X, y, D, th, g):
    XD = X[D]
    K = np.exp(-((XD[:, None, :] - XD[None, :, :]) ** 2).sum(-1) / th) + g * np.eye(len(D))
    _, ld = np.linalg.slogdet(K)
    return -0.5 * ld - 0.5 * len(D) * np.log(y[D] @ np.linalg.solve(K, y[D]))


def _numpy_J(X, y, x, D, cand, th, g):
    j = len(D)
    h = 1e-4 * th        # first differences
    h2 = 3e-3 * th       # the second difference: larger steps keep rounding below truncation
    F = -(_loglik(X, y, D, th + h2, g) - 2 * _loglik(X, y, D, th, g) + _loglik(X, y, D, th - h2, g)) / h2 ** 2
    dmux = (_dense(X, y, D, x, th + h, g)[0] - _dense(X, y, D, x, th - h, g)[0]) / (2 * h)
    psi = _dense(X, y, D, x, th, g)[2]
    J = []
    for c in cand:
        mp, Vp, _ = _dense(X, y, D, X[c], th + h, g)
        mm, Vm, _ = _dense(X, y, D, X[c], th - h, g)
        _, Vc, _ = _dense(X, y, D, X[c], th, g)
        dmu, dV = (mp - mm) / (2 * h), (Vp - Vm) / (2 * h)
        G = F + dV * dV / (2 * Vc * Vc) + dmu * dmu / Vc
        # V_j(x|c): psi_j/(j-2) times the correlation-scale variance at x with c added
        vxc = _dense_v(X, y, np.append(D, c), x, th, g)[1]
        J.append(psi / (j - 2) * vxc + dmux * dmux / G)
    return np.array(J), F, dmux


G_PIN = 1e-3   # a nugget that keeps v_{j+1}(x|c) well above rounding, so that both routes resolve it


def _case(t=7, j=12, nc=40):
    w = workloads.c0()
    w.g = G_PIN
    x = w.XX[t]
    rc, sel, _, _ = oracle.local(w.X, w.y, x, w.n0, 20, 1000, w.d, w.g)
    C, _ = oracle.knn(w.X, x, 200)
    D = sel[:j]
    cand = np.array([c for c in C if c not in D][:nc], np.int32)
    return w, x, D, cand


def pin_criterion_against_numpy(L=None):
    for t, j in ((7, 12), (40, 8), (81, 20)):
        w, x, D, cand = _case(t, j)
        rc, J, parts, scal = oracle.mspe(w.X, w.y, x, D, cand, w.d, w.g, L=L)
        Jn, F, dmux = _numpy_J(w.X, w.y, x, D, cand, w.d, w.g)
        assert rc == 0
        assert abs(scal[0] - F) <= 1e-4 * abs(F), (scal[0], F)
        assert abs(scal[1] - dmux) <= 1e-5 * abs(dmux) + 1e-12, (scal[1], dmux)
        assert np.allclose(J, Jn, rtol=1e-5, atol=0), np.max(np.abs(J / Jn - 1))


def pin_parts_against_numpy(L=None):
    w, x, D, cand = _case()
    rc, J, parts, scal = oracle.mspe(w.X, w.y, x, D, cand, w.d, w.g, L=L)
    h = 1e-5 * w.d
    for i in (0, 9, 33):
        c = cand[i]
        mp, Vp, _ = _dense(w.X, w.y, D, w.X[c], w.d + h, w.g)
        mm, Vm, _ = _dense(w.X, w.y, D, w.X[c], w.d - h, w.g)
        _, Vc, psi = _dense(w.X, w.y, D, w.X[c], w.d, w.g)
        assert abs(parts[i, 1] - (mp - mm) / (2 * h)) <= 1e-6 * abs(parts[i, 1]) + 1e-12
        assert abs(parts[i, 2] - (Vp - Vm) / (2 * h)) <= 1e-5 * abs(parts[i, 2]) + 1e-14
        assert abs(parts[i, 3] - Vc) <= 1e-9 * Vc
        assert abs(scal[2] - psi) <= 1e-9 * psi


def pin_greedy_choice_is_numpy_argmin(L=None):
    w = workloads.c0()
    w.g = G_PIN
    x = w.XX[55]
    M = 60
    rc, sel, out, diag = oracle.mspe_local(w.X, w.y, x, w.n0, w.n0 + 3, M, w.d, w.g, L=L)
    assert rc == 0
    C, _ = oracle.knn(w.X, x, M)
    for j in range(w.n0, w.n0 + 3):
        D = sel[:j]
        cand = np.array([c for c in C if c not in D], np.int32)
        Jn, _, _ = _numpy_J(w.X, w.y, x, D, cand, w.d, w.g)
        best = Jn.min()
        assert Jn[list(cand).index(sel[j])] <= best * (1 + 1e-6), (j, sel[j])
    rc2, o2 = oracle.predict(w.X, w.y, x, sel, w.d, w.g, L=L)
    assert np.array_equal(out, o2)


PINS = [pin_criterion_against_numpy, pin_parts_against_numpy, pin_greedy_choice_is_numpy_argmin]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin()


def test_mspe_needs_three_points():
    w, x, D, cand = _case()
    with pytest.raises(ValueError):
        oracle.mspe(w.X, w.y, x, D[:2], cand, w.d, w.g)
    with pytest.raises(ValueError):
        oracle.mspe_local(w.X, w.y, x, 2, 10, 100, w.d, w.g)


MUTATIONS = [
    ("printed +q in dV", r"dVc = \(-q \* vc", "dVc = (q * vc"),
    ("missing factor 2 in the dV cross term", r"2\.0 \* dot\(kd, kt, j\)", "dot(kd, kt, j)"),
    ("G without the mean-derivative term", r"\+ dmuc \* dmuc / Vc;", ";"),
    ("j-1 instead of j-2", r"const double sc = psi / \(j - 2\);", "const double sc = psi / (j - 1);"),
    ("argmax instead of argmin", r"J\[a\] < j1 \|\|", "J[a] > j1 ||"),
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
