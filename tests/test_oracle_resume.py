"""Pins for the oracle's design augmentation and stopping rule (Section 6's
discussion: designs saved as indices can be augmented, picking up where they
left off; a stopping rule on the variance ratio V_j(x) / V_{j+1}(x), in which
psi cancels).

Each pin checks the oracle against something other than the code path under
test: a resumed search against the uninterrupted search, a full given design
against a textbook GP solve by dense NumPy algebra, the first greedy choice
from an arbitrary start against a brute-force variance reduction by NumPy,
and the stopping point against the variance ratios of the uninterrupted
search computed by NumPy.  ``test_planted_*`` rebuilds the oracle with
deliberate mistakes and checks that a pin fails.
"""
import os
import re
import tempfile

import numpy as np
import pytest

import oracle
import workloads

N_FULL = 40


def _dense_v(X, D, x, d, g):
    """v(x) = 1 + g - k'K^{-1}k for the design rows D, by dense NumPy algebra."""
    XD = X[D]
    K = np.exp(-((XD[:, None, :] - XD[None, :, :]) ** 2).sum(-1) / d) + g * np.eye(len(D))
    k = np.exp(-((XD - x) ** 2).sum(-1) / d)
    return 1.0 + g - k @ np.linalg.solve(K, k)


def pin_resume_reproduces_full_run(L=None):
    w = workloads.c0()
    for t in (5, 62):
        rc, full, out, _ = oracle.local(w.X, w.y, w.XX[t], w.n0, N_FULL, 1000, w.d, w.g, L=L)
        for k in (w.n0, w.n0 + 1, 23, N_FULL - 1, N_FULL):
            rc2, sel, nu, o2, _ = oracle.local_ex(w.X, w.y, w.XX[t], w.n0, N_FULL, 1000, w.d, w.g,
                                                  start=full[:k], L=L)
            assert rc2 == 0 and nu == N_FULL
            assert np.array_equal(sel, full), (t, k)
            assert np.array_equal(o2, out), (t, k)


def pin_full_start_is_textbook_gp(L=None):
    w = workloads.c0()
    r = np.random.default_rng(2)
    x = w.XX[33]
    C, _ = oracle.knn(w.X, x, 300)
    D = r.choice(C, 25, replace=False).astype(np.int32)
    rc, sel, nu, out, _ = oracle.local_ex(w.X, w.y, x, 1, 25, 300, w.d, w.g, start=D, L=L)
    assert rc == 0 and nu == 25 and np.array_equal(sel, D)
    XD = w.X[D]
    K = np.exp(-((XD[:, None, :] - XD[None, :, :]) ** 2).sum(-1) / w.d) + w.g * np.eye(25)
    k = np.exp(-((XD - x) ** 2).sum(-1) / w.d)
    mu = k @ np.linalg.solve(K, w.y[D])
    psi = w.y[D] @ np.linalg.solve(K, w.y[D])
    v = 1.0 + w.g - k @ np.linalg.solve(K, k)
    assert abs(out[0] - mu) <= 1e-9 * max(abs(mu), np.std(w.y))
    assert abs(out[1] - psi * v / 25) <= 1e-6 * psi * v / 25


def pin_greedy_from_arbitrary_start(L=None):
    """From a start that is not the nearest neighbours, the next point is the
    candidate with the largest brute-force reduction v_j(x) - v_{j+1}(x|c)."""
    w = workloads.c0()
    r = np.random.default_rng(4)
    x = w.XX[71]
    M = 120
    C, _ = oracle.knn(w.X, x, M)
    D = r.choice(C, 8, replace=False).astype(np.int32)
    rc, sel, nu, out, _ = oracle.local_ex(w.X, w.y, x, 1, 9, M, w.d, w.g, start=D, L=L)
    assert rc == 0 and np.array_equal(sel[:8], D)
    v0 = _dense_v(w.X, D, x, w.d, w.g)
    red = {int(c): v0 - _dense_v(w.X, np.append(D, c), x, w.d, w.g) for c in C if c not in D}
    best = max(red.values())
    assert red[int(sel[8])] >= best * (1 - 1e-7), (sel[8], red[int(sel[8])], best)


def pin_stop_rule_against_variance_ratios(L=None):
    w = workloads.c0()
    for t in (5, 48):
        x = w.XX[t]
        rc, full, _, _ = oracle.local(w.X, w.y, x, w.n0, N_FULL, 1000, w.d, w.g, L=L)
        v = [_dense_v(w.X, full[:j], x, w.d, w.g) for j in range(1, N_FULL + 1)]   # v[j-1] = v_j(x)
        ratio = {j: v[j - 1] / v[j] for j in range(w.n0, N_FULL)}   # v_j / v_{j+1} for greedy step j
        for vr in (1.0, 1.02, 1.1, 1.5, 3.0):
            expect = next((j for j in range(w.n0, N_FULL) if ratio[j] < vr), N_FULL)
            near = any(abs(ratio[j] / vr - 1) < 1e-9 for j in ratio)
            rc2, sel, nu, out, _ = oracle.local_ex(w.X, w.y, x, w.n0, N_FULL, 1000, w.d, w.g, vratio=vr, L=L)
            assert rc2 == 0
            if not near:
                assert nu == expect, (t, vr, nu, expect)
            assert np.array_equal(sel, full[:nu])
            rc3, o3 = oracle.predict(w.X, w.y, x, full[:nu], w.d, w.g, L=L)
            assert np.array_equal(out, o3)


PINS = [pin_resume_reproduces_full_run, pin_full_start_is_textbook_gp, pin_greedy_from_arbitrary_start,
        pin_stop_rule_against_variance_ratios]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin()


def test_start_errors():
    w = workloads.c0()
    x = w.XX[10]
    C, _ = oracle.knn(w.X, x, 200)
    far = np.setdiff1d(np.arange(1000), C)[:1]
    with pytest.raises(ValueError):       # not among the candidates
        oracle.local_ex(w.X, w.y, x, 1, 20, 200, w.d, w.g, start=np.concatenate([C[:5], far]))
    with pytest.raises(ValueError):       # repeated
        oracle.local_ex(w.X, w.y, x, 1, 20, 200, w.d, w.g, start=np.array([C[0], C[3], C[0]]))
    with pytest.raises(ValueError):       # negative threshold
        oracle.local_ex(w.X, w.y, x, w.n0, 20, 200, w.d, w.g, vratio=-1.0)


MUTATIONS = [
    ("absolute instead of relative reduction", r"vx / vnext < vratio", "a1 < vratio - 1.0"),
    ("inverted variance ratio", r"vx / vnext < vratio", "vnext / vx < vratio"),
    ("start points stay candidates", r"sel\[j\] = C\[ci\];\n        used\[ci\] = 1;", "sel[j] = C[ci];"),
    ("start ignored", r"if \(start\) \{   /\*", "if (0) {   /*"),
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
        try:
            w = workloads.c0()
            C, _ = oracle.knn(w.X, w.XX[10], 200)
            oracle.local_ex(w.X, w.y, w.XX[10], 1, 20, 200, w.d, w.g, start=np.array([C[0], C[3], C[0]]), L=lib)
        except ValueError:
            pass
        else:
            failed.append("repeated start accepted")
        assert failed, f"no pin catches: {desc}"
