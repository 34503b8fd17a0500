"""Pins for the FP64 CPU oracle.

Each pin checks the oracle against something other than itself: a worked
example, a closed form, an identity of the paper written with an independent
dense-algebra route (NumPy solves and inverses), a special case that reduces
to textbook GP kriging, or brute force on a tiny input.  ``test_planted_*``
builds the oracle with deliberate mistakes and checks that some pin fails for
each one.
"""
import math
import os
import re
import tempfile

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- helpers
def corr_np(A, B, theta):
    """exp(-||a-b||^2/theta) for all pairs (dense NumPy route)."""
    d2 = ((A[:, None, :] - B[None, :, :]) ** 2).sum(-1)
    return np.exp(-d2 / theta)


def design_cov_np(XD, theta, eta):
    return corr_np(XD, XD, theta) + eta * np.eye(len(XD))


def gp_np(XD, yD, x, theta, eta):
    """Textbook GP prediction (eqs predgp, preds2) by dense solves."""
    K = design_cov_np(XD, theta, eta)
    k = corr_np(XD, x[None, :], theta)[:, 0]
    Kik = np.linalg.solve(K, k)
    Kiy = np.linalg.solve(K, yD)
    n = len(yD)
    mean = k @ Kiy
    psi = yD @ Kiy
    v = 1.0 + eta - k @ Kik
    return mean, psi * v / n, v, psi


def var_np(XD, x, theta, eta):
    K = design_cov_np(XD, theta, eta)
    k = corr_np(XD, x[None, :], theta)[:, 0]
    return 1.0 + eta - k @ np.linalg.solve(K, k)


def read_golden(name):
    design, x, meta = [], None, {}
    with open(os.path.join(GOLDEN, name)) as f:
        mode = None
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "design":
                mode = "design"
            elif tok[0] == "x":
                x = np.array([float(t) for t in tok[1:]])
                mode = None
            elif mode == "design":
                design.append((int(tok[0]), [float(t) for t in tok[1:]]))
            else:
                meta[tok[0]] = [int(t) for t in tok[1:]]
    design.sort()
    X = np.array([v for _, v in design])
    return X, x, meta


def small_problem(seed=7, N=80, p=2, lo=-2.0, hi=2.0):
    r = np.random.default_rng(seed)
    X = r.uniform(lo, hi, (N, p))
    y = np.sin(3 * X[:, 0]) + X[:, -1] ** 2
    x = r.uniform(lo / 2, hi / 2, p)
    return X, y, x


# -------------------------------------------------------------------- pins
def pin_knn_golden(L=None):
    X, x, meta = read_golden("knn_ties_1d.txt")
    idx, d2 = oracle.knn(X, x, len(X), L=L)
    assert list(idx) == meta["order"], (list(idx), meta["order"])


def pin_knn_nearest_set(L=None):
    r = np.random.default_rng(3)
    X = np.round(r.uniform(0, 1, (500, 3)), 2)   # coarse values: many exact ties
    x = np.array([0.5, 0.5, 0.5])
    for M in (1, 7, 60, 500):
        idx, d2 = oracle.knn(X, x, M, L=L)
        d2_all = ((X - x) ** 2).sum(1)
        order = np.lexsort((np.arange(len(X)), d2_all))
        assert np.array_equal(idx, order[:M])
        assert np.allclose(d2, d2_all[idx], rtol=1e-15, atol=0)


def pin_alc_three_forms(L=None):
    """cov^2/v (eq dxy2) == brute v_j(x) - v_{j+1}(x|c) == eq dxy with the
    partition-inverse sign of g (SM Section 1)."""
    for (seed, p, theta, eta) in ((1, 2, 0.5, 1e-4), (2, 8, 1.0, 1e-4), (5, 3, 0.3, 1e-3)):
        X, y, x = small_problem(seed, N=60, p=p, lo=0.0 if p > 2 else -2.0, hi=1.0 if p > 2 else 2.0)
        C, _ = oracle.knn(X, x, 40)
        D, cand = C[:7], C[7:]
        a, vc, cov, vx = oracle.alc(X, x, D, cand, theta, eta, L=L)
        # brute force by dense NumPy solves (independent of the oracle)
        v0 = var_np(X[D], x, theta, eta)
        brute = np.array([v0 - var_np(X[np.append(D, c)], x, theta, eta) for c in cand])
        # eq dxy with g = -K^{-1}k / v (partition inverse sign)
        Ki = np.linalg.inv(design_cov_np(X[D], theta, eta))
        kx = corr_np(X[D], x[None], theta)[:, 0]
        dxy = []
        for c in cand:
            kc = corr_np(X[D], X[c][None], theta)[:, 0]
            v = 1 + eta - kc @ Ki @ kc
            gvec = -Ki @ kc / v
            Kxc = corr_np(x[None], X[c][None], theta)[0, 0]
            dxy.append(kx @ np.outer(gvec, gvec) @ kx * v + 2 * kx @ gvec * Kxc + Kxc ** 2 / v)
        dxy = np.array(dxy)
        scale = max(np.abs(brute).max(), 1e-300)
        assert np.max(np.abs(a - brute)) <= 1e-8 * scale, (seed, np.max(np.abs(a - brute)) / scale)
        assert np.max(np.abs(a - dxy)) <= 1e-8 * scale
        assert abs(vx - v0) <= 1e-10 * max(v0, eta)


def pin_alc_closed_form_j1(L=None):
    """One design point a: v_1(c) = 1+eta - K(a,c)^2/(1+eta),
    cov_1(x,c) = K(x,c) - K(x,a) K(a,c)/(1+eta)."""
    theta, eta = 0.7, 1e-6
    X = np.array([[0.1], [-0.2], [0.3], [1.4], [-0.9]])
    x = np.array([0.0])
    K = lambda u, w: math.exp(-(u - w) ** 2 / theta)
    a, vc, cov, vx = oracle.alc(X, x, [0], [1, 2, 3, 4], theta, eta, L=L)
    for i, c in enumerate([1, 2, 3, 4]):
        v = 1 + eta - K(0.1, X[c, 0]) ** 2 / (1 + eta)
        cv = K(0.0, X[c, 0]) - K(0.0, 0.1) * K(0.1, X[c, 0]) / (1 + eta)
        assert abs(vc[i] - v) <= 1e-14
        assert abs(cov[i] - cv) <= 1e-14
        assert abs(a[i] - cv * cv / v) <= 1e-13 * max(cv * cv / v, 1e-300)
    assert abs(vx - (1 + eta - K(0.0, 0.1) ** 2 / (1 + eta))) <= 1e-14


def pin_symmetric_tie_golden(L=None):
    X, x, meta = read_golden("alc_symmetric_tie_1d.txt")
    rc, sel, out, diag = oracle.local(X, X[:, 0] * 0 + 1.0, x, 1, 2, len(X), 1.0, 1e-6, L=L)
    assert rc == 0 and list(sel) == meta["sel"], list(sel)
    assert diag[1, 0] == diag[1, 1]    # the top two scores are an exact tie


def pin_greedy_is_brute_argmax(L=None):
    """Each greedy choice maximises the brute-force variance reduction."""
    for (seed, theta, eta) in ((11, 0.5, 1e-4), (12, 0.2, 1e-3)):
        X, y, x = small_problem(seed, N=70)
        n0, n, M = 3, 12, 45
        rc, sel, out, diag = oracle.local(X, y, x, n0, n, M, theta, eta, L=L)
        assert rc == 0
        C, _ = oracle.knn(X, x, M)
        assert list(sel[:n0]) == list(C[:n0])
        for j in range(n0, n):
            D = sel[:j]
            rest = [c for c in C if c not in set(D)]
            v0 = var_np(X[D], x, theta, eta)
            red = np.array([v0 - var_np(X[np.append(D, c)], x, theta, eta) for c in rest])
            best = red.max()
            assert red[rest.index(sel[j])] >= best - 1e-9 * best, (j, seed)
            assert abs(diag[j, 0] - best) <= 1e-8 * best


def pin_bounds_along_path(L=None):
    """0 <= ALC <= v_j(x); v_j(c) >= eta (up to rounding); v_{j+1}(x) = v_j(x) - ALC(s)."""
    w = workloads.c0()
    for t in (0, 37, 99):
        x = w.XX[t]
        rc, sel, out, diag = oracle.local(w.X, w.y, x, w.n0, 20, w.ncand, w.d, w.g, L=L)
        assert rc == 0
        C, _ = oracle.knn(w.X, x, w.ncand)
        prev = None
        for j in range(w.n0, 20):
            D = sel[:j]
            rest = np.array([c for c in C if c not in set(D)])
            a, vc, cov, vx = oracle.alc(w.X, x, D, rest, w.d, w.g, L=L)
            assert np.all(a >= 0) and np.all(a <= vx * (1 + 1e-6) + 1e-15)
            assert np.all(vc >= w.g * (1 - 1e-3))
            if prev is not None:
                assert vx <= prev[0] * (1 + 1e-9) + 1e-18
                assert abs(vx - (prev[0] - prev[1])) <= 1e-6 * prev[0] + 1e-15
            prev = (vx, a.max())


def pin_pie_and_updates(L=None):
    """Partition-inverse update (SM Section 1) against a direct inverse;
    log|K_{j+1}| = log|K_j| + log v_j(x_{j+1}); psi update (eq psiup)."""
    w = workloads.c2(T=4)
    X, y = w.X[:3000], w.y[:3000]
    x = w.XX[1]
    rc, sel, out, diag = oracle.local(X, y, x, w.n0, 24, 400, w.d, w.g, L=L)
    assert rc == 0
    j0 = w.n0
    Ki = np.linalg.inv(design_cov_np(X[sel[:j0]], w.d, w.g))
    for j in range(j0, 24):
        D, s = sel[:j], sel[j]
        k = corr_np(X[D], X[s][None], w.d)[:, 0]
        v = 1 + w.g - k @ Ki @ k
        gvec = -Ki @ k / v
        Kn = np.block([[Ki + np.outer(gvec, gvec) * v, gvec[:, None]], [gvec[None, :], np.array([[1 / v]])]])
        Kd = np.linalg.inv(design_cov_np(X[sel[:j + 1]], w.d, w.g))
        assert np.linalg.norm(Kn - Kd) <= 1e-9 * np.linalg.norm(Kd)
        # oracle's v_j(s)
        _, vc, _, _ = oracle.alc(X, x, D, [s], w.d, w.g, L=L)
        assert abs(vc[0] - v) <= 1e-9 * v
        ld0 = np.linalg.slogdet(design_cov_np(X[D], w.d, w.g))[1]
        ld1 = np.linalg.slogdet(design_cov_np(X[sel[:j + 1]], w.d, w.g))[1]
        assert abs(ld1 - (ld0 + math.log(vc[0]))) <= 1e-8 * max(1.0, abs(ld1))
        # psi via eq psiup with h = Y_j' g
        _, o0 = oracle.predict(X, y, x, D, w.d, w.g, L=L)
        _, o1 = oracle.predict(X, y, x, sel[:j + 1], w.d, w.g, L=L)
        h = y[D] @ gvec
        psi1 = o0[4] + h * h * v + 2 * y[s] * h + y[s] ** 2 / v
        assert abs(psi1 - o1[4]) <= 1e-8 * abs(o1[4])
        Ki = Kn


def pin_full_gp(L=None):
    """n = N (all points as candidates): the local predictor is the full GP."""
    X, y, x = small_problem(21, N=14)
    theta, eta = 0.6, 1e-3
    rc, sel, out, _ = oracle.local(X, y, x, 2, 14, 14, theta, eta, L=L)
    assert rc == 0 and sorted(sel) == list(range(14))
    mean, s2, v, psi = gp_np(X, y, x, theta, eta)
    assert abs(out[0] - mean) <= 1e-10 * max(1.0, abs(mean))
    assert abs(out[1] - s2) <= 1e-9 * s2
    assert abs(out[2] - s2 * 14 / 12) <= 1e-9 * s2


def pin_nn_kriging(L=None):
    """n = n0: plain nearest-neighbour kriging."""
    X, y, x = small_problem(22, N=200)
    theta, eta = 0.3, 1e-5
    rc, sel, out, _ = oracle.local(X, y, x, 10, 10, 50, theta, eta, L=L)
    assert rc == 0
    nn = np.argsort(((X - x) ** 2).sum(1), kind="stable")[:10]
    assert list(sel) == list(nn)
    mean, s2, v, psi = gp_np(X[nn], y[nn], x, theta, eta)
    assert abs(out[0] - mean) <= 1e-9 * max(1.0, abs(mean))
    assert abs(out[1] - s2) <= 1e-8 * s2
    assert abs(out[3] - v) <= 1e-8 * v


def pin_interpolation(L=None):
    """At a design point, as eta -> 0: mean -> y_i and v_n(x) -> O(eta)."""
    X, y, _ = small_problem(23, N=300)
    for eta in (1e-6, 1e-8):
        for i in (5, 123):
            rc, sel, out, _ = oracle.local(X, y, X[i], 4, 16, 100, 0.4, eta, L=L)
            assert rc == 0 and sel[0] == i
            assert abs(out[0] - y[i]) <= 50 * eta * max(1.0, np.abs(y).max())
            assert 0.5 * eta <= out[3] <= 2.5 * eta


def pin_variance_nonnegative(L=None):
    w = workloads.c0()
    st, sel, out = oracle.batch(w.X, w.y, w.XX, w.n0, w.n, w.ncand, w.d, w.g, L=L)
    assert np.all(st == 0)
    assert np.all(out[:, 1] > 0) and np.all(out[:, 2] > 0)
    assert np.allclose(out[:, 2], out[:, 1] * w.n / (w.n - 2), rtol=1e-15)


def pin_alc_brute_dense(L=None):
    """The oracle's brute-force mode, v_j(x) - v_{j+1}(x|c) from two fresh
    factorisations, against the same difference by dense NumPy solves; an
    augmented matrix that is singular (a candidate duplicating a design
    point with no nugget) scores NaN."""
    for (seed, p, theta, eta) in ((3, 2, 0.5, 1e-4), (4, 8, 1.0, 1e-4)):
        X, y, x = small_problem(seed, N=60, p=p, lo=0.0 if p > 2 else -2.0, hi=1.0 if p > 2 else 2.0)
        C, _ = oracle.knn(X, x, 30)
        D, cand = C[:6], C[6:]
        a = oracle.alc_brute(X, x, D, cand, theta, eta, L=L)
        v0 = var_np(X[D], x, theta, eta)
        dense = np.array([v0 - var_np(X[np.append(D, c)], x, theta, eta) for c in cand])
        scale = max(np.abs(dense).max(), 1e-300)
        assert np.max(np.abs(a - dense)) <= 1e-9 * scale, (seed, np.max(np.abs(a - dense)) / scale)
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 0.0], [0.5, 0.5]])
    a = oracle.alc_brute(X, np.array([0.2, 0.1]), np.array([0, 1]), np.array([2, 3]), 0.5, 0.0, L=L)
    assert np.isnan(a[0]) and np.isfinite(a[1]) and a[1] > 0


def pin_batch_matches_local(L=None):
    """The batch over locations (Section 4.1) writes, for every location, what
    a single-location call gives: per-location n and N' override the uniform
    values, rows sit at the caller's stride, entries past a location's n are
    left alone, and the thread count changes nothing."""
    X, y, _ = small_problem(29, N=140)
    r = np.random.default_rng(30)
    T = 9
    XX = r.uniform(-1.8, 1.8, (T, 2))
    n_per = r.integers(5, 19, T).astype(np.int32)
    M_per = r.integers(20, 90, T).astype(np.int32)
    n0, d, g = 4, 0.5, 1e-5
    stride = int(n_per.max()) + 3
    st, sel, out = oracle.batch(X, y, XX, n0, 12, 60, d, g, n_per=n_per, M_per=M_per, threads=3,
                                sel_stride=stride, L=L)
    assert sel.shape == (T, stride)
    for t in range(T):
        rc, s1, o1, _ = oracle.local(X, y, XX[t], n0, int(n_per[t]), int(M_per[t]), d, g, L=L)
        assert st[t] == rc == 0
        assert np.array_equal(sel[t, :n_per[t]], s1), t
        assert np.all(sel[t, n_per[t]:] == -1), t
        assert np.array_equal(out[t], o1), t
    st1, sel1, out1 = oracle.batch(X, y, XX, n0, 12, 60, d, g, n_per=n_per, M_per=M_per, threads=1,
                                   sel_stride=stride, L=L)
    assert np.array_equal(sel1, sel) and np.array_equal(out1, out)
    # uniform sizes: every location uses the call's n and N'
    st2, sel2, out2 = oracle.batch(X, y, XX[:3], n0, 10, 50, d, g, L=L)
    for t in range(3):
        rc, s1, o1, _ = oracle.local(X, y, XX[t], n0, 10, 50, d, g, L=L)
        assert np.array_equal(sel2[t], s1) and np.array_equal(out2[t], o1)


def pin_design_ignores_y(L=None):
    X, y, x = small_problem(24, N=150)
    r1 = oracle.local(X, y, x, 4, 20, 100, 0.5, 1e-5, L=L)
    r2 = oracle.local(X, np.random.default_rng(0).standard_normal(150), x, 4, 20, 100, 0.5, 1e-5, L=L)
    assert np.array_equal(r1[1], r2[1])


def pin_permutation_invariance(L=None):
    X, y, x = small_problem(25, N=150)
    perm = np.random.default_rng(1).permutation(150)
    inv = np.argsort(perm)
    r1 = oracle.local(X, y, x, 4, 20, 100, 0.5, 1e-5, L=L)
    r2 = oracle.local(X[perm], y[perm], x, 4, 20, 100, 0.5, 1e-5, L=L)
    assert np.array_equal(perm[r2[1]], r1[1])
    assert np.array_equal(r1[2], r2[2])


def pin_rotation_invariance(L=None):
    """The correlation is isotropic: rotating X and x together keeps the design
    and, up to rounding, the prediction."""
    X, y, x = small_problem(26, N=150, p=3)
    Q, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((3, 3)))
    r1 = oracle.local(X, y, x, 4, 20, 100, 0.5, 1e-4, L=L)
    r2 = oracle.local(X @ Q.T, y, Q @ x, 4, 20, 100, 0.5, 1e-4, L=L)
    assert np.array_equal(r1[1], r2[1])
    assert abs(r1[2][0] - r2[2][0]) <= 1e-8 * max(1, abs(r1[2][0]))
    assert abs(r1[2][2] - r2[2][2]) <= 1e-6 * r1[2][2]


def pin_replay_follows(L=None):
    """Replaying the oracle's own choices reproduces its outputs; replaying a
    different valid choice reports a positive shortfall."""
    X, y, x = small_problem(27, N=120)
    rc, sel, out, diag = oracle.local(X, y, x, 3, 10, 80, 0.5, 1e-4, L=L)
    rc2, sel2, out2, diag2 = oracle.local(X, y, x, 3, 10, 80, 0.5, 1e-4, replay=sel, L=L)
    assert np.array_equal(sel, sel2) and np.array_equal(out, out2)
    assert np.all(diag2[3:, 0] == diag2[3:, 2])
    C, _ = oracle.knn(X, x, 80)
    alt = sel.copy()
    alt[5] = [c for c in C if c not in set(sel)][0]
    rc3, sel3, out3, diag3 = oracle.local(X, y, x, 3, 10, 80, 0.5, 1e-4, replay=alt, L=L)
    assert diag3[5, 2] < diag3[5, 0]


PINS = [pin_knn_golden, pin_knn_nearest_set, pin_alc_three_forms, pin_alc_closed_form_j1,
        pin_symmetric_tie_golden, pin_greedy_is_brute_argmax, pin_bounds_along_path,
        pin_pie_and_updates, pin_full_gp, pin_nn_kriging, pin_interpolation,
        pin_variance_nonnegative, pin_alc_brute_dense, pin_batch_matches_local, pin_design_ignores_y, pin_permutation_invariance,
        pin_rotation_invariance, pin_replay_follows]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin, oracle_lib):
    pin()


def test_notpd_duplicates_without_nugget(oracle_lib):
    """Duplicate design rows with eta = 0 make K_j singular: the location is
    flagged and its outputs are NaN."""
    X = np.array([[0.0, 0.0], [0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    rc, sel, out, _ = oracle.local(X, np.ones(4), np.array([0.1, 0.1]), 2, 3, 4, 0.5, 0.0)
    assert rc == oracle.NOTPD and np.all(np.isnan(out))


def test_invalid_arguments(oracle_lib):
    X, y, x = small_problem(28, N=20)
    for args in ((0, 5, 10), (6, 5, 10), (2, 11, 10), (2, 5, 21)):
        with pytest.raises(ValueError):
            oracle.local(X, y, x, *args, 0.5, 1e-4)


# ------------------------------------------------------ planted mistakes
# (description, regex on the oracle source, replacement)
MUTATIONS = [
    ("Cholesky drops the off-diagonal update",
     r"for \(int l = 0; l < m; l\+\+\) s -= L\[\(size_t\)i \* n \+ l\] \* L\[\(size_t\)m \* n \+ l\];",
     "for (int l = 0; l < m; l++) s -= 0.0 * L[(size_t)i * n + l];"),
    ("forward substitution sign flipped",
     r"s -= L\[\(size_t\)i \* n \+ l\] \* w\[l\];", "s += L[(size_t)i * n + l] * w[l];"),
    ("nugget missing from the design diagonal", r"\? 1\.0 \+ eta\n", "? 1.0\n"),
    ("cov adds instead of subtracts",
     r"corr\(x, xc, p, theta\) - dot\(wx, wc, j\)", "corr(x, xc, p, theta) + dot(wx, wc, j)"),
    ("criterion cov/v instead of cov^2/v", r"cov \* cov / vc", "fabs(cov) / vc"),
    ("candidate rows built from the NN list instead of the design",
     r"kc\[a\] = corr\(X \+ \(size_t\)sel\[a\] \* p, xc", "kc[a] = corr(X + (size_t)C[a] * p, xc"),
    ("kNN ties broken by larger index",
     r"return \(a->i > b->i\) - \(a->i < b->i\);", "return (a->i < b->i) - (a->i > b->i);"),
    ("argmax ties broken by larger index", r"alc == a1 && C\[ci\] < C\[best\]", "alc == a1 && C[ci] > C[best]"),
    ("scale divides by n-2", r"out\[1\] = psi \* vx / n;", "out[1] = psi * vx / (n - 2);"),
    ("lengthscale multiplies", r"exp\(-sqdist\(a, b, p\) / theta\)", "exp(-sqdist(a, b, p) * theta)"),
    ("distance drops the last coordinate", r"for \(int k = 0; k < p; k\+\+\) \{", "for (int k = 0; k < p - 1; k++) {"),
    ("predictive variance ignores the nugget", r"double vx = \(1\.0 \+ eta\) - dot\(wx, wx, n\);",
     "double vx = 1.0 - dot(wx, wx, n);"),
    ("mean uses the wrong vector", r"double mean = dot\(wx, u, n\);", "double mean = dot(wx, yd, n);"),
    ("brute form appends the first candidate for every candidate", r"D1\[j\] = cand\[ci\];", "D1[j] = cand[0];"),
    ("brute form reverses the difference", r"alc\[ci\] = v0 - v1;", "alc[ci] = v1 - v0;"),
    ("batch ignores the per-location design size", r"int32_t nt = n_per \? n_per\[t\] : n;", "int32_t nt = n;"),
    ("batch ignores the per-location candidate count", r"int64_t Mt = M_per \? M_per\[t\] : M;", "int64_t Mt = M;"),
    ("batch rows at the design size instead of the stride", r"sel \+ \(size_t\)t \* sel_stride",
     "sel + (size_t)t * nt"),
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
