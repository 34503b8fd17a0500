"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle."""
import numpy as np
import pytest

import oracle
import workloads
from parity import compare, gpu_predict

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="session")
def lagp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_1303_0383_amd as L   # raises if the HIP library is missing
    return L


@pytest.fixture(scope="session")
def c0(lagp):
    w = workloads.c0()
    return w, lagp.Design(w.X, w.y)


@pytest.fixture(scope="session")
def c1(lagp):
    w = workloads.c1()
    return w, lagp.Design(w.X, w.y)


@pytest.fixture(scope="session")
def c2(lagp):
    w = workloads.c2(T=100000)
    return w, lagp.Design(w.X, w.y)


def _knn_gpu(design, XX, M):
    import torch
    XXd = torch.as_tensor(XX, device="cuda:0")
    idx = design.knn(XXd, M)
    torch.cuda.synchronize()
    return idx.cpu().numpy()


# ------------------------------------------------------------------ kNN
@pytest.mark.parametrize("M", [1, 6, 50, 999, 1000])
def test_knn_c0_exact(c0, M):
    w, D = c0
    idx = _knn_gpu(D, w.XX, M)
    for t in range(w.T):
        ref, _ = oracle.knn(w.X, w.XX[t], M)
        assert np.array_equal(idx[t], ref), t


def test_knn_c1_exact(c1):
    w, D = c1
    sub = np.arange(0, w.T, 97)
    idx = _knn_gpu(D, w.XX[sub], w.ncand)
    for k, t in enumerate(sub):
        ref, _ = oracle.knn(w.X, w.XX[t], w.ncand)
        assert np.array_equal(idx[k], ref), t


def test_knn_c2_exact(c2):
    w, D = c2
    sub = np.arange(0, 300)
    idx = _knn_gpu(D, w.XX[sub], 2000)
    for k in range(0, 300, 7):
        ref, _ = oracle.knn(w.X, w.XX[sub[k]], 2000)
        assert np.array_equal(idx[k], ref), k


def test_knn_ties_grid(lagp):
    # A regular grid design has many exactly equal distances: ties go by index.
    g = np.linspace(-1, 1, 21)
    X = np.stack(np.meshgrid(g, g), -1).reshape(-1, 2)
    D = lagp.Design(X, np.zeros(len(X)))
    XX = np.array([[0.0, 0.0], [0.05, 0.05], [0.1, 0.0], [1.0, 1.0]])
    for M in (5, 13, 60, 441):
        idx = _knn_gpu(D, XX, M)
        for t in range(len(XX)):
            ref, _ = oracle.knn(X, XX[t], M)
            assert np.array_equal(idx[t], ref), (M, t)


@pytest.mark.parametrize("p", [3, 8, 12])
def test_knn_ragged_rows(lagp, p):
    """Design sizes whose last rows do not fill a group of four rows, split
    over several blocks (and estimated on a sample whose size is ragged too),
    with a location count that does not fill a block; p = 12 takes the
    runtime-dimension path."""
    r = np.random.default_rng(300 + p)
    for N in (4099, 70001):
        X = r.uniform(0.0, 1.0, (N, p))
        D = lagp.Design(X, np.zeros(N))
        XX = r.uniform(0.0, 1.0, (77, p))
        for M in (1, 37, 1000):
            idx = _knn_gpu(D, XX, M)
            for t in range(0, 77, 11):
                ref, _ = oracle.knn(X, XX[t], M)
                assert np.array_equal(idx[t], ref), (N, M, t)


@pytest.mark.parametrize("layout", ["far_sample", "near_sample", "duplicates"])
def test_knn_unrepresentative_sample(lagp, layout):
    """The kNN first estimates each location's candidate radius on every 16th
    design row.  Designs whose sample misrepresents the rest (the estimate
    misses low or high, or collapses to zero) must still give exact sets."""
    r = np.random.default_rng(17)
    N, p = 20000, 3
    X = r.uniform(0.0, 1.0, (N, p))
    if layout == "far_sample":
        X[::16] += 5.0                      # the sample lies far from every location
    elif layout == "near_sample":
        X[1::16] += 5.0                     # ... and the rest in part far away
        X[2::16] += 5.0
        X[::16] = 0.5 + 0.01 * (X[::16] - 0.5)   # the sample packed near the centre
    else:
        X[::16] = X[0]                      # the sample is one repeated point
    D = lagp.Design(X, np.zeros(N))
    XX = np.concatenate([r.uniform(0.0, 1.0, (300, p)), X[:5]])
    for M in (40, 700, 2000):
        idx = _knn_gpu(D, XX, M)
        for t in range(0, len(XX), 7):
            ref, _ = oracle.knn(X, XX[t], M)
            assert np.array_equal(idx[t], ref), (layout, M, t)


@pytest.mark.parametrize("layout", ["far", "tiny", "all_equal", "mixed_scales"])
def test_knn_octave_clamps(lagp, layout):
    """The first histogram bins squared distances by octave, clamped to
    [2^-51, 2^11); keys outside that range all fall in an end bin and must be
    resolved by the refinement passes (at most 18 in all): distances far above
    2^11, far below 2^-51, a design of one repeated point (every key differs
    only in its index), and a design spanning both clamps at once."""
    r = np.random.default_rng(23)
    N, p = 20000, 3
    X = r.uniform(0.0, 1.0, (N, p))
    XX = r.uniform(0.0, 1.0, (40, p))
    if layout == "far":
        X *= 1000.0                          # d^2 up to 3e6
        XX *= 1000.0
    elif layout == "tiny":
        X *= 1e-12                           # d^2 near 1e-24
        XX *= 1e-12
    elif layout == "all_equal":
        X[:] = X[0]
    else:
        X[: N // 2] *= 1e-12                 # half the design near the origin
        X[N // 2:] *= 1000.0                 # the other half far out
        XX = np.concatenate([XX[:20] * 1e-12, XX[20:] * 1000.0])
    D = lagp.Design(X, np.zeros(N))
    for M in (1, 50, 2000):
        idx = _knn_gpu(D, XX, M)
        for t in range(0, len(XX), 3):
            ref, _ = oracle.knn(X, XX[t], M)
            assert np.array_equal(idx[t], ref), (layout, M, t)


# ------------------------------------------------------------- predict
def test_predict_c0_full(c0):
    w, D = c0
    res = gpu_predict(D, w.XX, w.n0, w.n, w.ncand, w.d, w.g)
    summary = compare(w.X, w.y, w.XX, w.n0, w.n, w.ncand, w.d, w.g, res)
    print("c0", summary)
    assert summary["identical"] + summary["replayed"] == w.T


def test_predict_c1_subset(c1):
    w, D = c1
    sub = np.arange(0, w.T, 37)                       # 271 locations over the grid
    XX = w.XX[sub]
    res = gpu_predict(D, XX, w.n0, w.n, w.ncand, w.d, w.g)
    summary = compare(w.X, w.y, XX, w.n0, w.n, w.ncand, w.d, w.g, res)
    print("c1", summary)


@pytest.mark.parametrize("n", [50, 64])
def test_predict_c2_subset(c2, n):
    w, D = c2
    XX = w.XX[:300]
    res = gpu_predict(D, XX, w.n0, n, w.ncand, w.d, w.g)
    summary = compare(w.X, w.y, XX, w.n0, n, w.ncand, w.d, w.g, res, idx=range(0, 300, 10))
    print("c2 n=%d" % n, summary)


def test_predict_c2_full_size_sampled(c2):
    """The headline launch configuration (N=100k, T=100k, n=50), sampled."""
    w, D = c2
    res = gpu_predict(D, w.XX, w.n0, 50, w.ncand, w.d, w.g)
    assert np.all(res["status"] == 0)
    assert np.all(np.isfinite(res["mean"])) and np.all(res["s2"] > 0)
    sample = np.random.default_rng(5).choice(w.T, 24, replace=False)
    summary = compare(w.X, w.y, w.XX, w.n0, 50, w.ncand, w.d, w.g, res, idx=sample)
    print("c2 full sampled", summary)


def test_predict_uneven_sizes(c2):
    w, D = c2
    r = np.random.default_rng(11)
    T = 40
    XX = w.XX[1000:1000 + T]
    n_per = r.integers(16, 129, T).astype(np.int32)
    M_per = (256 * r.integers(1, 17, T)).astype(np.int32)
    res = gpu_predict(D, XX, w.n0, int(n_per.max()), int(M_per.max()), w.d, w.g, n_per=n_per, M_per=M_per)
    summary = compare(w.X, w.y, XX, w.n0, 0, 0, w.d, w.g, res, idx=range(0, T, 3), n_per=n_per, M_per=M_per)
    print("uneven", summary)


# ------------------------------------------------------------ edge cases
def test_empty_batch(c0):
    import torch
    w, D = c0
    out = D.predict(torch.empty((0, 2), dtype=torch.float64, device="cuda:0"), 6, 50, 1000, 0.5, 1e-6)
    assert out.mean.numel() == 0


@pytest.mark.parametrize("T", [1, 255, 257, 513])
def test_ragged_batches(c1, T):
    w, D = c1
    XX = w.XX[3:3 + T]
    res = gpu_predict(D, XX, w.n0, 20, 200, w.d, w.g)
    compare(w.X, w.y, XX, w.n0, 20, 200, w.d, w.g, res, idx=sorted({0, T // 2, T - 1}))


def test_n_equals_n0_is_nn_kriging(c1):
    w, D = c1
    XX = w.XX[:64]
    res = gpu_predict(D, XX, 12, 12, 40, w.d, w.g)
    compare(w.X, w.y, XX, 12, 12, 40, w.d, w.g, res)


def test_n_equals_ncand(c0):
    w, D = c0
    XX = w.XX[:10]
    res = gpu_predict(D, XX, 3, 30, 30, w.d, w.g)
    compare(w.X, w.y, XX, 3, 30, 30, w.d, w.g, res)


@pytest.mark.parametrize("p", [1, 3, 5, 12])
def test_other_dimensions(lagp, p):
    r = np.random.default_rng(100 + p)
    X = r.uniform(0, 1, (3000, p))
    y = np.sin(X @ r.standard_normal(p))
    XX = r.uniform(0, 1, (40, p))
    D = lagp.Design(X, y)
    res = gpu_predict(D, XX, 4, 24, 300, 0.5 * p, 1e-4)
    compare(X, y, XX, 4, 24, 300, 0.5 * p, 1e-4, res)
    idx = _knn_gpu(D, XX, 300)
    for t in range(0, 40, 9):
        assert np.array_equal(idx[t], oracle.knn(X, XX[t], 300)[0])


def test_small_n_variance(c0):
    w, D = c0
    res = gpu_predict(D, w.XX[:5], 1, 2, 10, w.d, w.g)
    assert np.all(np.isnan(res["var"])) and np.all(res["s2"] > 0)
    compare(w.X, w.y, w.XX[:5], 1, 2, 10, w.d, w.g, res)


def test_notpd_duplicates(lagp):
    # Duplicate rows with zero nugget: the starting design is singular.
    X = np.repeat(np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0]]), 3, axis=0)
    X = np.vstack([X, np.random.default_rng(1).uniform(2, 3, (40, 2))])
    y = np.arange(len(X), dtype=np.float64)
    D = lagp.Design(X, y)
    XX = np.array([[0.01, 0.0], [2.5, 2.5]])
    res = gpu_predict(D, XX, 2, 4, 10, 0.5, 0.0)
    assert res["status"][0] == 1 and np.isnan(res["mean"][0])
    rc, _, _, _ = oracle.local(X, y, XX[0], 2, 4, 10, 0.5, 0.0)
    assert rc == oracle.NOTPD


def test_alone_equals_in_batch(c1):
    """A location's result does not depend on the rest of the batch."""
    w, D = c1
    XX = w.XX[:300]
    full = gpu_predict(D, XX, w.n0, w.n, w.ncand, w.d, w.g)
    for t in (0, 150, 299):
        one = gpu_predict(D, XX[t:t + 1], w.n0, w.n, w.ncand, w.d, w.g)
        assert np.array_equal(one["sel"][0], full["sel"][t])
        assert one["mean"][0] == full["mean"][t] and one["s2"][0] == full["s2"][t]
    perm = np.random.default_rng(2).permutation(300)
    pr = gpu_predict(D, XX[perm], w.n0, w.n, w.ncand, w.d, w.g)
    assert np.array_equal(pr["mean"], full["mean"][perm])
    assert np.array_equal(pr["sel"], full["sel"][perm])


def test_invalid_arguments(c0, lagp):
    import torch
    w, D = c0
    XX = torch.as_tensor(w.XX[:4], device="cuda:0")
    bad = [dict(n0=0, n=10, ncand=20), dict(n0=5, n=4, ncand=20), dict(n0=2, n=30, ncand=20),
           dict(n0=2, n=10, ncand=1001), dict(n0=2, n=10, ncand=20, d=0.0), dict(n0=2, n=10, ncand=20, g=-1.0)]
    for b in bad:
        kw = dict(d=0.5, g=1e-6)
        kw.update(b)
        with pytest.raises(lagp.LagpError) as e:
            D.predict(XX, kw["n0"], kw["n"], kw["ncand"], kw["d"], kw["g"])
        assert e.value.code == lagp.LAGP_E_INVAL
    with pytest.raises(lagp.LagpError):
        D.predict(torch.as_tensor(w.XX[:4]), 2, 10, 20, 0.5, 1e-6)   # host tensor


# --------------------------------------------------- prediction from designs
def test_predict_designs_matches_oracle(c2, lagp):
    import torch
    w, D = c2
    XX = w.XX[500:540]
    sel = np.stack([oracle.local(w.X, w.y, XX[t], w.n0, 50, w.ncand, w.d, w.g)[1] for t in range(len(XX))])
    out = D.predict_designs(torch.as_tensor(XX, device="cuda:0"), torch.as_tensor(sel, device="cuda:0"), w.d, w.g)
    torch.cuda.synchronize()
    for t in range(len(XX)):
        rc, ref = oracle.predict(w.X, w.y, XX[t], sel[t], w.d, w.g)
        assert abs(out.mean[t].item() - ref[0]) <= 1e-9 * max(abs(ref[0]), np.std(w.y))
        assert abs(out.s2[t].item() - ref[1]) <= 1e-9 * ref[1]
        assert abs(out.var[t].item() - ref[2]) <= 1e-9 * ref[2]
        assert out.df[t].item() == 50 and out.status[t].item() == 0


def test_predict_designs_rejects_bad_indices(c0, lagp):
    import torch
    w, D = c0
    sel = torch.tensor([[0, 1, 2, 3], [0, 1, -1, 3], [0, 1, 2, 5000]], dtype=torch.int32, device="cuda:0")
    out = D.predict_designs(torch.as_tensor(w.XX[:3], device="cuda:0"), sel, w.d, w.g)
    torch.cuda.synchronize()
    st = out.status.cpu().numpy()
    assert st[0] == 0 and st[1] == 1 and st[2] == 1
    assert np.isnan(out.mean[1].item()) and np.isnan(out.mean[2].item())


# ------------------------------------------------------- mixed precision
@pytest.mark.parametrize("n", [50, 64])
def test_mixed_precision_c2(c2, lagp, n):
    w, D = c2
    XX = w.XX[2000:2200]
    res = gpu_predict(D, XX, w.n0, n, w.ncand, w.d, w.g, precision=lagp.LAGP_PREC_SCORE_FP32)
    assert np.all(res["status"] == 0)
    from parity import mixed_metrics
    m = mixed_metrics(w.X, w.y, XX, w.n0, n, w.ncand, w.d, w.g, res, idx=range(0, 200, 4))
    print("mixed c2 n=%d" % n, m)
    assert m["step_agreement"] >= 0.99
    assert m["prediction_parity"] <= 1e-9
    assert m["mean_rms_over_sd"] <= 1e-4
    # The short list is re-scored exactly in FP64 in the FP64 kernel's
    # operation order: where the sequences agree, the outputs are the FP64
    # path's bit for bit.
    ref = gpu_predict(D, XX, w.n0, n, w.ncand, w.d, w.g)
    same = np.all(res["sel"][:, :n] == ref["sel"][:, :n], axis=1)
    assert same.mean() >= 0.99, same.mean()
    for k in ("mean", "s2", "var"):
        assert np.array_equal(res[k][same], ref[k][same]), k


def test_mixed_precision_c1_reported(c1, lagp):
    # The 2-D workload has nugget 1e-6: the FP32 tile cannot resolve v_j(c)
    # near g (its sums are of order 1), so its short list often misses the
    # FP64 winner.  Reported here; the bar is gated (and expected to fail) below.
    w, D = c1
    XX = w.XX[::211]
    res = gpu_predict(D, XX, w.n0, w.n, w.ncand, w.d, w.g, precision=lagp.LAGP_PREC_SCORE_FP32)
    from parity import mixed_metrics
    m = mixed_metrics(w.X, w.y, XX, w.n0, w.n, w.ncand, w.d, w.g, res, idx=range(0, len(XX), 2))
    print("mixed c1", m)
    assert m["prediction_parity"] <= 1e-9


def test_bf16_tile_c2_reported(c2, lagp):
    """The BF16 ranking tile (rows stored as bfloat16, FP32 accumulation) with
    the same exact FP64 re-score of its short list: it runs, and the FP64
    prediction from its chosen indices matches the oracle's; its agreement is
    reported here and the bar gated (and expected to fail) below."""
    w, D = c2
    XX = w.XX[2000:2100]
    res = gpu_predict(D, XX, w.n0, w.n, w.ncand, w.d, w.g, precision=lagp.LAGP_PREC_SCORE_BF16)
    assert np.all(res["status"] == 0)
    from parity import mixed_metrics
    m = mixed_metrics(w.X, w.y, XX, w.n0, w.n, w.ncand, w.d, w.g, res, idx=range(0, 100, 4))
    print("bf16 tile c2", m)
    assert m["prediction_parity"] <= 1e-9


@pytest.mark.xfail(strict=True, reason="bfloat16 rows (2^-9 relative rounding) compound through the incremental "
                                       "tile: the short list rarely holds the FP64 winner")
def test_bf16_tile_c2_bar(c2, lagp):
    w, D = c2
    XX = w.XX[2000:2100]
    res = gpu_predict(D, XX, w.n0, w.n, w.ncand, w.d, w.g, precision=lagp.LAGP_PREC_SCORE_BF16)
    from parity import mixed_metrics
    m = mixed_metrics(w.X, w.y, XX, w.n0, w.n, w.ncand, w.d, w.g, res, idx=range(0, 100, 4))
    assert m["step_agreement"] >= 0.99 and m["mean_rms_over_sd"] <= 1e-4


@pytest.mark.xfail(strict=True, reason="FP32 ranking cannot resolve v_j(c) near the 1e-6 nugget of the 2-D workload")
def test_mixed_precision_c1_bar(c1, lagp):
    w, D = c1
    XX = w.XX[::211]
    res = gpu_predict(D, XX, w.n0, w.n, w.ncand, w.d, w.g, precision=lagp.LAGP_PREC_SCORE_FP32)
    from parity import mixed_metrics
    m = mixed_metrics(w.X, w.y, XX, w.n0, w.n, w.ncand, w.d, w.g, res, idx=range(0, len(XX), 2))
    assert m["step_agreement"] >= 0.99 and m["mean_rms_over_sd"] <= 1e-4
