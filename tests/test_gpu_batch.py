"""GPU tests of fixed-shape batches: uneven per-location sizes, bucketed
launches, and HIP-graph replay, through the C ABI, against the FP64 oracle
and against lagp_predict."""
import numpy as np
import pytest

import workloads
from parity import compare, gpu_predict, mixed_metrics

pytestmark = pytest.mark.gpu

FIELDS = ("mean", "s2", "df", "var", "sel", "status")


@pytest.fixture(scope="session")
def lagp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_1303_0383_amd as L
    return L


@pytest.fixture(scope="session")
def c3(lagp):
    w = workloads.c3()
    return w, lagp.Design(w.X, w.y)


@pytest.fixture(scope="session")
def c1(lagp):
    w = workloads.c1()
    return w, lagp.Design(w.X, w.y)


def _host(out):
    import torch
    torch.cuda.synchronize()
    return {k: getattr(out, k).cpu().numpy() for k in FIELDS}


def _same(a, b, n_per=None):
    """Bitwise equality of two result sets (NaN == NaN); sel compared over each location's n."""
    for k in ("mean", "s2", "var"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    for k in ("df", "status"):
        assert np.array_equal(a[k], b[k]), k
    if n_per is None:
        assert np.array_equal(a["sel"], b["sel"])
    else:
        for t, n in enumerate(n_per):
            assert np.array_equal(a["sel"][t, :n], b["sel"][t, :n]), t


def _uneven_small(r, T, N):
    """Small uneven sizes for full oracle parity on the 2-D design."""
    n_per = r.integers(6, 41, T).astype(np.int32)
    M_per = np.minimum(N, n_per + r.integers(0, 700, T)).astype(np.int32)
    return n_per, M_per


def test_batch_uneven_small_full_parity(c1, lagp):
    """Every location of an uneven batch (several buckets, ragged tail) against the oracle."""
    import torch
    w, D = c1
    r = np.random.default_rng(31)
    T = 300
    XX = w.XX[:T]
    n_per, M_per = _uneven_small(r, T, w.N)
    B = lagp.Batch(D, T, w.n0, 0, 0, w.d, w.g, n_per=n_per, ncand_per=M_per)
    buckets, ws = B.info()
    assert buckets > 1 and ws > 0
    XXd = torch.as_tensor(XX, device="cuda:0")
    res = _host(B.run(XXd, graph=True))
    summary = compare(w.X, w.y, XX, w.n0, 0, 0, w.d, w.g, res, n_per=n_per, M_per=M_per)
    print("batch uneven small", summary)
    B.close()


def test_batch_c3_full_size_sampled(c3, lagp):
    """The full 50,000-location uneven batch in one graph launch; sampled
    locations (including the largest n and candidate sets) against the oracle."""
    import torch
    w, D = c3
    B = lagp.Batch(D, w.T, w.n0, w.n, w.ncand, w.d, w.g, n_per=w.n_per, ncand_per=w.ncand_per)
    XXd = torch.as_tensor(w.XX, device="cuda:0")
    res = _host(B.run(XXd, graph=True))
    assert np.all(res["status"] == 0)
    assert np.array_equal(res["df"], w.n_per)
    r = np.random.default_rng(7)
    cost = w.n_per.astype(float) ** 2 * w.ncand_per
    big = np.argsort(-cost)[:2]
    small = np.argsort(cost)[:3]
    sample = np.unique(np.concatenate([big, small, r.choice(w.T, 7, replace=False)]))
    summary = compare(w.X, w.y, w.XX, w.n0, 0, 0, w.d, w.g, res, idx=sample, n_per=w.n_per, M_per=w.ncand_per)
    print("c3 sampled", summary)
    B.close()


def test_batch_graph_replays_match_eager(c3, lagp):
    """A captured batch replayed several times, with other GPU work and
    synchronisations between replays: every replay equals lagp_predict."""
    import torch
    w, D = c3
    sub = w.subset(np.arange(3000, 5000))
    XXd = torch.as_tensor(sub.XX, device="cuda:0")
    ref = gpu_predict(D, sub.XX, sub.n0, sub.n, sub.ncand, sub.d, sub.g, n_per=sub.n_per, M_per=sub.ncand_per)
    B = lagp.Batch(D, sub.T, sub.n0, sub.n, sub.ncand, sub.d, sub.g, n_per=sub.n_per, ncand_per=sub.ncand_per)
    out = B.outputs(XXd.device)
    eager = _host(B.run(XXd, out=out, graph=False))
    _same(eager, ref, sub.n_per)
    other = torch.as_tensor(w.XX[:64], device="cuda:0")
    for rep in range(3):
        for k in FIELDS:
            getattr(out, k).fill_(-7 if k in ("df", "sel", "status") else float("nan"))
        B.run(XXd, out=out, graph=True)
        torch.cuda.synchronize()
        _same(_host(out), ref, sub.n_per)
        # unrelated eager work on the same design between replays
        D.predict(other, sub.n0, 20, 300, sub.d, sub.g)
        torch.cuda.synchronize()
    # new output buffers: the batch records a new graph
    res2 = _host(B.run(XXd, graph=True))
    _same(res2, ref, sub.n_per)
    B.close()


def test_batch_uniform_matches_predict(c1, lagp):
    """A batch without per-location sizes (one bucket) equals lagp_predict, with and without sel/status."""
    import torch
    w, D = c1
    XX = w.XX[:777]
    ref = gpu_predict(D, XX, w.n0, w.n, w.ncand, w.d, w.g)
    XXd = torch.as_tensor(XX, device="cuda:0")
    B = lagp.Batch(D, len(XX), w.n0, w.n, w.ncand, w.d, w.g)
    assert B.info()[0] == 1
    _same(_host(B.run(XXd, graph=True)), ref)
    B.close()
    B = lagp.Batch(D, len(XX), w.n0, w.n, w.ncand, w.d, w.g, with_sel=False, with_status=False)
    out = B.run(XXd, graph=True)
    torch.cuda.synchronize()
    assert np.array_equal(out.mean.cpu().numpy(), ref["mean"])
    assert np.array_equal(out.s2.cpu().numpy(), ref["s2"])
    B.close()


def test_batch_mixed_precision(c3, lagp):
    """Mixed mode in a graph equals the eager mixed lagp_predict and meets the mixed-precision bar."""
    import torch
    w, D = c3
    sub = w.subset(np.arange(0, 600))
    ref = gpu_predict(D, sub.XX, sub.n0, sub.n, sub.ncand, sub.d, sub.g, n_per=sub.n_per, M_per=sub.ncand_per,
                      precision=lagp.LAGP_PREC_SCORE_FP32)
    B = lagp.Batch(D, sub.T, sub.n0, sub.n, sub.ncand, sub.d, sub.g, n_per=sub.n_per, ncand_per=sub.ncand_per,
                   precision=lagp.LAGP_PREC_SCORE_FP32)
    XXd = torch.as_tensor(sub.XX, device="cuda:0")
    for rep in range(2):
        _same(_host(B.run(XXd, graph=True)), ref, sub.n_per)
    B.close()
    m = mixed_metrics(sub.X, sub.y, sub.XX, sub.n0, sub.n, sub.ncand, sub.d, sub.g, ref, idx=range(0, 600, 10),
                      n_per=sub.n_per, M_per=sub.ncand_per)
    print("c3 mixed", m)
    assert m["step_agreement"] >= 0.99 and m["mean_rms_over_sd"] <= 1e-4


def test_mixed_redo_on_device(c1, lagp):
    """C1's tiny nugget makes some FP32 rankings lose positive definiteness;
    those locations are redone in FP64 on the device: every location the
    FP64 oracle finishes is finished, and equals the FP64 path when redone."""
    import torch
    w, D = c1
    XX = w.XX[:2000]
    mix = gpu_predict(D, XX, w.n0, w.n, w.ncand, w.d, w.g, precision=lagp.LAGP_PREC_SCORE_FP32)
    f64 = gpu_predict(D, XX, w.n0, w.n, w.ncand, w.d, w.g)
    assert np.all(mix["status"][f64["status"] == 0] == 0)
    B = lagp.Batch(D, len(XX), w.n0, w.n, w.ncand, w.d, w.g, precision=lagp.LAGP_PREC_SCORE_FP32)
    XXd = torch.as_tensor(XX, device="cuda:0")
    _same(_host(B.run(XXd, graph=True)), mix)
    B.close()
    m = mixed_metrics(w.X, w.y, XX, w.n0, w.n, w.ncand, w.d, w.g, mix, idx=range(0, 2000, 200))
    print("c1 mixed with device redo", m)


def test_batch_invalid_arguments(c1, lagp):
    import torch
    w, D = c1
    E = lagp.LagpError
    dev_sizes = torch.full((10,), 20, dtype=torch.int32, device="cuda:0")
    prm = lagp.lagp_params(w.n0, 20, 100, w.d, w.g, 0, 0)
    import ctypes
    h = ctypes.c_void_p()
    rc = lagp._lib.lagp_batch_create(D.handle, 10, ctypes.byref(prm), dev_sizes.data_ptr(), None, 0,
                                     ctypes.byref(h))
    assert rc == lagp.LAGP_E_INVAL and not h.value   # size arrays must be host arrays
    with pytest.raises(E):
        lagp.Batch(D, 10, w.n0, 20, 100, w.d, w.g, n_per=np.array([5] * 10))   # n < n0
    with pytest.raises(E):
        lagp.Batch(D, 10, w.n0, 20, 100, w.d, w.g, ncand_per=np.array([5000] * 10))   # ncand above 4096
    with pytest.raises(E):
        lagp.Batch(D, 0, w.n0, 20, 100, w.d, w.g)
    with pytest.raises(E):
        lagp.lagp_batch_create(D.handle, 10, lagp.lagp_params(w.n0, 20, 100, w.d, w.g, 0, lagp.LAGP_STRICT))
    B = lagp.Batch(D, 10, w.n0, 20, 100, w.d, w.g)
    XXd = torch.as_tensor(w.XX[:10], device="cuda:0")
    out = B.outputs(XXd.device)
    with pytest.raises(E):   # sel promised but missing
        lagp.lagp_batch_enqueue(B.handle, XXd, out.mean, out.s2, out.df, out.var, None, 20, out.status)
    with pytest.raises(E):   # sel_stride below n
        lagp.lagp_batch_enqueue(B.handle, XXd, out.mean, out.s2, out.df, out.var, out.sel, 5, out.status)
    B.close()
    del dev_sizes


def test_batch_multi_chunk_graph(c1, lagp):
    """A batch of more than 2^17 locations (several launch chunks) as one graph
    equals lagp_predict; ragged per-location sizes and the last partial chunk."""
    import torch
    w, D = c1
    T = (1 << 17) + 1234
    r = np.random.default_rng(41)
    XX = r.uniform(-2.0, 2.0, (T, 2))
    n_per = r.integers(6, 13, T).astype(np.int32)
    M_per = r.integers(16, 65, T).astype(np.int32)
    ref = gpu_predict(D, XX, w.n0, int(n_per.max()), int(M_per.max()), w.d, w.g, n_per=n_per, M_per=M_per)
    B = lagp.Batch(D, T, w.n0, 0, 0, w.d, w.g, n_per=n_per, ncand_per=M_per)
    XXd = torch.as_tensor(XX, device="cuda:0")
    for rep in range(2):
        _same(_host(B.run(XXd, graph=True)), ref, n_per)
    B.close()
    idx = r.choice(T, 6, replace=False)
    summary = compare(w.X, w.y, XX, w.n0, 0, 0, w.d, w.g, ref, idx=idx, n_per=n_per, M_per=M_per)
    print("multi-chunk", summary)
