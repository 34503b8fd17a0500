"""GPU tests of the serving engine (continuous batching under an HBM budget)
through the C ABI: results against lagp_predict and the FP64 oracle, a
request alone against the same request mixed into other traffic, requests cut
into pieces, a short request admitted and completed while a long one runs,
admission against the budget, and mixed models in one queue."""
import numpy as np
import pytest

import workloads
from parity import compare, gpu_predict

pytestmark = pytest.mark.gpu

GiB = 1 << 30


@pytest.fixture(scope="session")
def lagp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_1303_0383_amd as L
    return L


@pytest.fixture(scope="session")
def c4(lagp):
    X, y, _ = workloads.c4_design()
    return X, y, lagp.Design(X, y)


def _served_equals(a, b):
    for k in ("mean", "s2", "var"):
        assert np.array_equal(getattr(a, k), getattr(b, k), equal_nan=True), k
    for k in ("df", "sel", "status"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k


def test_server_matches_predict_and_oracle(c4, lagp):
    X, y, D = c4
    prm = workloads.C4_PARAMS
    reqs = workloads.c4_requests(6, 100.0)
    S = lagp.Server(D, 8 * GiB)
    tickets = [S.submit(r.XX, prm["n0"], r.n, r.ncand, prm["d"], prm["g"]) for r in reqs]
    outs = [S.wait(t) for t in tickets]
    for r, o in zip(reqs, outs):
        assert np.all(o.status == 0)
        assert np.all(o.df == r.n)
        assert o.done >= o.submitted
        ref = gpu_predict(D, r.XX, prm["n0"], r.n, r.ncand, prm["d"], prm["g"])
        for k in ("mean", "s2", "var", "df", "status"):
            assert np.array_equal(getattr(o, k), ref[k]), k
        assert np.array_equal(o.sel, ref["sel"][:, :r.n])
    # a few locations against the oracle (the kNN scan of 10^6 points dominates its cost)
    r, o = reqs[0], outs[0]
    res = {"mean": o.mean, "s2": o.s2, "var": o.var, "df": o.df, "sel": o.sel, "status": o.status}
    summary = compare(X, y, r.XX, prm["n0"], r.n, r.ncand, prm["d"], prm["g"], res, idx=range(min(3, len(r.XX))))
    print("served vs oracle", summary)
    S.close()


def test_alone_equals_mixed(c4, lagp):
    """A request's results are bitwise the same alone and batched with other traffic."""
    X, y, D = c4
    prm = workloads.C4_PARAMS
    reqs = workloads.c4_requests(40, 100.0)
    S = lagp.Server(D, 16 * GiB)
    probe = reqs[7]
    alone = S.wait(S.submit(probe.XX, prm["n0"], probe.n, probe.ncand, prm["d"], prm["g"]))
    b0, _, r0, _ = S.stats()
    # a burst: everything queued while the first batch runs is batched together
    tickets = []
    for k, r in enumerate(reqs):
        tickets.append(S.submit(r.XX, prm["n0"], r.n, r.ncand, prm["d"], prm["g"]))
        if k == 20:
            tp = S.submit(probe.XX, prm["n0"], probe.n, probe.ncand, prm["d"], prm["g"])
    mixed = S.wait(tp)
    for t in tickets:
        S.wait(t)
    b1, _, r1, _ = S.stats()
    print("burst: requests", r1 - r0, "pieces", b1 - b0)
    assert r1 - r0 == len(reqs) + 1
    assert b1 - b0 < r1 - r0, "the burst was not batched"
    _served_equals(alone, mixed)
    S.close()


def test_pieces_split_requests(c4, lagp):
    """Pieces of 7 locations: every request is cut across pieces and pieces
    hold parts of several requests (one with per-location n and N'); the
    results equal lagp_predict's bitwise."""
    X, y, D = c4
    prm = workloads.C4_PARAMS
    reqs = workloads.c4_requests(5, 100.0)
    r = np.random.default_rng(21)
    xu = r.uniform(0.0, 1.0, (23, 4))
    nu = r.integers(8, 65, 23).astype(np.int32)
    mu = r.integers(200, 1500, 23).astype(np.int32)
    S = lagp.Server(D, 4 * GiB, slots=4, piece=7)
    tickets = [S.submit(q.XX, prm["n0"], q.n, q.ncand, prm["d"], prm["g"]) for q in reqs]
    tu = S.submit(xu, prm["n0"], nu, mu, prm["d"], prm["g"])
    for q, t in zip(reqs, tickets):
        o = S.wait(t)
        ref = gpu_predict(D, q.XX, prm["n0"], q.n, q.ncand, prm["d"], prm["g"])
        for k in ("mean", "s2", "var", "df", "status"):
            assert np.array_equal(getattr(o, k), ref[k], equal_nan=True), k
        assert np.array_equal(o.sel, ref["sel"][:, :q.n])
    o = S.wait(tu)
    ref = gpu_predict(D, xu, prm["n0"], int(nu.max()), int(mu.max()), prm["d"], prm["g"], n_per=nu, M_per=mu)
    for k in ("mean", "s2", "var", "df", "status"):
        assert np.array_equal(getattr(o, k), ref[k], equal_nan=True), k
    for t in range(len(xu)):
        assert np.array_equal(o.sel[t, :nu[t]], ref["sel"][t, :nu[t]])
    pieces, locs, nreq, _ = S.stats()
    total = sum(len(q.XX) for q in reqs) + len(xu)
    assert locs == total and nreq == len(reqs) + 1
    assert pieces >= -(-total // 7)
    S.close()


def test_short_request_overtakes_long_work(c4, lagp):
    """Continuous batching: a one-location request submitted while a long
    request (16384 locations, n = 100, N' = 4000) is on the device is admitted
    at once, runs beside it and completes first, at its own completion time;
    both give lagp_predict's results bitwise."""
    import time
    X, y, D = c4
    prm = workloads.C4_PARAMS
    r = np.random.default_rng(11)
    big = r.uniform(0.0, 1.0, (16384, 4))
    small = r.uniform(0.0, 1.0, (1, 4))
    S = lagp.Server(D, 16 * GiB)
    tb = S.submit(big, prm["n0"], 100, 4000, prm["d"], prm["g"])
    time.sleep(0.05)
    ts = S.submit(small, prm["n0"], 32, 1000, prm["d"], prm["g"])
    o_s = S.wait(ts)
    o_b = S.wait(tb)
    print(f"long: {1e3 * (o_b.done - o_b.submitted):.1f} ms; short: submitted "
          f"{1e3 * (o_s.submitted - o_b.submitted):.1f} ms later, served in {1e3 * (o_s.done - o_s.submitted):.1f} ms")
    assert o_b.submitted < o_s.submitted and o_s.done < o_b.done
    pieces, _, _, _ = S.stats()
    assert pieces >= 16384 // 1024 + 1      # the default piece cap
    ref = gpu_predict(D, small, prm["n0"], 32, 1000, prm["d"], prm["g"])
    assert np.array_equal(o_s.mean, ref["mean"]) and np.array_equal(o_s.sel, ref["sel"][:, :32])
    ref = gpu_predict(D, big, prm["n0"], 100, 4000, prm["d"], prm["g"])
    for k in ("mean", "s2", "var", "df", "status"):
        assert np.array_equal(getattr(o_b, k), ref[k], equal_nan=True), k
    assert np.array_equal(o_b.sel, ref["sel"][:, :100])
    S.close()


def test_budget_admission(c4, lagp):
    X, y, D = c4
    prm = workloads.C4_PARAMS
    small = 96 << 20
    S = lagp.Server(D, small)
    r = np.random.default_rng(3).uniform(0.0, 1.0, (512, 4))
    with pytest.raises(lagp.LagpError) as e:
        S.submit(r, prm["n0"], 100, 4000, prm["d"], prm["g"])
    assert e.value.code == lagp.LAGP_E_BUDGET
    # requests that fit the budget are served
    tickets = [S.submit(r[k * 8:(k + 1) * 8], prm["n0"], 32, 1000, prm["d"], prm["g"]) for k in range(12)]
    outs = [S.wait(t) for t in tickets]
    ref = gpu_predict(D, r[:96], prm["n0"], 32, 1000, prm["d"], prm["g"])
    got = np.concatenate([o.mean for o in outs])
    assert np.array_equal(got, ref["mean"])
    S.close()


def test_mixed_models_in_queue(c4, lagp):
    """Requests with different lengthscales or precisions share the queue; each is run with its own model."""
    X, y, D = c4
    prm = workloads.C4_PARAMS
    reqs = workloads.c4_requests(8, 100.0)
    S = lagp.Server(D, 8 * GiB)
    cases = []
    for k, r in enumerate(reqs):
        d = prm["d"] if k % 2 == 0 else 0.2
        prec = lagp.LAGP_PREC_FP64 if k % 3 else lagp.LAGP_PREC_SCORE_FP32
        cases.append((r, d, prec, S.submit(r.XX, prm["n0"], r.n, r.ncand, d, prm["g"], precision=prec)))
    for r, d, prec, t in cases:
        o = S.wait(t)
        ref = gpu_predict(D, r.XX, prm["n0"], r.n, r.ncand, d, prm["g"], precision=prec)
        assert np.array_equal(o.mean, ref["mean"])
        assert np.array_equal(o.sel, ref["sel"][:, :r.n])
    S.close()


def test_server_invalid_requests(c4, lagp):
    import torch
    X, y, D = c4
    prm = workloads.C4_PARAMS
    S = lagp.Server(D, 1 * GiB)
    E = lagp.LagpError
    xx = np.random.default_rng(1).uniform(0.0, 1.0, (4, 4))
    with pytest.raises(E):
        S.submit(xx, prm["n0"], 5, 100, prm["d"], prm["g"])          # n < n0
    with pytest.raises(E):
        S.submit(xx, prm["n0"], 50, 5000, prm["d"], prm["g"])        # ncand above 4096
    with pytest.raises(E):
        S.submit(xx, prm["n0"], 50, 100, -1.0, prm["g"])             # d <= 0
    import ctypes                                                    # device arrays are refused
    dev = torch.as_tensor(xx, device="cuda:0")
    prm_c = lagp.lagp_params(prm["n0"], 50, 100, prm["d"], prm["g"], 0, 0)
    ticket = ctypes.c_uint64()
    rc = lagp._lib.lagp_server_submit(S._h, dev.data_ptr(), 4, ctypes.byref(prm_c), None, None, ctypes.byref(ticket))
    assert rc == lagp.LAGP_E_INVAL
    with pytest.raises(E):                                           # unknown ticket
        lagp.lagp_server_poll(S._h, 12345678, 0, None, None, None, None, None, 0, None, None)
    S.close()
    with pytest.raises(E):
        lagp.lagp_server_create(D.handle, 1000)                      # budget below 1 MiB
    for slots, piece in ((1, 0), (9, 0), (0, -1), (0, 1 << 18)):     # slot count, piece size
        with pytest.raises(E):
            lagp.lagp_server_create_ex(D.handle, 1 * GiB, slots, piece)
