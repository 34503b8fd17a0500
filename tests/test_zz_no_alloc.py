"""lagp_predict_noalloc (the entry point for callers that cannot allocate
device memory) against lagp_predict, through the C ABI.

Both run the same kernels; the allocation-free call takes its workspace from
the library's fixed device array and runs locations in chunks that fit it.
Locations are independent (Section 4.1), so every output must be bitwise
equal to lagp_predict's.  Two calls in a row, the second with fewer
locations (the array keeps the first call's contents), in FP64 and in the
mixed mode, and a workload large enough to need several chunks.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lagp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_1303_0383_amd as L
    return L


def _run(L, D, fn, XX, n0, n, M, d, g, prec):
    import torch
    T = XX.shape[0]
    dev = XX.device
    mean = torch.full((T,), np.nan, dtype=torch.float64, device=dev)
    s2 = torch.full((T,), np.nan, dtype=torch.float64, device=dev)
    var = torch.full((T,), np.nan, dtype=torch.float64, device=dev)
    df = torch.full((T,), -7, dtype=torch.int32, device=dev)
    sel = torch.full((T, n + 2), -7, dtype=torch.int32, device=dev)
    st = torch.full((T,), 9, dtype=torch.int8, device=dev)
    prm = L.lagp_params(n0, n, M, d, g, prec, 0)
    if fn == "noalloc":
        L.lagp_predict_noalloc(D.handle, XX, T, prm, mean, s2, df, var, sel, n + 2, st)
    else:
        L.lagp_predict(D.handle, XX, T, prm, None, None, mean, s2, df, var, sel, n + 2, st)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in
            dict(mean=mean, s2=s2, var=var, df=df, sel=sel, status=st).items()}


def _same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=(a[k].dtype.kind == "f")), k


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_equals_predict_c0(lagp, prec):
    import torch
    w = workloads.c0()
    D = lagp.Design(w.X, w.y)
    XX = torch.as_tensor(w.XX, device="cuda:0")
    for T in (100, 37):   # the second call is smaller
        ref = _run(lagp, D, "predict", XX[:T], w.n0, w.n, w.ncand, w.d, w.g, prec)
        got = _run(lagp, D, "noalloc", XX[:T], w.n0, w.n, w.ncand, w.d, w.g, prec)
        _same(got, ref)
        assert np.all(got["status"] == 0)
    D.close()


def test_noalloc_equals_predict_several_chunks(lagp):
    """8-D design, N' = 2000: the 256 MiB array holds a few thousand locations
    per chunk, so 12,000 locations take several chunks."""
    import torch
    w = workloads.c2(n=50, T=12000)
    D = lagp.Design(w.X, w.y)
    XX = torch.as_tensor(w.XX, device="cuda:0")
    for T in (12000, 3001):
        ref = _run(lagp, D, "predict", XX[:T], w.n0, w.n, w.ncand, w.d, w.g, 0)
        got = _run(lagp, D, "noalloc", XX[:T], w.n0, w.n, w.ncand, w.d, w.g, 0)
        _same(got, ref)
        assert np.all(got["status"] == 0)
    D.close()


def test_noalloc_argument_errors(lagp):
    import torch
    w = workloads.c0()
    D = lagp.Design(w.X, w.y)
    XX = torch.as_tensor(w.XX[:4], device="cuda:0")
    out = torch.empty(4, dtype=torch.float64, device="cuda:0")
    E = lagp.LagpError
    with pytest.raises(E):   # strict mode needs a host wait
        lagp.lagp_predict_noalloc(D.handle, XX, 4, lagp.lagp_params(6, 20, 100, w.d, w.g, 0, lagp.LAGP_STRICT),
                                  out, out, None, None, None, 0, None)
    with pytest.raises(E):   # n > ncand
        lagp.lagp_predict_noalloc(D.handle, XX, 4, lagp.lagp_params(6, 200, 100, w.d, w.g, 0, 0),
                                  out, out, None, None, None, 0, None)
    assert lagp.lagp_noalloc_scratch_bytes() == 256 << 20
    D.close()
