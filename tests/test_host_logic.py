"""Host-side logic of the measurement and tuning scripts (no GPU): the
roofline bound and fractions, the stale-counter guard, the algorithmic work
counts, the autotuner's variant space and the serving request stream."""
import importlib.util
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_roofline_bound_is_the_larger_fraction(bench):
    # 1 TFLOP and 6e12 counted bytes in one second: 1/78.6 of the FP64 roof
    # against 0.75 of the HBM roof, so the memory roof binds and `achieved`
    # is in algorithmic GB/s.
    e = bench.roofline_entry("k", 1e12, 2e11, 6e12, 1.0)
    assert e["bound"] == "hbm" and e["unit"] == "GB/s"
    assert e["achieved"] == pytest.approx(200.0)
    assert e["frac"] == pytest.approx(200.0 / bench.HBM_PEAK_GBS, rel=1e-3)
    assert e["traffic_frac_of_hbm_peak"] == pytest.approx(0.75)
    assert e["flop_frac"] == pytest.approx(1.0 / bench.FP64_PEAK_TFLOPS, abs=1e-4)
    assert e["traffic_over_alg_bytes"] == pytest.approx(30.0)
    # without counters, or with little traffic, the flop roof is reported
    e = bench.roofline_entry("k", 39.3e12, 1e9, None, 1.0)
    assert e["bound"] == "alu" and e["frac"] == pytest.approx(0.5, rel=1e-3)
    e = bench.roofline_entry("k", 39.3e12, 1e9, 1e12, 1.0)
    assert e["bound"] == "alu"


def test_stale_counter_files_are_ignored(bench, tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_w_traffic.txt").write_text("# test\nkernel_source_sha16: abc\nbytes_per_launch: 1.5e+11\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda kernel="design_kernel": "abc")
    assert bench.read_traffic("k", "w") == pytest.approx(1.5e11)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda kernel="design_kernel": "def")
    assert bench.read_traffic("k", "w") is None          # taken with other sources
    assert bench.read_traffic("k", "other") is None      # no file


def test_committed_counter_files_parse(bench):
    for f in os.listdir(os.path.join(ROOT, "profiles")):
        if f.endswith("_traffic.txt"):
            vals = dict(l.split(":", 1) for l in open(os.path.join(ROOT, "profiles", f))
                        if ":" in l and not l.startswith("#"))
            assert float(vals["bytes_per_launch"]) > 0, f
            assert len(vals["kernel_source_sha16"].strip()) == 16, f


def test_algorithmic_counts(bench):
    # n = 2, n0 = 1: the gather (3pM) and one step over M - 1 live candidates
    # (3p + 2*0 + 5 + 2 for the score from step n0 - 1 = 0 on).
    M, p = 10, 3
    assert bench.design_flops(2, M, p, 1) == 3 * p * M + (M - 1) * (3 * p + 5 + 2)
    assert bench.design_flops(2, M, p, 2) == 3 * p * M + (M - 1) * (3 * p + 5)
    # c2_n50: about 7.65 MFLOP and 152,292 algorithmic bytes per location
    assert bench.design_flops(50, 2000, 8, 8) == pytest.approx(7.65e6, rel=2e-3)
    assert bench.design_alg_bytes(50, 2000, 8) == 152292
    assert bench.knn_alg_flops(100000, 100000, 8) == 240 * 10**9


def test_autotuner_variant_space():
    spec = importlib.util.spec_from_file_location(
        "autotune_under_test", os.path.join(ROOT, "paper_1303_0383_amd", "autotune.py"))
    at = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(at)
    v = at.variants(2048)
    assert len(v) == 12 and {t for t, _, _ in v} == {256, 512}
    assert {l for _, _, l in v} == set(at.LDS_SHARES) == {0, 50, 100}
    assert {t for t, _, _ in at.variants(4096)} == {512}     # above 2048 candidates: 512 threads


def test_committed_tune_table_is_well_formed():
    rows = [l.split("#")[0].split() for l in open(os.path.join(ROOT, "paper_1303_0383_amd", "tune", "table.txt"))
            if l.strip() and not l.startswith("#")]
    assert rows
    for r in rows:
        arch, prec, mc, nc, threads, coords, lds = r
        assert arch.startswith("gfx") and int(prec) in (0, 1, 2)
        assert int(mc) in (256, 512, 1024, 2048, 4096) and int(nc) in (32, 64, 128)
        assert int(threads) in (256, 512) and int(coords) in (0, 1) and 0 <= int(lds) <= 100
        if int(mc) > 2048:
            assert int(threads) == 512


def test_serving_request_stream_is_seeded():
    import workloads
    a = workloads.c4_requests(20, 100.0)
    b = workloads.c4_requests(20, 100.0)
    assert [len(r.XX) for r in a] == [len(r.XX) for r in b]
    assert all(np.array_equal(x.XX, y.XX) for x, y in zip(a, b))
    assert all(1 <= len(r.XX) <= 512 and r.n in (32, 50, 64, 100) and 1000 <= r.ncand <= 4000 for r in a)
    t = [r.arrival_s for r in a]
    assert all(t1 > t0 for t0, t1 in zip(t, t[1:]))


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU; a request for more exits with a message
    before touching any device."""
    import subprocess
    import sys
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2 and "exactly one GPU" in out.stderr and out.stdout == ""
