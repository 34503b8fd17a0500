#!/usr/bin/env python3
"""Throughput benchmark: predictive locations per second of greedy ALC local
GP prediction on one MI355X.

A step is one full lagp_predict call over the batch: exact kNN candidate
sets, greedy ALC local designs and local predictions for every location,
with the design and the locations already resident in HBM.  The default
workload is the headline case N = 100,000 design points in [0,1]^8
(sinusoid-sum response + noise), T = 100,000 uniform locations, n0 = 8,
n = 50, N' = 2000 candidates, d = 1.0, g = 1e-4.

Printed: one JSON line (metric, value, roofline of the greedy-design kernel
from live HIP-event timing, CPU oracle baseline on a bounded sample, and a
parity summary of that sample against the GPU outputs).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "predictive locations/sec (n=50, N=100k) at stated accuracy; p50/p99 request latency"
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector: 256 CU x 128 flop/clk x 2.4 GHz
HBM_PEAK_GBS = 8000.0


def design_flops(n: int, M: int, p: int, n0: int) -> int:
    """Algorithmic FP64 flops of the greedy-design kernel for one location.

    Gather: M squared distances to x (3p - 1 flops) and one division by d.
    Step i = 0 .. n-2 (row i of the whitened tile) for each of the M - i - 1
    live candidates: K(s,c) distance and scaling (3p flops), the dot
    product with the chosen column (2i), the division by delta (1), the
    variance and covariance updates (2 + 2), and from step n0-1 on the ALC
    score cov^2 / v (2).  Exponentials are counted separately (see
    design_exps)."""
    f = M * 3 * p
    for i in range(n - 1):
        live = M - i - 1
        f += live * (3 * p + 2 * i + 5 + (2 if i + 1 >= n0 else 0))
    return f


def design_alg_bytes(n: int, M: int, p: int) -> int:
    """Algorithmic HBM bytes of the greedy-design kernel for one location: the
    location (8p), its candidate list (4M), the candidates' coordinates and
    responses gathered from the design (8M(p+1)), and the outputs (mean, s2,
    var, df and n design indices: 28 + 4n).  The whitened tile and every
    other intermediate could stay on chip, so they are not counted."""
    return 8 * p + 4 * M + 8 * M * (p + 1) + 28 + 4 * n


def knn_alg_flops(T: int, N: int, p: int) -> int:
    """One squared distance (3p flops: p subtractions, p squares, p - 1 adds
    and the comparison's share rounded to p) per location-design pair."""
    return T * N * 3 * p


def mle_iterate_flops(n: int) -> float:
    """FP64 flops of one Newton iterate of the likelihood kernel: Cholesky,
    in-place inversion, the K^{-1}-entry traces, the dK L^{-T} panels and the
    L^{-1} H products, about 4/3 n^3 multiply-adds."""
    return 8.0 / 3.0 * n ** 3


# Files whose text decides each kernel's memory traffic: its sources and, for
# the design kernel, the tuned variant table (the variant sets the row split).
KERNEL_SOURCES = {"design_kernel": ("design_kernel.h", "design.hip", os.path.join("..", "tune", "table.txt")),
                  "mspe_kernel": ("mspe.hip", "design_kernel.h")}


def kernel_source_hash(kernel: str = "design_kernel") -> str:
    """Hash of a kernel's sources: counter files record the hash they were
    taken with, and a counter file taken with other sources is stale."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1303_0383_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary, or None when
    it is missing or was taken with other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha16") != kernel_source_hash(kernel):
        return None
    return float(vals["bytes_per_launch"]) if "bytes_per_launch" in vals else None


def roofline_entry(kernel: str, flops: float, alg_bytes: float, traffic, avg_s: float) -> dict:
    """The kernel's bound is the larger of its FP64 flop fraction and its
    measured-traffic fraction of HBM peak; `achieved` and `frac` are against
    that roof (algorithmic bytes for the memory roof).  All three fractions
    are reported."""
    flop_rate = flops / avg_s / 1e12
    flop_frac = flop_rate / FP64_PEAK_TFLOPS
    alg_rate = alg_bytes / avg_s / 1e9
    e = {"kernel": kernel}
    traffic_frac = None
    if traffic:
        traffic_frac = traffic / avg_s / 1e9 / HBM_PEAK_GBS
    if traffic_frac is not None and traffic_frac > flop_frac:
        e.update(bound="hbm", achieved=round(alg_rate, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                 frac=round(alg_rate / HBM_PEAK_GBS, 5))
    else:
        e.update(bound="alu", achieved=round(flop_rate, 3), peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                 frac=round(flop_frac, 4))
    e.update(traffic=traffic, avg_launch_ms=round(avg_s * 1e3, 3),
             flop_frac=round(flop_frac, 4), flops_per_launch=flops,
             alg_bytes_per_launch=alg_bytes, alg_byte_frac=round(alg_rate / HBM_PEAK_GBS, 5),
             traffic_frac_of_hbm_peak=None if traffic_frac is None else round(traffic_frac, 4),
             traffic_over_alg_bytes=None if not traffic else round(traffic / alg_bytes, 1))
    return e


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def design_exps(n: int, M: int) -> int:
    return M + sum(M - i - 1 for i in range(n - 1))


def mspe_flops(n: int, M: int, p: int, n0: int) -> int:
    """Algorithmic FP64 flops of the MSPE kernel for one location: gather
    (3p - 1 per candidate); per step i = 0 .. n-2 and live candidate: four
    dot products over the candidate's two tile columns (8i), K(s,c) and its
    theta-derivative (3p + 3), the new tile rows (4), the updates of v, cov,
    a, b, Q and the W-column dot with z (12), and from step n0-1 on the
    criterion J (24).  The location-level bordering is O(n^3) in total and
    left out."""
    f = M * 3 * p
    for i in range(n - 1):
        live = M - i - 1
        f += live * (8 * i + 3 * p + 19 + (24 if i + 1 >= n0 else 0))
    return f


def workload(name: str, T: int | None):
    import workloads
    if name == "c2_n50":
        w = workloads.c2(n=50)
    elif name == "c2":
        w = workloads.c2(n=64)
    elif name == "c1":
        w = workloads.c1()
    elif name == "c0":
        w = workloads.c0()
    elif name == "c3":
        w = workloads.c3()
    else:
        raise SystemExit(f"unknown workload {name}")
    if T is not None and T < w.T:
        w = w.subset(np.arange(T))
    return w


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2_n50", choices=["c2_n50", "c2", "c1", "c0", "c3", "c4"])
    ap.add_argument("--T", type=int, default=None, help="use only the first T locations")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"],
                    help="ranking tile: fp64, or fp32 / bf16 with the exact FP64 short-list re-score")
    ap.add_argument("--method", default="alc", choices=["alc", "alc2", "mspe"],
                    help="alc: designs at the fixed lengthscale; alc2: the two-stage scheme with local MLEs; "
                         "mspe: greedy designs by the MSPE criterion")
    ap.add_argument("--cpu-sample", type=int, default=2048, help="locations in the CPU oracle sample (0: skip)")
    ap.add_argument("--parity-sample", type=int, default=64, help="sampled locations checked against the oracle")
    ap.add_argument("--graph", default="auto", choices=["auto", "on", "off"],
                    help="run each step as one HIP-graph launch of a fixed-shape batch (auto: for uneven sizes)")
    ap.add_argument("--burst", type=int, default=256, help="c4: requests per saturating burst (one step)")
    ap.add_argument("--requests", type=int, default=2000, help="c4: requests per offered-load level")
    ap.add_argument("--loads", default="0.5,0.8,0.95", help="c4: offered loads as fractions of saturation")
    ap.add_argument("--budget-gib", type=int, default=32, help="c4: serving HBM budget")
    ap.add_argument("--serve-requests", type=int, default=500,
                    help="requests of the serving leg of the default run (0: skip the leg)")
    ap.add_argument("--serve-load", type=float, default=0.8, help="serving leg: offered load, fraction of saturation")
    ap.add_argument("--serve-burst", type=int, default=128, help="serving leg: requests per saturating burst")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only copy this many bytes device-to-device (calibrates HBM byte counters) and exit")
    args = ap.parse_args()

    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe // 8, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 8}))
        return 0

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(locations are independent, so the multi-GPU form is a partition of the batch).",
              file=sys.stderr)
        return 2

    import torch
    import paper_1303_0383_amd as lagp

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "c4":
        return serve_bench(args, lagp, torch)
    dev = torch.device("cuda:0")
    w = workload(args.workload, args.T)
    prec = {"fp64": lagp.LAGP_PREC_FP64, "fp32": lagp.LAGP_PREC_SCORE_FP32,
            "bf16": lagp.LAGP_PREC_SCORE_BF16}[args.precision]
    D = lagp.Design(w.X, w.y)
    XX = torch.as_tensor(w.XX, device=dev)
    n_per = None if w.n_per is None else torch.as_tensor(w.n_per, device=dev)
    M_per = None if w.ncand_per is None else torch.as_tensor(w.ncand_per, device=dev)
    nmax = int(w.n_per.max()) if w.n_per is not None else w.n
    Mmax = int(w.ncand_per.max()) if w.ncand_per is not None else w.ncand
    T = w.T
    out = lagp.Prediction(mean=torch.empty(T, dtype=torch.float64, device=dev),
                          s2=torch.empty(T, dtype=torch.float64, device=dev),
                          df=torch.empty(T, dtype=torch.int32, device=dev),
                          var=torch.empty(T, dtype=torch.float64, device=dev),
                          sel=torch.empty((T, nmax), dtype=torch.int32, device=dev),
                          status=torch.empty(T, dtype=torch.int8, device=dev))

    alc2 = args.method == "alc2"
    mspe = args.method == "mspe"
    if mspe and (w.n_per is not None or args.precision != "fp64"):
        raise SystemExit("--method mspe runs uniform sizes in FP64")
    # graphs capture fixed-shape batches of the one-stage scheme
    use_graph = not (alc2 or mspe) and (args.graph == "on" or (args.graph == "auto" and w.n_per is not None))
    if alc2:
        import workloads
        tmin, tmax = workloads.mle_range(w.X)
        out.theta1 = torch.empty(T, dtype=torch.float64, device=dev)
        out.theta2 = torch.empty(T, dtype=torch.float64, device=dev)

    def eager_step():
        if mspe:
            D.predict_mspe(XX, w.n0, nmax, Mmax, w.d, w.g, out=out)
        elif alc2:
            D.predict_alc2(XX, w.n0, nmax, Mmax, w.d, w.g, tmin, tmax, n_per=n_per, ncand_per=M_per,
                           precision=prec, out=out)
        else:
            D.predict(XX, w.n0, nmax, Mmax, w.d, w.g, n_per=n_per, ncand_per=M_per, precision=prec, out=out)

    if use_graph:
        # The batch plan (buckets, work lists, kernel variants, workspace) is
        # made once, outside the timed region; each step is one graph launch.
        B = lagp.Batch(D, T, w.n0, nmax, Mmax, w.d, w.g, n_per=w.n_per, ncand_per=w.ncand_per, precision=prec)

        def step():
            B.run(XX, out=out, graph=True)
    else:
        step = eager_step

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if not use_graph:
        lagp.lagp_timing_enable(D.handle, True)
        lagp.lagp_phase_times(D.handle)
    step_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        step()
        torch.cuda.synchronize()
        step_ms.append(1e3 * (time.perf_counter() - ts))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if use_graph:
        # Per-phase device time from one eager pass with HIP events on the
        # launch stream (graph launches carry no events inside).
        lagp.lagp_timing_enable(D.handle, True)
        lagp.lagp_phase_times(D.handle)
        eager_step()
        torch.cuda.synchronize()
        phase, launches = lagp.lagp_phase_times(D.handle)
        lagp.lagp_timing_enable(D.handle, False)
        phase = {k: v * args.steps for k, v in phase.items()}
        launches *= args.steps
    else:
        phase, launches = lagp.lagp_phase_times(D.handle)
        lagp.lagp_timing_enable(D.handle, False)
    des_ms = phase["design"]

    value = T * args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps

    # Roofline of the dominant kernel (greedy design): algorithmic FP64 flops per launch
    # over its average launch duration from HIP events on the launch stream.
    if w.n_per is not None:
        flops = sum(design_flops(int(a), int(b), w.p, w.n0) for a, b in zip(w.n_per, w.ncand_per))
        exps = sum(design_exps(int(a), int(b)) for a, b in zip(w.n_per, w.ncand_per))
    else:
        flops = T * design_flops(w.n, w.ncand, w.p, w.n0)
        exps = T * design_exps(w.n, w.ncand)
    passes = 2 if alc2 else 1   # design passes per step
    flops, exps = passes * flops, passes * exps
    if mspe:
        flops = T * mspe_flops(w.n, w.ncand, w.p, w.n0)
    launches_per_step = max(1, launches // args.steps)
    per_launch_flops = flops / launches_per_step
    avg_launch_s = des_ms / max(launches, 1) / 1e3
    if w.n_per is not None:
        alg_bytes = sum(design_alg_bytes(int(a), int(b), w.p) for a, b in zip(w.n_per, w.ncand_per))
    else:
        alg_bytes = T * design_alg_bytes(w.n, w.ncand, w.p)
    kname = "mspe_kernel" if mspe else "design_kernel"
    # counter files hold the one-stage kernel's traffic for a workload and precision
    tag = args.workload + ("" if args.precision == "fp64" else "_" + args.precision)
    traffic = read_traffic(kname, tag) if not alc2 else None
    roofline = roofline_entry(kname, per_launch_flops, passes * alg_bytes / launches_per_step, traffic, avg_launch_s)
    roofline.update(launches_per_step=launches_per_step, exps_per_launch=exps / launches_per_step,
                    exp_rate_G_per_s=round(exps / launches_per_step / avg_launch_s / 1e9, 2))
    # Each kernel's fraction of its roof: the kNN (one distance per
    # location-design pair, FP64 flops; its scans run about two full passes),
    # the design kernel (above) and, in the two-stage scheme, the likelihood kernel.
    kernels = {"design": {k: roofline[k] for k in ("bound", "frac", "flop_frac", "alg_byte_frac",
                                                    "traffic_frac_of_hbm_peak")}}
    knn_ms = phase["knn"] / args.steps
    if knn_ms > 0:
        kf = knn_alg_flops(T, w.N, w.p) / (knn_ms / 1e3) / 1e12
        kernels["knn"] = {"bound": "alu", "ms_per_step": round(knn_ms, 3), "achieved_TFLOPs": round(kf, 3),
                          "frac": round(kf / FP64_PEAK_TFLOPS, 4), "alg_flops": knn_alg_flops(T, w.N, w.p)}

    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "locations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f64+f32-tile", "bf16": "f64+bf16-tile"}[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload, "method": args.method, "N": w.N, "p": w.p, "T": T, "n0": w.n0,
                   "n": nmax, "ncand": Mmax, "d": w.d, "g": w.g, "uneven": w.n_per is not None, "graph": use_graph},
        "phase_ms_per_step": {k: round(v / args.steps, 3) for k, v in phase.items() if v > 0 or k in ("knn", "design")},
        "step_ms_p50": round(float(np.percentile(step_ms, 50)), 3),
        "step_ms_p99": round(float(np.percentile(step_ms, 99)), 3),
        "roofline": roofline,
        "kernels": kernels,
    }

    if alc2:
        # Newton iterates of the two likelihood passes, measured outside the
        # timed region by repeating them through lagp_mle (same kernel, same
        # designs and starting values): the MLE from d0 of the designs at d0,
        # and the MLE from theta1 of the second designs.
        first = D.predict(XX, w.n0, nmax, Mmax, w.d, w.g, n_per=n_per, ncand_per=M_per, precision=prec)
        _, it1, _ = D.mle(first.sel, w.d, w.g, tmin, tmax, n_per=n_per)
        _, it2, _ = D.mle(out.sel, out.theta1, w.g, tmin, tmax, n_per=n_per)
        torch.cuda.synchronize()
        n_it = int(it1.sum().item()) + int(it2.sum().item())
        mle_ms = phase.get("mle", 0.0) / args.steps
        result["mle"] = {"iterates_from_d0": round(float(it1.double().mean().item()), 3),
                         "iterates_from_theta1": round(float(it2.double().mean().item()), 3),
                         "location_iterates_per_step": n_it,
                         "ns_per_location_iterate": round(mle_ms * 1e6 / max(n_it, 1), 2)}
        if mle_ms > 0:
            # iterates by design size: the two passes' designs have the step's sizes
            sizes = w.n_per if w.n_per is not None else np.full(T, w.n)
            per_loc = (it1.cpu().numpy() + it2.cpu().numpy()).astype(np.float64)
            mf = float(np.sum(per_loc * mle_iterate_flops(sizes.astype(np.float64))))
            rate = mf / (mle_ms / 1e3) / 1e12
            kernels["mle"] = {"bound": "alu", "ms_per_step": round(mle_ms, 3), "achieved_TFLOPs": round(rate, 3),
                              "frac": round(rate / FP64_PEAK_TFLOPS, 4), "alg_flops": mf}
        del first

    res = {k: getattr(out, k).cpu().numpy() for k in ("mean", "s2", "df", "var", "sel", "status")}
    rng = np.random.default_rng(20130383)

    # Parity of sampled outputs against the FP64 oracle.
    if args.parity_sample > 0 and args.precision != "fp64":
        # Mixed precision: per-step agreement under replay, sequence identity,
        # mean RMS difference from the FP64 oracle over sd(y), and the FP64
        # prediction from the chosen indices against the oracle's.
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from parity import mixed_metrics
        idx = np.sort(rng.choice(T, min(args.parity_sample, T), replace=False))
        try:
            m = mixed_metrics(w.X, w.y, w.XX, w.n0, w.n, w.ncand, w.d, w.g, res, idx=idx,
                              n_per=w.n_per, M_per=w.ncand_per)
            m = {k: (float(f"{v:.4g}") if isinstance(v, float) else v) for k, v in m.items()}
            m["selection_bar_met"] = m["step_agreement"] >= 0.99
            m["mean_rms_bar_met"] = m["mean_rms_over_sd"] <= 1e-4
            m["ok"] = m["selection_bar_met"] and m["prediction_parity"] <= 1e-9
        except AssertionError as e:
            m = {"ok": False, "error": str(e)}
        result["parity"] = {"locations": len(idx), "kind": "mixed", **m}
    elif args.parity_sample > 0 and mspe:
        # sequences against the oracle's greedy MSPE search; predictions where they agree
        import oracle
        idx = np.sort(rng.choice(T, min(args.parity_sample, T), replace=False))
        same = 0
        worst = 0.0
        for t in idx:
            rc, so, o, _ = oracle.mspe_local(w.X, w.y, w.XX[t], w.n0, w.n, w.ncand, w.d, w.g)
            if np.array_equal(so, res["sel"][t, :w.n]):
                same += 1
                worst = max(worst, abs(res["mean"][t] - o[0]) / max(abs(o[0]), float(np.std(w.y))),
                            abs(res["s2"][t] - o[1]) / o[1])
        result["parity"] = {"locations": len(idx), "kind": "mspe", "identical": same,
                            "worst_rel": float(f"{worst:.3e}"), "ok": bool(same == len(idx) and worst <= 1e-9)}
    elif args.parity_sample > 0 and alc2:
        # Stage by stage on a sample, each stage fed the GPU's previous one:
        # the second designs against the oracle's at the GPU's theta1, theta2
        # against the oracle's MLE of those designs, the prediction against
        # the oracle's from them at the GPU's theta2.
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        import oracle
        from parity import compare
        idx = np.sort(rng.choice(T, min(args.parity_sample, T), replace=False))
        th1, th2 = out.theta1.cpu().numpy(), out.theta2.cpu().numpy()
        try:
            worst_th = worst_mu = 0.0
            for t in idx:
                nt = int(w.n_per[t]) if w.n_per is not None else w.n
                s2_ = res["sel"][t, :nt]
                rc, tho, _ = oracle.mle(w.X, w.y, s2_, th1[t], w.g, tmin, tmax)
                worst_th = max(worst_th, abs(th2[t] - tho) / tho)
                rc, o = oracle.predict(w.X, w.y, w.XX[t], s2_, th2[t], w.g)
                worst_mu = max(worst_mu, abs(res["mean"][t] - o[0]) / max(abs(o[0]), float(np.std(w.y))))
            ti = torch.as_tensor(idx, device=dev)
            nps = None if w.n_per is None else w.n_per[idx]
            mps = None if w.ncand_per is None else w.ncand_per[idx]
            d1 = D.predict(XX[ti], w.n0, nmax, Mmax, w.d, w.g, d_per=out.theta1[ti],
                           n_per=None if nps is None else n_per[ti], ncand_per=None if mps is None else M_per[ti])
            torch.cuda.synchronize()
            r1 = {k: getattr(d1, k).cpu().numpy() for k in ("mean", "s2", "df", "var", "sel", "status")}
            nts = [int(nps[i]) if nps is not None else w.n for i in range(len(idx))]
            same = all(np.array_equal(r1["sel"][i, :nts[i]], res["sel"][t, :nts[i]]) for i, t in enumerate(idx))
            summ = compare(w.X, w.y, w.XX[idx], w.n0, w.n, w.ncand, th1[idx], w.g, r1, n_per=nps, M_per=mps)
            ok = bool(same and worst_th <= 1e-8 and worst_mu <= 1e-9)
            result["parity"] = {"locations": len(idx), "ok": ok, "kind": "stagewise",
                                "theta2_rel": float(f"{worst_th:.3e}"), "mean_rel": float(f"{worst_mu:.3e}"),
                                "second_designs": {k: (float(f"{v:.3e}") if isinstance(v, float) else v)
                                                   for k, v in summ.items()}}
        except AssertionError as e:
            result["parity"] = {"locations": len(idx), "ok": False, "error": str(e)}
    elif args.parity_sample > 0:
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from parity import compare
        idx = np.sort(rng.choice(T, min(args.parity_sample, T), replace=False))
        try:
            summ = compare(w.X, w.y, w.XX, w.n0, w.n, w.ncand, w.d, w.g, res, idx=idx,
                           n_per=w.n_per, M_per=w.ncand_per)
            result["parity"] = {"locations": len(idx), "ok": True,
                                **{k: (float(f"{v:.3e}") if isinstance(v, float) else v) for k, v in summ.items()}}
        except AssertionError as e:
            result["parity"] = {"locations": len(idx), "ok": False, "error": str(e)}

    # CPU baseline: the oracle, as it stands, on a bounded sample of the same workload.
    if args.cpu_sample > 0:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        idx = np.sort(rng.choice(T, min(args.cpu_sample, T), replace=False))
        sub = w.subset(idx)
        tc = time.perf_counter()
        if mspe:
            from concurrent.futures import ThreadPoolExecutor
            with ThreadPoolExecutor(threads) as ex:
                list(ex.map(lambda t: oracle.mspe_local(sub.X, sub.y, sub.XX[t], sub.n0, sub.n, sub.ncand, sub.d,
                                                        sub.g), range(len(idx))))
        elif alc2:
            # the oracle's two-stage function is per location: a thread pool over
            # the sample (the ctypes calls release the interpreter lock)
            from concurrent.futures import ThreadPoolExecutor
            with ThreadPoolExecutor(threads) as ex:
                list(ex.map(lambda t: oracle.alc2(sub.X, sub.y, sub.XX[t], sub.n0,
                                                  int(sub.n_per[t]) if sub.n_per is not None else sub.n,
                                                  int(sub.ncand_per[t]) if sub.ncand_per is not None else sub.ncand,
                                                  sub.d, sub.g, tmin, tmax), range(len(idx))))
        else:
            oracle.batch(sub.X, sub.y, sub.XX, sub.n0, sub.n, sub.ncand, sub.d, sub.g, n_per=sub.n_per,
                         M_per=sub.ncand_per, threads=threads)
        cpu_s = time.perf_counter() - tc
        result["cpu_baseline"] = {"value": round(len(idx) / cpu_s, 2), "unit": "locations/s", "cores": threads,
                                  "kind": "oracle", "cpu_model": cpu_model(),
                                  "sample": f"{len(idx)} seeded locations of the same workload, {cpu_s:.1f} s, "
                                            f"OpenMP over locations"}
        if not (mspe or alc2):
            # single-thread rate on a smaller sample of the same locations
            k1 = max(4, len(idx) // (2 * max(threads, 1)))
            sub1 = w.subset(idx[:k1])
            tc = time.perf_counter()
            oracle.batch(sub1.X, sub1.y, sub1.XX, sub1.n0, sub1.n, sub1.ncand, sub1.d, sub1.g, n_per=sub1.n_per,
                         M_per=sub1.ncand_per, threads=1)
            one_s = time.perf_counter() - tc
            result["cpu_baseline"]["single_thread"] = {"value": round(k1 / one_s, 2), "unit": "locations/s",
                                                       "sample": f"first {k1} locations of that sample, {one_s:.1f} s"}
    if args.serve_requests > 0 and args.workload == "c2_n50" and args.method == "alc":
        # request latency beside throughput: a short open-loop serving leg
        result["serving"] = serving_leg(lagp, args)
    print(json.dumps(result), flush=True)
    return 0


def _saturate(S, prm, burst, steps, warmup):
    """Locations/s of the server with `burst` submitted at once and drained,
    over `steps` timed bursts after `warmup` untimed ones."""
    def step():
        ts = [S.submit(r.XX, prm["n0"], r.n, r.ncand, prm["d"], prm["g"], precision=prm.get("precision", 0)) for r in burst]
        for t in ts:
            S.wait(t)

    for _ in range(warmup):
        step()
    step_ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        step()
        step_ms.append(1e3 * (time.perf_counter() - ts))
    elapsed = time.perf_counter() - t0
    return sum(len(r.XX) for r in burst) * steps / elapsed, elapsed, step_ms


def _open_loop(S, lagp, prm, reqs, rate):
    """Submit `reqs` at their Poisson arrival times (open loop); latency of a
    request is its completion minus its scheduled arrival."""
    mono = lagp.lagp_monotonic_seconds
    b0 = S.stats()
    start = mono() + 0.05
    tickets = []
    for r in reqs:
        delay = start + r.arrival_s - mono()
        if delay > 0:
            time.sleep(delay)
        tickets.append(S.submit(r.XX, prm["n0"], r.n, r.ncand, prm["d"], prm["g"], precision=prm.get("precision", 0)))
    lat, last = [], start
    for r, t in zip(reqs, tickets):
        o = S.wait(t)
        lat.append(o.done - (start + r.arrival_s))
        last = max(last, o.done)
    b1 = S.stats()
    locs = sum(len(r.XX) for r in reqs)
    return {"offered_req_per_s": round(rate, 1), "requests": len(reqs),
            "achieved_locations_per_s": round(locs / (last - start), 1),
            "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 2),
            "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 2),
            "pieces": b1[0] - b0[0], "mean_piece_locations": round((b1[1] - b0[1]) / max(1, b1[0] - b0[0]), 1)}


C4_MEAN_REQUEST = 256.5   # mean locations per serving request (uniform on 1..512)


def serving_leg(lagp, args) -> dict:
    """The default run's serving leg on the 4-D serving workload (N = 10^6):
    saturation from bursts of --serve-burst requests, then --serve-requests
    Poisson arrivals at --serve-load of saturation, FP64, open loop."""
    import workloads
    prm = workloads.C4_PARAMS
    X, y, _ = workloads.c4_design()
    D = lagp.Design(X, y)
    S = lagp.Server(D, args.budget_gib << 30)
    sat, _, _ = _saturate(S, prm, workloads.c4_requests(args.serve_burst, 1.0), steps=1, warmup=1)
    rate = args.serve_load * sat / C4_MEAN_REQUEST
    level = _open_loop(S, lagp, prm, workloads.c4_requests(args.serve_requests, rate), rate)
    S.close()
    D.close()
    return {"workload": "c4", "N": len(X), "p": 4, "dtype": "f64", "budget_gib": args.budget_gib,
            "saturation_locations_per_s": round(sat, 1), "load": args.serve_load, **level}


def serve_bench(args, lagp, torch) -> int:
    """Serving workload: N = 10^6 design points in [0,1]^4; requests of
    1..512 locations with n in {32, 50, 64, 100} and N' in [1000, 4000],
    n0 = 6, d = 0.3, g = 1e-5.  A step is one burst of --burst requests
    submitted at once and drained (value: locations/s at saturation); then
    Poisson arrivals at fractions of that rate give p50/p99 latency
    (completion minus scheduled arrival, open loop)."""
    import workloads
    prec = {"fp64": lagp.LAGP_PREC_FP64, "fp32": lagp.LAGP_PREC_SCORE_FP32,
            "bf16": lagp.LAGP_PREC_SCORE_BF16}[args.precision]
    prm = dict(workloads.C4_PARAMS, precision=prec)
    X, y, _ = workloads.c4_design()
    D = lagp.Design(X, y)
    S = lagp.Server(D, args.budget_gib << 30)
    burst = workloads.c4_requests(args.burst, 1.0)
    burst_locs = sum(len(r.XX) for r in burst)
    sat, elapsed, step_ms = _saturate(S, prm, burst, args.steps, args.warmup)
    levels = {}
    for load in [float(v) for v in args.loads.split(",") if v]:
        rate = load * sat / C4_MEAN_REQUEST
        levels[f"{load:.2f}"] = _open_loop(S, lagp, prm, workloads.c4_requests(args.requests, rate), rate)
        print(f"# load {load:.2f}: {levels[f'{load:.2f}']}", file=sys.stderr, flush=True)
    S.close()

    # Roofline of the design kernel: one eager lagp_predict over the burst's
    # locations (per-location sizes, size buckets), HIP events on its stream.
    XX = np.concatenate([r.XX for r in burst])
    n_per = np.concatenate([np.full(len(r.XX), r.n, np.int32) for r in burst])
    M_per = np.concatenate([np.full(len(r.XX), r.ncand, np.int32) for r in burst])
    dev = torch.device("cuda:0")
    XXd = torch.as_tensor(XX, device=dev)
    npd, mpd = torch.as_tensor(n_per, device=dev), torch.as_tensor(M_per, device=dev)
    D.predict(XXd, prm["n0"], int(n_per.max()), int(M_per.max()), prm["d"], prm["g"], n_per=npd, ncand_per=mpd,
              precision=prec)
    torch.cuda.synchronize()
    lagp.lagp_timing_enable(D.handle, True)
    lagp.lagp_phase_times(D.handle)
    D.predict(XXd, prm["n0"], int(n_per.max()), int(M_per.max()), prm["d"], prm["g"], n_per=npd, ncand_per=mpd,
              precision=prec)
    torch.cuda.synchronize()
    phase, launches = lagp.lagp_phase_times(D.handle)
    knn_ms, des_ms = phase["knn"], phase["design"]
    lagp.lagp_timing_enable(D.handle, False)
    flops = sum(design_flops(int(a), int(b), 4, prm["n0"]) for a, b in zip(n_per, M_per))
    alg = sum(design_alg_bytes(int(a), int(b), 4) for a, b in zip(n_per, M_per))
    nl = max(launches, 1)
    roofline = roofline_entry("design_kernel", flops / nl, alg / nl, None, des_ms / nl / 1e3)
    roofline.update(launches_per_step=launches, knn_ms_per_burst=round(knn_ms, 3))

    result = {
        "metric": METRIC, "value": round(sat, 1), "unit": "locations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f64+f32-tile", "bf16": "f64+bf16-tile"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "c4", "N": len(X), "p": 4, "n0": prm["n0"], "d": prm["d"], "g": prm["g"],
                   "burst_requests": args.burst, "burst_locations": burst_locs, "budget_gib": args.budget_gib},
        "step_ms_p50": round(float(np.percentile(step_ms, 50)), 3),
        "step_ms_p99": round(float(np.percentile(step_ms, 99)), 3),
        "serving": levels, "roofline": roofline,
    }
    if args.cpu_sample > 0:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        k = min(args.cpu_sample, 96, len(XX))
        idx = np.sort(np.random.default_rng(20130383).choice(len(XX), k, replace=False))
        tc = time.perf_counter()
        oracle.batch(X, y, XX[idx], prm["n0"], int(n_per.max()), int(M_per.max()), prm["d"], prm["g"],
                     n_per=n_per[idx], M_per=M_per[idx], threads=threads)
        cpu_s = time.perf_counter() - tc
        result["cpu_baseline"] = {"value": round(k / cpu_s, 2), "unit": "locations/s", "cores": threads,
                                  "kind": "oracle", "cpu_model": cpu_model(),
                                  "sample": f"{k} seeded locations of the serving burst, {cpu_s:.1f} s, "
                                            f"OpenMP over locations"}
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
