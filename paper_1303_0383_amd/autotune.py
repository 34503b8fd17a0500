"""Autotuner for the greedy-design kernel.

For every size class the library buckets locations into -- precision mode x
candidate-set class (256 .. 4096) x design-size class (32, 64, 128) -- it
times each kernel variant on the GPU with a seeded batch of locations on the
8-D sinusoid design and writes the fastest to a text table.  A variant is the
tile shape of one location's workgroup: its size (256 or 512 threads, which
sets the candidate slots per thread and the tile rows a lane can hold in
registers), where the candidate coordinates live (LDS or global memory), and
the share of the remaining LDS given to tile rows (100, 50 or 0 %; rows that
fit neither registers nor LDS stream from global memory).  Register rows per
variant are the largest count that compiles without spills.

    <arch> <precision> <ncand class> <n class> <threads> <coords> <lds %>   # timings

The library reads ``tune/table.txt`` next to liblagp.so (or the file named by
LAGP_TUNE_TABLE) and uses an entry when the device architecture matches;
classes without an entry fall back to the traffic model.

    python -m paper_1303_0383_amd.autotune [--out PATH] [--T 2048] [--reps 3]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(_PKG))

MCLASSES = (256, 512, 1024, 2048, 4096)
NCLASSES = (32, 64, 128)


LDS_SHARES = (100, 50, 0)


def variants(mclass: int):
    """(threads, coords, LDS share for tile rows) triples timed for a class."""
    threads = (512,) if mclass > 2048 else (256, 512)
    return [(t, c, l) for t in threads for c in (0, 1) for l in LDS_SHARES]


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(_PKG, "tune", "table.txt"))
    ap.add_argument("--T", type=int, default=2048, help="locations per timing run")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()

    import torch
    import paper_1303_0383_amd as L
    import workloads

    assert torch.cuda.is_available(), "the autotuner runs on the GPU"
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    w = workloads.c2(n=64)
    D = L.Design(w.X, w.y)
    XX = torch.as_tensor(w.XX[: args.T], device="cuda:0")
    lines = [f"# greedy-design kernel variants, {args.T} locations of the 8-D sinusoid design "
             f"(d={w.d}, g={w.g}, n0={w.n0}); best of {args.reps} runs, design-phase ms per variant",
             "# arch precision ncand_class n_class threads coords lds_pct"]
    for prec in (L.LAGP_PREC_FP64, L.LAGP_PREC_SCORE_FP32):
        for mc in MCLASSES:
            for nc in NCLASSES:
                if nc > mc:
                    continue
                times = {}
                for (t, c, l) in variants(mc):
                    L.lagp_design_set_variant_ex(D.handle, t, c, l)
                    D.predict(XX, w.n0, nc, mc, w.d, w.g, precision=prec)   # warm-up
                    torch.cuda.synchronize()
                    best = float("inf")
                    for _ in range(args.reps):
                        L.lagp_timing_enable(D.handle, True)
                        L.lagp_phase_times(D.handle)
                        D.predict(XX, w.n0, nc, mc, w.d, w.g, precision=prec)
                        torch.cuda.synchronize()
                        des_ms = L.lagp_phase_times(D.handle)[0]["design"]
                        L.lagp_timing_enable(D.handle, False)
                        best = min(best, des_ms)
                    times[(t, c, l)] = best
                (t, c, l) = min(times, key=times.get)
                detail = " ".join(f"{tt}/{'lds' if cc else 'glb'}/{ll}={ms:.2f}"
                                  for (tt, cc, ll), ms in sorted(times.items()))
                lines.append(f"{arch} {prec} {mc} {nc} {t} {c} {l}   # {detail}")
                print(lines[-1], flush=True)
    L.lagp_design_set_variant_ex(D.handle, 0, -1, -1)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
