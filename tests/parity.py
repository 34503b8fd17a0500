"""Parity checks of the HIP path against the FP64 CPU oracle.

Tolerances (FP64 mode):
  * selections: the GPU sequence must equal the oracle's, except that a
    choice may differ where the oracle's relative top-2 gap (a1 - a2) / a1 is
    below 1e-8; such locations are replayed through the oracle with the GPU's
    choices and every GPU choice must then lie within 1e-8 (relative) of the
    oracle's largest ALC at that step;
  * mean:  |dmu| / max(|mu_oracle|, sd(y)) <= 1e-9;
  * s2 and var: relative error <= 1e-9.
The oracle's outputs for a replayed sequence are the reference when the
sequences differ.
"""
from __future__ import annotations

import numpy as np

import oracle

GAP_TOL = 1e-8
MEAN_TOL = 1e-9
VAR_TOL = 1e-9


def gpu_predict(design, XX, n0, n, M, d, g, n_per=None, M_per=None, precision=0):
    import torch
    dev = torch.device("cuda:0")
    XXd = torch.as_tensor(np.ascontiguousarray(XX), dtype=torch.float64, device=dev)
    npd = None if n_per is None else torch.as_tensor(np.asarray(n_per, np.int32), device=dev)
    mpd = None if M_per is None else torch.as_tensor(np.asarray(M_per, np.int32), device=dev)
    out = design.predict(XXd, n0, n, M, d, g, n_per=npd, ncand_per=mpd, precision=precision)
    torch.cuda.synchronize()
    return {k: getattr(out, k).cpu().numpy() for k in ("mean", "s2", "df", "var", "sel", "status")}


def compare(X, y, XX, n0, n, M, d, g, res, idx=None, n_per=None, M_per=None):
    """Compare GPU results `res` with the oracle at locations `idx` (default all);
    d is one lengthscale or one per location.

    Returns a summary dict; raises AssertionError on a parity failure."""
    T = XX.shape[0]
    idx = range(T) if idx is None else idx
    sdy = float(np.std(y))
    identical = replayed = 0
    worst = {"mean": 0.0, "s2": 0.0, "var": 0.0, "shortfall": 0.0}
    for t in idx:
        nt = int(n_per[t]) if n_per is not None else n
        mt = int(M_per[t]) if M_per is not None else M
        dt = float(d[t]) if np.ndim(d) else d      # per-location lengthscale
        rc, s_o, o, diag = oracle.local(X, y, XX[t], n0, nt, mt, dt, g)
        s_g = res["sel"][t, :nt]
        if rc == oracle.NOTPD:
            assert res["status"][t] == 1, f"location {t}: oracle NOTPD, GPU status {res['status'][t]}"
            assert np.isnan(res["mean"][t])
            continue
        assert res["status"][t] == 0, f"location {t}: GPU status {res['status'][t]}"
        assert int(res["df"][t]) == nt
        if np.array_equal(s_g, s_o):
            identical += 1
            ref = o
        else:
            k = int(np.argmax(s_g != s_o))
            gap = (diag[k, 0] - diag[k, 1]) / diag[k, 0] if diag[k, 0] > 0 else 0.0
            assert gap < GAP_TOL, f"location {t}: selections differ at step {k} with gap {gap:.3e}"
            rc2, s_r, o_r, diag_r = oracle.local(X, y, XX[t], n0, nt, mt, dt, g, replay=s_g)
            assert rc2 == 0
            a1, ach = diag_r[n0:, 0], diag_r[n0:, 2]
            short = np.max((a1 - ach) / np.where(a1 > 0, a1, 1.0)) if len(a1) else 0.0
            assert short <= GAP_TOL, f"location {t}: replay shortfall {short:.3e}"
            worst["shortfall"] = max(worst["shortfall"], float(short))
            replayed += 1
            ref = o_r
        em = abs(res["mean"][t] - ref[0]) / max(abs(ref[0]), sdy)
        es = abs(res["s2"][t] - ref[1]) / ref[1]
        worst["mean"] = max(worst["mean"], em)
        worst["s2"] = max(worst["s2"], es)
        if nt > 2:
            ev = abs(res["var"][t] - ref[2]) / ref[2]
            worst["var"] = max(worst["var"], ev)
        assert em <= MEAN_TOL, f"location {t}: mean rel err {em:.3e}"
        assert es <= VAR_TOL, f"location {t}: s2 rel err {es:.3e}"
        if nt > 2:
            assert ev <= VAR_TOL, f"location {t}: var rel err {ev:.3e}"
    worst.update(identical=identical, replayed=replayed)
    return worst


def mixed_metrics(X, y, XX, n0, n, M, d, g, res, idx=None, n_per=None, M_per=None):
    """Mixed-precision quality against the FP64 oracle.

    * step agreement: the oracle replays the GPU's choices; a greedy step
      agrees when the GPU's choice is the oracle's argmax within a relative
      gap of 1e-8 (counted over all greedy steps of all locations);
    * sequence agreement: fraction of locations whose whole sequence equals
      the oracle's own;
    * mean RMS difference from the oracle's own prediction, over sd(y);
    * prediction parity: the GPU's FP64 prediction from its own selections
      against the oracle's prediction from the same selections."""
    T = XX.shape[0]
    idx = list(range(T)) if idx is None else list(idx)
    steps = agree = same_seq = 0
    dmu = []
    worst_pred = 0.0
    sdy = float(np.std(y))
    notpd = 0
    for t in idx:
        nt = int(n_per[t]) if n_per is not None else n
        mt = int(M_per[t]) if M_per is not None else M
        rc, s_o, o, _ = oracle.local(X, y, XX[t], n0, nt, mt, d, g)
        if res["status"][t] != 0:
            assert rc == oracle.NOTPD, f"location {t}: GPU NOTPD where the FP64 oracle succeeds"
            notpd += 1
            continue
        s_g = res["sel"][t, :nt]
        rc2, _, o_r, diag = oracle.local(X, y, XX[t], n0, nt, mt, d, g, replay=s_g)
        a1, ach = diag[n0:, 0], diag[n0:, 2]
        ok = (a1 - ach) <= GAP_TOL * np.where(a1 > 0, a1, 1.0)
        steps += len(ok)
        agree += int(ok.sum())
        same_seq += int(np.array_equal(s_g, s_o))
        dmu.append(res["mean"][t] - o[0])
        worst_pred = max(worst_pred, abs(res["mean"][t] - o_r[0]) / max(abs(o_r[0]), sdy),
                         abs(res["s2"][t] - o_r[1]) / o_r[1])
    return {"step_agreement": agree / max(steps, 1), "sequence_agreement": same_seq / max(len(idx), 1),
            "mean_rms_over_sd": float(np.sqrt(np.mean(np.square(dmu)))) / sdy, "prediction_parity": worst_pred,
            "notpd": notpd}
