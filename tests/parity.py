"""Shared helpers for GPU-vs-oracle parity tests (no method arithmetic here:
only comparisons and bookkeeping)."""
from __future__ import annotations

import numpy as np

POS_TOL = 1e-3        # mm, per axis
REL_TOL = 1e-5        # on lnL (scale max(|lnL|, N)) and chi2 (scale max(chi2, ndf))


def to_np(out):
    return {k: v.detach().cpu().numpy() for k, v in out.items()}


def compare(ref, gpu, signals, stat=0, three_d=False):
    """Element-wise comparison of one batch (status bits compared whole,
    TIE included).  Returns a dict with the match mask and mismatch classes:
    'tie' when the oracle's gap at the first iteration where the two paths
    diverge is within REL_TOL of the scale, 'other' otherwise."""
    n = len(ref["x"])
    sg = np.asarray(signals, np.float64)
    N = np.where(np.isfinite(sg), sg, 0.0).sum(1)   # passive columns may hold NaN
    st_ref = ref["status"]
    st_gpu = gpu["status"]
    bad = (st_ref & 7) != 0
    ok = st_ref == st_gpu
    with np.errstate(invalid="ignore"):
        dpos = np.maximum(np.abs(gpu["x"] - ref["x"]), np.abs(gpu["y"] - ref["y"]))
        if three_d:
            dpos = np.maximum(dpos, np.abs(gpu["z"] - ref["z"]))
        pos_ok = dpos <= POS_TOL
        l_ok = np.abs(gpu["lnl"] - ref["lnl"]) <= REL_TOL * np.maximum(np.abs(ref["lnl"]), N)
        c_ok = np.abs(gpu["chi2"] - ref["chi2"]) <= REL_TOL * np.maximum(
            np.abs(ref["chi2"]), np.maximum(ref["ndf"], 1))
        e_ok = np.abs(gpu["E"] - ref["E"]) <= 1e-5 * np.abs(ref["E"])
    good = pos_ok & l_ok & c_ok & e_ok
    nan_ok = np.isnan(gpu["x"]) & np.isnan(gpu["E"]) & np.isnan(gpu["lnl"])
    # no valid point at the end (e.g. a search that never entered the LRF
    # domain): position as the oracle's, energy and statistics NaN on both
    none_ok = pos_ok & np.isnan(gpu["E"]) & np.isnan(gpu["lnl"]) & np.isnan(gpu["chi2"])
    none = ~bad & np.isnan(ref["E"])
    ok &= np.where(bad, nan_ok, np.where(none, none_ok, good))
    ok &= gpu["ndf"] == ref["ndf"]
    cls = {"tie": 0, "other": 0}
    first_div = np.full(n, -1)
    if "path" in gpu:
        for e in np.where(~ok)[0]:
            d = np.where(gpu["path"][e] != ref["path"][e])[0]
            if len(d):
                k = d[0]
                first_div[e] = k
                scale = max(abs(ref["lnl"][e]), N[e]) if stat == 0 else max(ref["chi2"][e],
                                                                             ref["ndf"][e])
                if ref["gaps"][e, k] <= REL_TOL * scale:
                    cls["tie"] += 1
                    continue
            cls["other"] += 1
    return {"ok": ok, "frac": ok.mean() if n else 1.0, "classes": cls, "first_div": first_div,
            "dpos": dpos}


def summary(res):
    bad = np.where(~res["ok"])[0]
    return (f"match {res['frac'] * 100:.3f}% ({len(bad)} mismatches: {res['classes']}); "
            f"first bad {bad[:8].tolist()}")
