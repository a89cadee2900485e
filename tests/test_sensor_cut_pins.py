"""Pins of the oracle's per-event sensor cuts (Sec. 5.1.2: sensors with a
signal below a threshold, or farther than a distance from the start
position, are ignored).  Pinned by equivalence: an event reconstructed with
a cut equals the same event reconstructed on a detector where exactly the
cut sensors are passive (start positions chosen so that they do not depend
on the sensor set)."""
import dataclasses

import numpy as np

import oracle
import workloads as W


def _passive(lrf, keep):
    return dataclasses.replace(lrf, active=(np.asarray(lrf.active, bool) & keep).astype(np.uint8))


def _same(a, b, e):
    for k in ("x", "y", "z", "E", "lnl", "chi2"):
        np.testing.assert_array_equal(a[k][e], b[k][0], err_msg=k)
    assert a["ndf"][e] == b["ndf"][0] and a["status"][e] == b["status"][0]
    np.testing.assert_array_equal(a["path"][e], b["path"][0])


def test_signal_cut_equals_passive_sensors():
    wl = W.workload(0)
    sig, _ = oracle.make_events(wl.lrf, wl.events, 40, W.streams(900))
    # strongest-sensor start: the strongest sensor survives the cut, so the
    # start is the same with and without the other sensors
    g = dataclasses.replace(wl.grid, start=1, cut_signal=3.0)
    got = oracle.reconstruct(wl.lrf, g, sig)
    g0 = dataclasses.replace(wl.grid, start=1)
    for e in range(len(sig)):
        keep = sig[e] >= 3.0
        ref = oracle.reconstruct(_passive(wl.lrf, keep), g0, sig[e:e + 1])
        _same(got, ref, e)
        assert got["ndf"][e] == int(keep.sum()) - 3


def test_distance_cut_equals_passive_sensors():
    lrf, rec = W.mixed_geometries()[1]
    grid = W.workload(3).grid
    sig, truth = oracle.generate(lrf, 0, rec.extent, 0.0, 0.0, rec.e_lo, rec.e_hi, 30, 61)
    seeds = np.zeros((30, 4))
    seeds[:, :2] = truth[:, :2] + 3.0
    g = dataclasses.replace(grid, start=2, cut_distance=70.0)
    got = oracle.reconstruct(lrf, g, sig, seeds=seeds)
    g0 = dataclasses.replace(grid, start=2)
    for e in range(len(sig)):
        keep = np.hypot(lrf.sxy[:, 0] - seeds[e, 0], lrf.sxy[:, 1] - seeds[e, 1]) <= 70.0
        ref = oracle.reconstruct(_passive(lrf, keep), g0, sig[e:e + 1], seeds=seeds[e:e + 1])
        _same(got, ref, e)


def test_cut_statuses():
    wl = W.workload(0)
    sig, _ = oracle.make_events(wl.lrf, wl.events, 5, W.streams(901))
    # threshold above every signal: no sensor left
    g = dataclasses.replace(wl.grid, cut_signal=1e9)
    out = oracle.reconstruct(wl.lrf, g, sig)
    assert np.all(out["status"] == 4) and np.all(np.isnan(out["x"]))
    assert np.all(out["ndf"] == -3)
    # a distance cut that keeps only sensors without signal: empty
    z = sig.copy()
    z[:, 1:] = 0.0
    z[:, 0] = 50.0
    g = dataclasses.replace(wl.grid, start=2, cut_distance=5.0)
    seeds = np.tile(np.r_[wl.lrf.sxy[3], 0.0, 0.0], (5, 1))
    out = oracle.reconstruct(wl.lrf, g, z, seeds=seeds)
    assert np.all(out["status"] == 1)
