"""Pins of the oracle's k-NN reconstruction (Sec. 5.1.4: the position is
the centroid of the known positions of the k calibration events closest in
the space of normalised sensor signals).

* Distances: the single-precision squared distances the oracle reports
  equal the double-precision squared Euclidean distance between the
  normalised active-sensor signals within the error bound of
  single-precision signals.
* Selection: the neighbours are the k first of a stable library sort of
  the reported distances (NumPy lexsort on (distance, index)), for every
  query, including exact ties (duplicated calibration rows).
* Position: the mean of the neighbours' known positions.
* An event equal to a calibration event is its own nearest neighbour at
  distance 0 (k = 1 returns that position exactly).
* Normalisation: doubling every signal of a query changes nothing;
  passive sensors are ignored whatever they hold.
* Invalid calibration events never become neighbours; invalid queries get
  NaN with the grid's status bits.
"""
import numpy as np
import pytest

import oracle
import workloads as W


@pytest.fixture(scope="module")
def data():
    wl = W.workload(0)
    cs, ct = oracle.make_events(wl.lrf, wl.events, 3000, W.streams(60))
    qs, qt = oracle.make_events(wl.lrf, wl.events, 150, W.streams(61))
    return wl, cs.astype(np.float64), ct["pos"], qs.astype(np.float64), qt["pos"]


def _norm(sig, active):
    s = sig[:, active.astype(bool)]
    return s / s.sum(1, keepdims=True)


def test_distances_selection_and_position(data):
    wl, cs, cpos, qs, qpos = data
    cal = oracle.KnnCal(wl.lrf, cs, cpos)
    k = 12
    r = oracle.knn_reconstruct(cal, k, qs)
    C = _norm(cs, wl.lrf.active)
    Q = _norm(qs, wl.lrf.active)
    for e in range(len(qs)):
        d64 = ((Q[e][None, :] - C) ** 2).sum(1)
        # the reported distances are those of the selected neighbours, to the
        # rounding of single-precision signals: each difference carries an
        # error of about 2^-24 (|q| + |c|), i.e. 2^-23 |q - c| (|q| + |c|)
        # on its square
        bound = 4 * 2.0 ** -24 * (np.abs(Q[e][None, :] - C) * (Q[e][None, :] + C)).sum(1) \
            + 64 * 2.0 ** -24 * d64
        sel = r["idx"][e]
        assert np.all(np.abs(r["dist"][e] - d64[sel]) <= bound[sel])
        # the oracle's own single-precision distances of every calibration
        # event, recomputed here in the same order and precision
        q32 = Q[e].astype(np.float32)
        c32 = C.astype(np.float32)
        dd = np.zeros(len(C), np.float32)
        for a in range(C.shape[1]):
            t = (q32[a] - c32[:, a]).astype(np.float32)
            dd = (dd + (t * t).astype(np.float32)).astype(np.float32)
        order = np.lexsort((np.arange(len(C)), dd))[:k]
        np.testing.assert_array_equal(r["idx"][e], order)
        np.testing.assert_array_equal(r["dist"][e], dd[order])
        np.testing.assert_allclose([r["x"][e], r["y"][e], r["z"][e]], cpos[order].mean(0),
                                   rtol=0, atol=1e-12)


def test_exact_ties_go_to_the_lower_index(data):
    wl, cs, cpos, qs, qpos = data
    cs2 = np.concatenate([cs[:500], cs[:500]])          # every row twice
    pos2 = np.concatenate([cpos[:500], cpos[:500] + 1.0])
    cal = oracle.KnnCal(wl.lrf, cs2, pos2)
    r = oracle.knn_reconstruct(cal, 6, qs[:30])
    for e in range(30):
        idx = r["idx"][e]
        # pairs (i, i + 500) at equal distance: the lower index first
        for j in range(0, 6, 2):
            assert idx[j] < 500 and idx[j + 1] == idx[j] + 500
            assert r["dist"][e, j] == r["dist"][e, j + 1]


def test_calibration_event_is_its_own_neighbour(data):
    wl, cs, cpos, qs, qpos = data
    cal = oracle.KnnCal(wl.lrf, cs, cpos)
    r = oracle.knn_reconstruct(cal, 1, cs[:40])
    assert (r["dist"][:, 0] == 0).all()
    np.testing.assert_array_equal(r["x"], cpos[:40, 0])
    np.testing.assert_array_equal(r["y"], cpos[:40, 1])


def test_normalisation_and_passive_sensors(data):
    wl, cs, cpos, qs, qpos = data
    cal = oracle.KnnCal(wl.lrf, cs, cpos)
    a = oracle.knn_reconstruct(cal, 8, qs)
    b = oracle.knn_reconstruct(cal, 8, 2.0 * qs)
    np.testing.assert_array_equal(a["idx"], b["idx"])
    lrf = W.axial_lrf(wl.lrf.sxy)
    lrf.active = np.ones(19, np.uint8)
    lrf.active[[3, 11]] = 0
    cal_p = oracle.KnnCal(lrf, cs, cpos)
    q = qs.copy()
    q[:, 3] = np.nan
    q[:, 11] = 1e9
    c = oracle.knn_reconstruct(cal_p, 8, qs)
    d = oracle.knn_reconstruct(cal_p, 8, q)
    np.testing.assert_array_equal(c["idx"], d["idx"])
    assert (c["status"] == 0).all()


def test_invalid_events(data):
    wl, cs, cpos, qs, qpos = data
    cs2 = cs[:200].copy()
    cs2[5] = 0.0                  # empty
    cs2[6, 2] = np.nan            # bad
    cal = oracle.KnnCal(wl.lrf, cs2, cpos[:200])
    r = oracle.knn_reconstruct(cal, 199, cs2[:10])
    assert not np.isin([5, 6], r["idx"][r["status"] == 0]).any()
    assert r["status"][5] == 1 and r["status"][6] == 2 and np.isnan(r["x"][[5, 6]]).all()
    ok = r["status"] == 0
    assert (r["idx"][ok, :198] >= 0).all() and (r["idx"][ok, 198] == -1).all()
    assert np.isinf(r["dist"][ok, 198]).all()
