"""Pins of the FP64 LRF-fit oracle (Sec. 6, 6.2, 8) against facts other than
itself: exact recovery of a spline LRF from noiseless events, a brute-force
design matrix built from the C oracle's spline, scale invariances, the event
filter, and convergence of the iterative procedure from a wrong LRF."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import lrf_fit as F


def _events(lrf, rec, n, seed, noiseless):
    sig, truth = oracle.generate(lrf, 0, rec.extent, 0.0, 0.0, rec.e_lo, rec.e_hi, n, seed,
                                 noiseless=noiseless)
    return sig, truth


def test_weights_match_c_oracle_and_sum_to_one():
    for t in (0.0, 0.13, 0.5, 0.77, 1.0):
        np.testing.assert_allclose(F.bspline_weights(t), oracle.basis(t), rtol=0, atol=1e-15)
        assert abs(F.bspline_weights(t).sum() - 1.0) < 1e-15


def test_design_matches_brute_force_lstsq():
    # small case: every row built by evaluating the C oracle's spline with unit
    # coefficient vectors (independent of the weights above), solved by lstsq
    rng = np.random.default_rng(3)
    nb, lo, hi = 6, 0.0, 40.0
    sxy = rng.uniform(-15, 15, (7, 2))
    gain = rng.uniform(0.8, 1.2, 7)
    active = np.ones(7, np.uint8)
    active[4] = 0
    n_ev = 150
    x, y = rng.uniform(-20, 20, n_ev), rng.uniform(-20, 20, n_ev)
    E = rng.uniform(100, 300, n_ev)
    sig = rng.uniform(0, 50, (n_ev, 7))
    rows, rhs = [], []
    for e in range(n_ev):
        for i in range(7):
            r = np.hypot(x[e] - sxy[i, 0], y[e] - sxy[i, 1])
            if not active[i] or r > hi:
                continue
            rows.append([oracle.spline1(np.eye(nb + 2)[j], nb, lo, hi, r)[0]
                         for j in range(nb + 2)])
            rhs.append(sig[e, i] / (E[e] * gain[i]))
    ref = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)[0]
    got = F.fit_axial_shared(sxy, gain, active, sig, x, y, E, np.ones(n_ev, bool), nb, lo, hi,
                             ridge=0.0)
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-12)
    M, v, npairs = F.normal_equations(sxy, gain, active, sig, x, y, E, np.ones(n_ev, bool), nb,
                                      lo, hi)
    A = np.array(rows)
    np.testing.assert_allclose(M, A.T @ A, rtol=1e-12, atol=1e-12)
    assert npairs == len(rows)


def test_noiseless_events_recover_the_spline_exactly():
    # a spline LRF is inside the fitted family: least squares returns it
    lrf, rec = W.mixed_geometries()[1]          # 61 sensors: distances cover [0, 150]
    sig, truth = _events(lrf, rec, 4000, 21, noiseless=True)
    use = np.ones(len(sig), bool)
    # the generator spreads E_tot over the sensors: the LRF scale is E_tot / S
    S = oracle.lrf_values(lrf, truth[:, :3]) @ np.asarray(lrf.gain, np.float64)
    c = F.fit_axial_shared(lrf.sxy, lrf.gain, lrf.active, sig, truth[:, 0], truth[:, 1],
                           truth[:, 3] / S, use, lrf.nb[0], lrf.lo[0], lrf.hi[0], ridge=0.0)
    ref = np.asarray(lrf.coef).reshape(-1)
    assert np.max(np.abs(c - ref)) < 1e-9 * np.max(np.abs(ref))


def test_gain_and_signal_scale_invariances():
    lrf, rec = W.mixed_geometries()[0]
    sig, truth = _events(lrf, rec, 2000, 22, noiseless=False)
    use = np.ones(len(sig), bool)
    args = (truth[:, 0], truth[:, 1], truth[:, 3], use, lrf.nb[0], lrf.lo[0], lrf.hi[0])
    c0 = F.fit_axial_shared(lrf.sxy, lrf.gain, lrf.active, sig, *args)
    # sensor 5 twice as sensitive and its gain doubled: same LRF
    g2 = np.array(lrf.gain, np.float64).copy()
    g2[5] *= 2.0
    s2 = sig.copy()
    s2[:, 5] *= 2.0
    c1 = F.fit_axial_shared(lrf.sxy, g2, lrf.active, s2, *args)
    np.testing.assert_allclose(c1, c0, rtol=1e-10, atol=1e-14)
    # every signal doubled: LRF doubled
    c2 = F.fit_axial_shared(lrf.sxy, lrf.gain, lrf.active, 2.0 * sig, *args)
    np.testing.assert_allclose(c2, 2.0 * c0, rtol=1e-10, atol=1e-14)


def test_event_filter():
    E = np.array([100.0, np.nan, 50.0, 80.0, -1.0, 70.0])
    st = np.array([0, 0, 8, 0, 0, 0])
    chi2 = np.array([10.0, 1.0, 1.0, 90.0, 1.0, 30.0])
    ndf = np.array([15, 15, 15, 15, 15, 0])
    got = F.event_mask(E, st, chi2, ndf, chi2ndf_max=2.0)
    assert got.tolist() == [True, False, False, False, False, False]
    assert F.event_mask(E, st).tolist() == [True, False, False, True, False, True]


def test_iterations_converge_from_a_wrong_lrf():
    # Sec. 8: reconstruct with the current LRF, refit from the reconstructed
    # positions and energies, repeat; start from an LRF made for a source
    # 13 mm (instead of 10 mm) above the sensors.  The LRF scale is
    # degenerate with the event energy, so shapes are compared after the
    # least-squares optimal scaling.
    true_lrf, rec = W.mixed_geometries()[1]
    wrong = W.axial_lrf(true_lrf.sxy, h=13.0)
    grid = W.workload(3).grid
    sig, truth = _events(true_lrf, rec, 1500, 23, noiseless=True)
    r = np.linspace(0.0, 100.0, 201)
    ref = oracle.spline1(np.asarray(true_lrf.coef).reshape(-1), true_lrf.nb[0], 0.0, 150.0, r)
    cur, shape, pos = wrong, [], []
    for _ in range(3):
        c = np.asarray(cur.coef).reshape(-1)
        Lc = oracle.spline1(c, cur.nb[0], 0.0, 150.0, r)
        k = (Lc @ ref) / (Lc @ Lc)
        shape.append(np.sqrt(np.mean((k * Lc - ref) ** 2)))
        out = oracle.reconstruct(cur, grid, sig)
        pos.append(np.mean(np.hypot(out["x"] - truth[:, 0], out["y"] - truth[:, 1])))
        use = F.event_mask(out["E"], out["status"])
        c = F.fit_axial_shared(cur.sxy, cur.gain, cur.active, sig, out["x"], out["y"], out["E"],
                               use, cur.nb[0], cur.lo[0], cur.hi[0])
        cur = W.LRFSet(cur.kind, cur.sxy, cur.gain, cur.active, cur.shared, cur.nb, cur.lo,
                       cur.hi, c.reshape(np.asarray(cur.coef).shape))
    assert all(b < a for a, b in zip(pos, pos[1:])), pos
    assert pos[-1] < 0.8 * pos[0], pos
    assert all(b < a for a, b in zip(shape, shape[1:])), shape
