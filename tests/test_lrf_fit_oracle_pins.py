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
    # each status bit alone: the four failure bits drop the event, the tie
    # (32) and fallback (16) bits describe a valid position and keep it
    st = np.array([0, 1, 2, 4, 8, 16, 32, 48, 40])
    got = F.event_mask(np.full(9, 100.0), st)
    assert got.tolist() == [True, False, False, False, False, True, True, True, False]


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


# ---- groups (Sec. 6.2), shifts (Sec. 8), gains within groups (Sec. 6.3)

def _hex61_per_sensor_model(group_of=None, gain_seed=4):
    """The 61-sensor hexagonal detector with a distinct positive spline per
    group of sensors (every sensor its own unless group_of is given)."""
    lrf, rec = W.mixed_geometries()[1]
    n = lrf.n_sensors
    g = np.arange(n) if group_of is None else np.asarray(group_of)
    base = np.asarray(lrf.coef, np.float64).reshape(-1)
    j = np.arange(base.size)
    rng = np.random.default_rng(gain_seed)
    a = rng.uniform(0.3, 1.7, g.max() + 1)
    s = rng.uniform(0.8, 1.2, g.max() + 1)
    tabs = np.stack([base * s[k] * (1.0 + 0.15 * np.cos(j * a[k])) for k in range(g.max() + 1)])
    coef = tabs[g].reshape(n, 1, -1)
    model = W.LRFSet(lrf.kind, lrf.sxy, np.asarray(lrf.gain, np.float64),
                     np.asarray(lrf.active, np.uint8), 0, lrf.nb, lrf.lo, lrf.hi, coef)
    # events out to 175 mm: every sensor sees distances over the whole
    # domain [0, 150], so every table is determined without a ridge
    rec = W.EventRecipe("disc", 175.0, rec.e_lo, rec.e_hi)
    return model, rec, tabs, g


def _noiseless(model, rec, n, seed):
    sig, truth = _events(model, rec, n, seed, noiseless=True)
    S = oracle.lrf_values(model, truth[:, :3]) @ np.asarray(model.gain, np.float64)
    return sig, truth, truth[:, 3] / S


def test_axial_value_equals_c_oracle_lrf():
    model, rec, tabs, g = _hex61_per_sensor_model()
    rng = np.random.default_rng(8)
    pos = np.zeros((300, 3))
    pos[:, :2] = rng.uniform(-160, 160, (300, 2))
    ref = oracle.lrf_values(model, pos)
    for i in (0, 7, 33, 60):
        r = np.hypot(pos[:, 0] - model.sxy[i, 0], pos[:, 1] - model.sxy[i, 1])
        got = F.axial_value(tabs[g[i]], model.nb[0], model.lo[0], model.hi[0], r)
        np.testing.assert_allclose(got, ref[:, i], rtol=1e-13, atol=1e-15)


def test_per_sensor_groups_recover_every_sensors_spline():
    model, rec, tabs, g = _hex61_per_sensor_model()
    sig, truth, E = _noiseless(model, rec, 6000, 31)
    use = np.ones(len(sig), bool)
    args = (model.sxy, model.gain, model.active, sig, truth[:, 0], truth[:, 1], E, use,
            model.nb[0], model.lo[0], model.hi[0])
    coef, pairs = F.fit_axial_grouped(*args, np.arange(model.n_sensors), ridge=0.0)
    err = np.max(np.abs(coef - tabs), axis=1) / np.max(np.abs(tabs), axis=1)
    assert err.max() < 1e-8, err.max()
    assert pairs.sum() == F.normal_equations(*args)[2]
    # one shared table cannot describe them
    shared = F.fit_axial_shared(*args, ridge=0.0)
    assert np.max(np.abs(shared - tabs[0])) > 1e-3 * np.max(np.abs(tabs[0]))


def test_distance_groups_recover_each_rings_spline():
    lrf, rec = W.mixed_geometries()[1]
    d = np.hypot(lrf.sxy[:, 0], lrf.sxy[:, 1])
    _, ring = np.unique(np.round(d, 6), return_inverse=True)
    model, rec, tabs, g = _hex61_per_sensor_model(ring)
    sig, truth, E = _noiseless(model, rec, 5000, 32)
    coef, pairs = F.fit_axial_grouped(model.sxy, model.gain, model.active, sig, truth[:, 0],
                                      truth[:, 1], E, np.ones(len(sig), bool), model.nb[0],
                                      model.lo[0], model.hi[0], ring, ridge=0.0)
    assert coef.shape == tabs.shape and ring.max() >= 5
    assert np.max(np.abs(coef - tabs)) < 1e-8 * np.max(np.abs(tabs))


def test_excluded_sensors_and_empty_groups():
    lrf, rec = W.mixed_geometries()[0]
    sig, truth = _events(lrf, rec, 1500, 33, noiseless=False)
    use = np.ones(len(sig), bool)
    n = lrf.n_sensors
    args = (sig, truth[:, 0], truth[:, 1], truth[:, 3], use, lrf.nb[0], lrf.lo[0], lrf.hi[0])
    groups = np.zeros(n, np.int64)
    groups[[2, 9]] = -1
    groups[5] = 2                                   # group 1 has no member
    coef, pairs = F.fit_axial_grouped(lrf.sxy, lrf.gain, lrf.active, *args, groups)
    act = np.asarray(lrf.active, np.uint8).copy()
    act[[2, 9, 5]] = 0
    ref = F.fit_axial_shared(lrf.sxy, lrf.gain, act, *args)
    np.testing.assert_allclose(coef[0], ref, rtol=1e-12, atol=1e-15)
    assert np.isnan(coef[1]).all() and pairs[1] == 0 and pairs[2] > 0


def test_shift_equals_shifted_positions():
    lrf, rec = W.mixed_geometries()[1]
    sig, truth = _events(lrf, rec, 2000, 34, noiseless=False)
    use = np.ones(len(sig), bool)
    sh = np.random.default_rng(9).normal(0.0, 2.0, (len(sig), 2))
    groups = np.arange(lrf.n_sensors) % 3
    a = F.fit_axial_grouped(lrf.sxy, lrf.gain, lrf.active, sig, truth[:, 0], truth[:, 1],
                            truth[:, 3], use, lrf.nb[0], lrf.lo[0], lrf.hi[0], groups, shift=sh)
    b = F.fit_axial_grouped(lrf.sxy, lrf.gain, lrf.active, sig, truth[:, 0] + sh[:, 0],
                            truth[:, 1] + sh[:, 1], truth[:, 3], use, lrf.nb[0], lrf.lo[0],
                            lrf.hi[0], groups)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    c = F.fit_axial_grouped(lrf.sxy, lrf.gain, lrf.active, sig, truth[:, 0], truth[:, 1],
                            truth[:, 3], use, lrf.nb[0], lrf.lo[0], lrf.hi[0], groups)
    assert np.max(np.abs(a[0] - c[0])) > 0.0


def test_gains_within_groups_recover_true_gains():
    lrf, rec = W.mixed_geometries()[1]
    d = np.hypot(lrf.sxy[:, 0], lrf.sxy[:, 1])
    _, ring = np.unique(np.round(d, 6), return_inverse=True)
    model, rec, tabs, g = _hex61_per_sensor_model(ring)
    sig, truth, E = _noiseless(model, rec, 3000, 35)
    gains, pairs = F.fit_gains(model.sxy, model.active, sig, truth[:, 0], truth[:, 1], E,
                               np.ones(len(sig), bool), model.nb[0], model.lo[0], model.hi[0],
                               tabs, ring)
    act = np.asarray(model.active, bool)
    np.testing.assert_allclose(gains[act], np.asarray(model.gain)[act], rtol=1e-11)
    assert (pairs[act] > 0).all()
    # a table scaled by k gives gains scaled by 1 / k
    g2, _ = F.fit_gains(model.sxy, model.active, sig, truth[:, 0], truth[:, 1], E,
                        np.ones(len(sig), bool), model.nb[0], model.lo[0], model.hi[0],
                        2.0 * tabs, ring)
    np.testing.assert_allclose(g2[act], 0.5 * gains[act], rtol=1e-13)


# ---- two-dimensional LRFs (r-z and XY)

def test_2d_value_equals_c_oracle_lrf():
    for k, kind in ((2, "rz"), (1, "xy")):
        wl = W.workload(k)
        m = wl.lrf
        rng = np.random.default_rng(20 + k)
        pos = np.zeros((200, 3))
        pos[:, :2] = rng.uniform(-100, 100, (200, 2)) if k == 2 else rng.uniform(-26, 26, (200, 2))
        pos[:, 2] = rng.uniform(-5, 55, 200)
        ref = oracle.lrf_values(m, pos)
        coef = np.asarray(m.coef, np.float64)
        for i in (0, 5, 17):
            t = 0 if m.shared else i
            u, w = (np.hypot(pos[:, 0] - m.sxy[i, 0], pos[:, 1] - m.sxy[i, 1]), pos[:, 2]) \
                if kind == "rz" else (pos[:, 0], pos[:, 1])
            got = F.value_2d(coef[t], m.nb, m.lo, m.hi, u, w)
            np.testing.assert_allclose(got, ref[:, i], rtol=1e-12, atol=1e-15)


def test_2d_design_matches_brute_force_lstsq():
    rng = np.random.default_rng(5)
    # events reach every part of the (r, z) domain: a well-posed system
    nb, lo, hi = (5, 4), (0.0, 0.0), (25.0, 20.0)
    sxy = rng.uniform(-10, 10, (5, 2))
    gain = rng.uniform(0.8, 1.2, 5)
    active = np.ones(5, np.uint8)
    n_ev = 600
    x, y = rng.uniform(-15, 15, n_ev), rng.uniform(-15, 15, n_ev)
    z = rng.uniform(-1, 21, n_ev)
    E = rng.uniform(100, 300, n_ev)
    sig = rng.uniform(0, 50, (n_ev, 5))
    nc = (nb[0] + 2) * (nb[1] + 2)
    rows, rhs = [], []
    for e in range(n_ev):
        for i in range(5):
            r = np.hypot(x[e] - sxy[i, 0], y[e] - sxy[i, 1])
            if not (0.0 <= r <= 25.0 and 0.0 <= z[e] <= 20.0):
                continue
            rows.append([oracle.spline2(np.eye(nc)[j].reshape(nb[1] + 2, nb[0] + 2), nb, lo, hi,
                                        r, z[e])[0] for j in range(nc)])
            rhs.append(sig[e, i] / (E[e] * gain[i]))
    A = np.array(rows)
    use = np.ones(n_ev, bool)
    M, v, npairs = F.normal_equations_2d("rz", sxy, gain, active, sig, x, y, z, E, use, nb, lo, hi)
    np.testing.assert_allclose(M, A.T @ A, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(v, A.T @ np.array(rhs), rtol=1e-12, atol=1e-12)
    assert npairs == len(rows)
    ref = np.linalg.lstsq(A, np.array(rhs), rcond=None)[0]
    got, _ = F.fit_2d_grouped("rz", sxy, gain, active, sig, x, y, z, E, use, nb, lo, hi,
                              np.zeros(5, np.int64), ridge=0.0)
    assert np.linalg.cond(A) < 1e6
    np.testing.assert_allclose(got[0].reshape(-1), ref, rtol=1e-8, atol=1e-10)


def test_rz_shared_fit_recovers_the_lrf_where_events_reach():
    wl = W.workload(2)
    sig, truth = oracle.generate(wl.lrf, 0, wl.events.extent, wl.events.z_lo, wl.events.z_hi,
                                 wl.events.e_lo, wl.events.e_hi, 3000, 41, noiseless=True)
    S = oracle.lrf_values(wl.lrf, truth[:, :3]) @ np.asarray(wl.lrf.gain, np.float64)
    m = wl.lrf
    use = np.ones(len(sig), bool)
    coef, pairs = F.fit_2d_grouped("rz", m.sxy, m.gain, m.active, sig, truth[:, 0], truth[:, 1],
                                   truth[:, 2], truth[:, 3] / S, use, m.nb, m.lo, m.hi,
                                   np.zeros(m.n_sensors, np.int64), ridge=1e-12)
    # the fitted LRF equals the true one wherever the events probe it
    ref = oracle.lrf_values(m, truth[:, :3])
    for i in (0, 9, 30):
        r = np.hypot(truth[:, 0] - m.sxy[i, 0], truth[:, 1] - m.sxy[i, 1])
        got = F.value_2d(coef[0], m.nb, m.lo, m.hi, r, truth[:, 2])
        assert np.max(np.abs(got - ref[:, i])) < 1e-7 * np.max(ref[:, i]), i


def test_xy_individual_fits_recover_each_sensors_lrf():
    wl = W.workload(1)
    m = wl.lrf
    sig, truth = oracle.generate(m, 1, wl.events.extent, 0.0, 0.0, wl.events.e_lo,
                                 wl.events.e_hi, 6000, 42, noiseless=True)
    S = oracle.lrf_values(m, truth[:, :3]) @ np.asarray(m.gain, np.float64)
    use = np.ones(len(sig), bool)
    ind = np.arange(m.n_sensors)
    ind[ind >= 8] = -1                                  # the first row of sensors only
    coef, pairs = F.fit_2d_grouped("xy", m.sxy, m.gain, m.active, sig, truth[:, 0], truth[:, 1],
                                   truth[:, 2], truth[:, 3] / S, use, m.nb, m.lo, m.hi, ind,
                                   ridge=1e-12)
    assert coef.shape[0] == 8 and (pairs > 0).all()
    ref = oracle.lrf_values(m, truth[:, :3])
    for i in range(8):
        got = F.value_2d(coef[i], m.nb, m.lo, m.hi, truth[:, 0], truth[:, 1])
        assert np.max(np.abs(got - ref[:, i])) < 1e-7 * np.max(ref[:, i]), i


# ---- composite LRFs (Sec. 6.1.1): axial part + XY residual

def _composite_shared_residual(xy_nb=12):
    sxy = W.hex_array(2, 30.0)
    comp = W.composite_lrf(sxy, xy_nb=xy_nb)
    return W.LRFSet(comp.kind, comp.sxy, comp.gain, comp.active, 1, comp.nb, comp.lo, comp.hi,
                    comp.coef, xy_nb=comp.xy_nb, xy_lo=comp.xy_lo, xy_hi=comp.xy_hi,
                    xy_coef=np.asarray(comp.xy_coef)[9:10], xy_shared=1)


def test_composite_value_equals_c_oracle_lrf():
    lrf = W.composite_lrf(W.hex_array(2, 30.0))
    rng = np.random.default_rng(4)
    pos = np.zeros((500, 3))
    pos[:, :2] = rng.uniform(-110.0, 110.0, (500, 2))
    ref = oracle.lrf_values(lrf, pos)
    ax = np.asarray(lrf.coef).reshape(-1)
    for i, (X, Y) in enumerate(lrf.sxy):
        r = np.hypot(pos[:, 0] - X, pos[:, 1] - Y)
        got = F.composite_value(ax, lrf.nb[0], lrf.lo[0], lrf.hi[0], lrf.xy_coef[i], lrf.xy_nb,
                                lrf.xy_lo, lrf.xy_hi, r, pos[:, 0], pos[:, 1])
        np.testing.assert_allclose(got, ref[:, i], rtol=1e-12, atol=1e-15)


def test_residual_fit_on_the_true_axial_recovers_a_shared_residual():
    # noiseless events of a composite LRF with one residual for all sensors:
    # with the true axial spline subtracted, every estimate is the residual
    # at the event, and the fit returns its table
    lrf = _composite_shared_residual()
    sig, truth = oracle.generate(lrf, 1, 90.0, 0.0, 0.0, 500.0, 2000.0, 3000, 52,
                                 noiseless=True)
    L = oracle.lrf_values(lrf, truth[:, :3])
    ax = np.asarray(lrf.coef).reshape(-1)
    base = (ax, lrf.nb[0], lrf.lo[0], lrf.hi[0])
    for i, (X, Y) in enumerate(lrf.sxy):   # no pair is clamped at 0
        r = np.hypot(truth[:, 0] - X, truth[:, 1] - Y)
        assert (F.axial_spline(*base, r) + F.spline_2d(lrf.xy_coef[0], lrf.xy_nb, lrf.xy_lo,
                                                       lrf.xy_hi, truth[:, 0], truth[:, 1]) > 0).all()
    E = truth[:, 3] / (L @ np.asarray(lrf.gain, np.float64))
    use = np.ones(len(sig), bool)
    res, pairs = F.fit_2d_grouped("xy", lrf.sxy, lrf.gain, lrf.active, sig, truth[:, 0],
                                  truth[:, 1], np.zeros(len(sig)), E, use, lrf.xy_nb, lrf.xy_lo,
                                  lrf.xy_hi, np.zeros(19, np.int64), ridge=1e-12, base=base)
    assert pairs[0] == 19 * len(sig)
    ref = np.asarray(lrf.xy_coef[0])
    np.testing.assert_allclose(res[0], ref, rtol=0, atol=1e-7 * np.abs(ref).max())
    # without the subtraction the fit is not the residual
    off, _ = F.fit_2d_grouped("xy", lrf.sxy, lrf.gain, lrf.active, sig, truth[:, 0], truth[:, 1],
                              np.zeros(len(sig)), E, use, lrf.xy_nb, lrf.xy_lo, lrf.xy_hi,
                              np.zeros(19, np.int64), ridge=1e-12)
    assert np.abs(off[0] - ref).max() > 0.1 * np.abs(ref).max()


def test_two_stage_fit_of_an_axial_truth_leaves_no_residual():
    # purely axial noiseless events: the first stage returns the true axial
    # spline and every per-sensor residual vanishes (to the ridge's pull on
    # the last coefficient, whose support the events barely reach)
    sxy = W.hex_array(2, 30.0)
    lrf = W.axial_lrf(sxy)
    sig, truth = oracle.generate(lrf, 1, 90.0, 0.0, 0.0, 500.0, 2000.0, 2000, 53,
                                 noiseless=True)
    E = truth[:, 3] / (oracle.lrf_values(lrf, truth[:, :3]) @ np.asarray(lrf.gain, np.float64))
    use = np.ones(len(sig), bool)
    ax, res, pairs = F.fit_composite(lrf.sxy, lrf.gain, lrf.active, sig, truth[:, 0], truth[:, 1],
                                     E, use, lrf.nb[0], lrf.lo[0], lrf.hi[0], (8, 8),
                                     (-90.0, -90.0), (90.0, 90.0), np.arange(19), ridge=1e-12)
    true_ax = np.asarray(lrf.coef).reshape(-1)
    np.testing.assert_allclose(ax, true_ax, rtol=0, atol=1e-7 * np.abs(true_ax).max())
    assert (pairs == len(sig)).all()
    assert np.abs(res).max() <= 1e-7 * np.abs(true_ax).max()


# ---- sliced LRFs (Sec. 6.1.2): XY tables on z planes

def test_slice_windows_cover_every_depth_once():
    w = F.slice_windows(6, 0.0, 50.0)
    z = np.linspace(-20.0, 70.0, 9001)
    hits = sum((z >= a) & (z < b) for a, b in w)
    assert (hits == 1).all()
    # each plane's own depth lies in its window, halfway cuts between planes
    for p, (a, b) in enumerate(w):
        assert a <= 10.0 * p < b
    assert w[1] == (5.0, 15.0)


def test_sliced_fit_recovers_each_planes_tables():
    # noiseless events exactly on the planes: each plane's per-sensor fit
    # reproduces that plane's tables wherever the plane's events probe them
    sxy = W.hex_array(2, 30.0)
    lrf = W.sliced_lrf(sxy, n_planes=3, nb=20)
    zp = np.linspace(lrf.z_lo, lrf.z_hi, lrf.n_planes)
    parts = [oracle.generate(lrf, 1, 130.0, z, z, 500.0, 2000.0, 2000, 60 + p, noiseless=True)
             for p, z in enumerate(zp)]
    sig = np.concatenate([s for s, _ in parts])
    truth = np.concatenate([t for _, t in parts])
    E = truth[:, 3] / (oracle.lrf_values(lrf, truth[:, :3]) @ np.asarray(lrf.gain, np.float64))
    tabs = np.asarray(lrf.coef)
    for i in (0, 9):   # no pair is clamped at 0
        for p in range(lrf.n_planes):
            on = truth[:, 2] == zp[p]
            assert (F.spline_2d(tabs[i, p], lrf.nb, lrf.lo, lrf.hi, truth[on, 0],
                                truth[on, 1]) > 0).all()
    use = np.ones(len(sig), bool)
    got, pairs = F.fit_sliced(lrf.sxy, lrf.gain, lrf.active, sig, truth[:, 0], truth[:, 1],
                              truth[:, 2], E, use, lrf.nb, lrf.lo, lrf.hi, lrf.n_planes,
                              lrf.z_lo, lrf.z_hi, np.arange(19), ridge=1e-12)
    assert got.shape == tabs.shape
    assert (pairs == 2000).all()
    for i in range(19):
        for p in range(lrf.n_planes):
            on = truth[:, 2] == zp[p]
            ref = F.spline_2d(tabs[i, p], lrf.nb, lrf.lo, lrf.hi, truth[on, 0], truth[on, 1])
            fit = F.spline_2d(got[i, p], lrf.nb, lrf.lo, lrf.hi, truth[on, 0], truth[on, 1])
            assert np.max(np.abs(fit - ref)) < 1e-7 * np.max(ref), (i, p)
            # another plane's table does not fit this plane's events
            q = (p + 1) % lrf.n_planes
            other = F.spline_2d(tabs[i, q], lrf.nb, lrf.lo, lrf.hi, truth[on, 0], truth[on, 1])
            assert np.max(np.abs(other - ref)) > 0.01 * np.max(ref)
