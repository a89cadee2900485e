"""Pins for the FP64 oracle: facts fixed by the paper or by mathematics,
independent of the oracle's own formulas (Sec. 5.1.1, 5.1.2, 5.1.2.2, 5.3, 6).

Each test is chosen so that a plausible slip in the oracle (a dropped term,
a wrong sign or index, a transposed operand) fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _grid(**kw):
    g = W.GridCfg()
    for k, v in kw.items():
        setattr(g, k, v)
    return g


# ----------------------------------------------------------------- B-splines


def test_partition_of_unity():
    # all coefficients equal -> the spline is that constant everywhere
    nb, lo, hi = 20, 0.0, 150.0
    c = np.full(nb + 2, 3.25)
    u = np.linspace(lo, hi, 1001)
    np.testing.assert_allclose(oracle.spline1(c, nb, lo, hi, u), 3.25, rtol=0, atol=1e-14)
    for t in np.linspace(0, 1, 11):
        assert abs(oracle.basis(t).sum() - 1.0) < 1e-15


def test_cubic_reproduction_1d_and_2d():
    # cubic B-splines reproduce cubic polynomials; the quasi-interpolant of a
    # cubic therefore gives back the cubic exactly
    p = lambda u: 0.3 - 1.7 * u + 0.05 * u ** 2 - 0.002 * u ** 3
    nb, lo, hi = 13, -5.0, 31.0
    c = W.quasi_interp_1d(p, lo, hi, nb)
    u = np.linspace(lo, hi, 777)
    np.testing.assert_allclose(oracle.spline1(c, nb, lo, hi, u), p(u), rtol=1e-12, atol=1e-12)
    q = lambda a, b: 1.0 + 0.2 * a - 0.1 * b + 0.01 * a * b - 0.003 * a ** 3 + 0.0007 * b ** 3 \
        + 1e-4 * a ** 2 * b
    nb2, lo2, hi2 = (9, 7), (-2.0, 0.0), (6.0, 50.0)
    c2 = W.quasi_interp_2d(q, lo2, hi2, nb2)
    rng = np.random.default_rng(1)
    a = rng.uniform(lo2[0], hi2[0], 300)
    b = rng.uniform(lo2[1], hi2[1], 300)
    np.testing.assert_allclose(oracle.spline2(c2, nb2, lo2, hi2, a, b), q(a, b), rtol=1e-11,
                               atol=1e-11)


def test_de_boor_recursion_agrees_with_closed_form():
    rng = np.random.default_rng(2)
    nb, lo, hi = 24, 0.0, 200.0
    c = rng.normal(size=nb + 2)
    u = np.concatenate([rng.uniform(lo, hi, 500), lo + (hi - lo) / (nb - 1) * np.arange(nb - 1)])
    np.testing.assert_allclose(oracle.spline1(c, nb, lo, hi, u), oracle.deboor1(c, nb, lo, hi, u),
                               rtol=0, atol=1e-13)


def test_c2_continuity_at_breakpoints():
    rng = np.random.default_rng(3)
    nb, lo, hi = 20, 0.0, 150.0
    c = rng.normal(size=nb + 2)
    d = (hi - lo) / (nb - 1)
    h = 1e-6
    for m in range(1, nb - 1):
        u = lo + m * d
        v = oracle.spline1(c, nb, lo, hi, [u - h, u, u + h])
        assert abs(v[0] - 2 * v[1] + v[2]) < 1e-9        # no kink
        dl = oracle.spline1_du(c, nb, lo, hi, [u - 1e-9, u + 1e-9])
        assert abs(dl[0] - dl[1]) < 1e-7                   # C1
        # second derivative from both sides by one-sided differences
        s = 1e-3
        left = oracle.spline1(c, nb, lo, hi, [u - 2 * s, u - s, u])
        right = oracle.spline1(c, nb, lo, hi, [u, u + s, u + 2 * s])
        assert abs((left[0] - 2 * left[1] + left[2]) - (right[0] - 2 * right[1] + right[2])) / s**2 < 2e-3


def test_spline_derivative_matches_finite_difference():
    wl = W.workload(0)
    c = wl.lrf.coef.reshape(-1)
    nb, lo, hi = wl.lrf.nb[0], wl.lrf.lo[0], wl.lrf.hi[0]
    u = np.linspace(1, 149, 97)
    h = 1e-5
    fd = (oracle.spline1(c, nb, lo, hi, u + h) - oracle.spline1(c, nb, lo, hi, u - h)) / (2 * h)
    np.testing.assert_allclose(oracle.spline1_du(c, nb, lo, hi, u), fd, rtol=1e-6, atol=1e-9)


def test_lrf_outside_domain_is_zero_and_fit_quality():
    wl = W.workload(0)
    far = oracle.lrf_values(wl.lrf, np.array([[500.0, 0.0, 0.0]]))
    assert np.all(far[0] == 0.0)
    # data quality of the quasi-interpolant (not parity): 20 breakpoints over
    # 150 mm resolve the 10 mm-wide peak to within 8% of its height, and the
    # tail (r > 30 mm) to 0.5%
    r = np.linspace(0, 150, 3001)
    c = wl.lrf.coef.reshape(-1)
    err = np.abs(oracle.spline1(c, 20, 0.0, 150.0, r) - W.solid_angle(10.0, r * r))
    assert err.max() < 0.08
    assert err[r > 30].max() < 0.005


# ----------------------------------------------------------------- centroid


def test_cog_two_sensors_is_gain_weighted_mean():
    # Sec. 5.1.1: x = sum X S/g / sum S/g.  Zero iterations return the start.
    sxy = np.array([[-10.0, 0.0], [20.0, 6.0]])
    lrf = W.axial_lrf(sxy, gain=np.array([2.0, 0.5]))
    g = _grid(iterations=0)
    sig = np.array([[10.0, 3.0]])
    r = oracle.reconstruct(lrf, g, sig)
    w = np.array([10.0 / 2.0, 3.0 / 0.5])
    assert r["x"][0] == pytest.approx((w @ sxy[:, 0]) / w.sum(), abs=1e-12)
    assert r["y"][0] == pytest.approx((w @ sxy[:, 1]) / w.sum(), abs=1e-12)


def test_cog_symmetric_signals_give_array_centre():
    sxy = W.hex_array(2, 30.0)
    lrf = W.axial_lrf(sxy)
    ring = np.hypot(sxy[:, 0], sxy[:, 1])
    sig = (100.0 / (1.0 + ring / 30.0))[None, :]
    r = oracle.reconstruct(lrf, _grid(iterations=0), sig)
    assert abs(r["x"][0]) < 1e-12 and abs(r["y"][0]) < 1e-12


def test_strongest_sensor_start():
    sxy = W.hex_array(2, 30.0)
    lrf = W.axial_lrf(sxy)
    sig = np.ones((1, 19))
    sig[0, 7] = 50.0
    sig[0, 11] = 50.0           # tie between sensors 7 and 11: lowest index
    r = oracle.reconstruct(lrf, _grid(iterations=0, start=1), sig)
    assert (r["x"][0], r["y"][0]) == (sxy[7, 0], sxy[7, 1])


# ----------------------------------------------------- energy and statistic


def _event(k, noiseless, n=64, seed_offset=0):
    wl = W.workload(k)
    rngs = W.streams(k + 100 * seed_offset)
    pos, etot = W.draw_sources(wl.events, n, rngs[0], rngs[1])
    mu = oracle.expected_counts(wl.lrf, pos, etot)
    sig = mu if noiseless else W.poisson_counts(mu, rngs[3]).astype(np.float64)
    return wl, pos, etot, mu, sig


@pytest.mark.parametrize("k", [0, 1, 2])
def test_energy_ratio_is_stationary_point_of_likelihood(k):
    # Sec. 5.1.2.2: the energy is the ratio of the summed signals to the
    # summed LRFs; for Poisson counts that is exactly where dl/dA = 0
    wl, pos, etot, mu, sig = _event(k, noiseless=False, n=8)
    g = wl.lrf.gain
    for e in range(8):
        p = pos[e] + np.array([0.7, -0.4, 0.5 if k == 2 else 0.0])
        p[:2] = np.clip(p[:2], -23.0, 23.0) if k == 1 else p[:2]
        res = oracle.node_eval(wl.lrf, wl.grid, sig[e], *p)
        A = res[2]
        L = oracle.lrf_values(wl.lrf, p[None, :])[0]

        def ell(a):
            Lt = np.maximum(L, 1e-9)
            return np.sum(np.where(sig[e] > 0, sig[e] * np.log(np.where(sig[e] > 0, a * g * Lt, 1.0)), 0.0)
                          - a * g * L)
        assert ell(A) == pytest.approx(res[3], rel=1e-12)
        assert ell(A * (1 + 1e-4)) < ell(A) and ell(A * (1 - 1e-4)) < ell(A)
        assert A == pytest.approx(sig[e].sum() / np.sum(g * L), rel=1e-13)


@pytest.mark.parametrize("k", [0, 2])
def test_noiseless_energy_at_truth(k):
    wl, pos, etot, mu, sig = _event(k, noiseless=True, n=16)
    for e in range(16):
        res = oracle.node_eval(wl.lrf, wl.grid, sig[e], *pos[e])
        S = np.sum(wl.lrf.gain * oracle.lrf_values(wl.lrf, pos[e][None, :])[0])
        assert res[2] == pytest.approx(etot[e] / S, rel=1e-12)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_gibbs_inequality_for_noiseless_events(k):
    # with n_i = mu_i(truth), the Poisson likelihood is largest at the truth
    wl, pos, etot, mu, sig = _event(k, noiseless=True, n=12)
    rng = np.random.default_rng(5)
    for e in range(12):
        at_truth = oracle.node_eval(wl.lrf, wl.grid, sig[e], *pos[e])[0]
        for _ in range(40):
            p = pos[e] + rng.normal(scale=[3.0, 3.0, 5.0 if k == 2 else 0.0])
            assert oracle.node_eval(wl.lrf, wl.grid, sig[e], *p)[0] >= at_truth - 1e-9


def test_one_pass_decomposition_matches_direct_form():
    # l = sum n ln L~ + sum n ln g + N ln(N/S) - N, because A S = N
    wl, pos, etot, mu, sig = _event(1, noiseless=False, n=10)
    g = wl.lrf.gain
    for e in range(10):
        p = np.clip(pos[e] + 0.3, -23.0, 23.0)
        L = oracle.lrf_values(wl.lrf, p[None, :])[0]
        N, S = sig[e].sum(), np.sum(g * L)
        one_pass = (np.sum(sig[e] * np.log(np.maximum(L, 1e-9))) + np.sum(sig[e] * np.log(g))
                    + N * math.log(N / S) - N)
        assert oracle.node_eval(wl.lrf, wl.grid, sig[e], *p)[3] == pytest.approx(one_pass, rel=1e-12)


def test_chi2_definition_hand_case():
    # Pearson chi2 with variance floor 1: two sensors, hand-computed
    sxy = np.array([[0.0, 0.0], [30.0, 0.0]])
    lrf = W.axial_lrf(sxy)
    L = oracle.lrf_values(lrf, np.array([[5.0, 0.0, 0.0]]))[0]
    n = np.array([80.0, 0.0])
    A = 80.0 / L.sum()
    mu = A * L
    want = (80 - mu[0]) ** 2 / max(mu[0], 1) + (0 - mu[1]) ** 2 / max(mu[1], 1)
    res = oracle.node_eval(lrf, _grid(stat=1), n, 5.0, 0.0)
    assert res[0] == pytest.approx(want, rel=1e-13) and res[4] == pytest.approx(want, rel=1e-13)


# ------------------------------------------------------------------- search


@pytest.mark.parametrize("k", [0, 2])
def test_single_iteration_is_brute_force_over_the_lattice(k):
    wl, pos, etot, mu, sig = _event(k, noiseless=False, n=20)
    g = W.GridCfg(**{**wl.grid.__dict__, "iterations": 1})
    r = oracle.reconstruct(wl.lrf, g, sig)
    for e in range(20):
        start = oracle.reconstruct(wl.lrf, W.GridCfg(**{**g.__dict__, "iterations": 0}),
                                   sig[e:e + 1])
        c = [start["x"][0], start["y"][0], start["z"][0]]
        st = oracle.lattice_stats(wl.lrf, g, sig[e], c, g.step0, g.nodes)
        j = int(np.argmin(st))        # numpy argmin: first (lowest) index on ties
        assert r["path"][e, 0] == j


@pytest.mark.parametrize("k", [0, 1, 2])
def test_noiseless_events_land_within_final_step(k):
    # fiducial region: the grid search is a heuristic, and at the rim of a
    # hexagonal array its coarse first grid can settle in a side minimum
    wl, pos, etot, mu, sig = _event(k, noiseless=True, n=400 if k != 2 else 150)
    r = oracle.reconstruct(wl.lrf, wl.grid, sig)
    sf = wl.grid.final_step
    d = np.abs(np.stack([r["x"] - pos[:, 0], r["y"] - pos[:, 1], r["z"] - pos[:, 2]], 1))
    rad = np.hypot(pos[:, 0], pos[:, 1])
    fid = rad < (45.0 if k == 0 else 75.0) if k != 1 else np.ones(len(rad), bool)
    ok = (d[:, 0] <= sf[0]) & (d[:, 1] <= sf[1])
    if wl.grid.nodes[2] > 1:
        ok &= d[:, 2] <= sf[2]
    assert ok[fid].all(), np.where(fid & ~ok)
    assert ok.mean() > 0.97


def test_statistic_never_increases_with_more_iterations():
    wl, pos, etot, mu, sig = _event(0, noiseless=False, n=50)
    prev = None
    for K in range(1, 7):
        g = W.GridCfg(**{**wl.grid.__dict__, "iterations": K})
        r = oracle.reconstruct(wl.lrf, g, sig)
        cur = -r["lnl"]
        if prev is not None:
            assert np.all(cur <= prev + 1e-9)
        prev = cur


def test_tiny_array_against_dense_brute_force():
    # 7-sensor hexagon (one ring): dense 0.02 mm lattice over +-6 mm around
    # the truth; the grid result lies within the final step of the dense
    # minimiser
    sxy = W.hex_array(1, 30.0)
    lrf = W.axial_lrf(sxy)
    grid = W.GridCfg((9, 9, 1), 6, 0.5, (7.5, 7.5, 0.0), 0.0)
    rngs = W.streams(77)
    pos, etot = W.draw_sources(W.EventRecipe("disc", 20.0, 800.0, 1500.0), 6, rngs[0], rngs[1])
    mu = oracle.expected_counts(lrf, pos, etot)
    sig = W.poisson_counts(mu, rngs[3]).astype(np.float64)
    r = oracle.reconstruct(lrf, grid, sig)
    step = 0.02
    nn = 601
    for e in range(6):
        st = oracle.lattice_stats(lrf, grid, sig[e], [pos[e, 0], pos[e, 1], 0.0],
                                  [step, step, 0.0], [nn, nn, 1])
        j = int(np.argmin(st))
        bx = pos[e, 0] + (j % nn - (nn - 1) // 2) * step
        by = pos[e, 1] + (j // nn - (nn - 1) // 2) * step
        assert abs(r["x"][e] - bx) <= grid.final_step[0] + step
        assert abs(r["y"][e] - by) <= grid.final_step[1] + step


def _mirror_perm(sxy, axis):
    m = sxy.copy()
    m[:, axis] = -m[:, axis]
    perm = np.array([int(np.argmin(np.hypot(*(sxy - p).T))) for p in m])
    assert np.allclose(sxy[perm], m)
    return perm


@pytest.mark.parametrize("axis", [0, 1])
def test_hexagonal_mirror_symmetry(axis):
    wl, pos, etot, mu, sig = _event(0, noiseless=False, n=200)
    perm = _mirror_perm(wl.lrf.sxy, axis)
    a = oracle.reconstruct(wl.lrf, wl.grid, sig)
    b = oracle.reconstruct(wl.lrf, wl.grid, sig[:, perm])
    key = ["x", "y"][axis]
    other = ["y", "x"][axis]
    good = (a["status"] & 32) == 0
    np.testing.assert_allclose(b[key][good], -a[key][good], atol=1e-9)
    np.testing.assert_allclose(b[other][good], a[other][good], atol=1e-9)
    np.testing.assert_allclose(b["lnl"][good], a["lnl"][good], rtol=1e-12)


def test_all_nodes_tie_lowest_index_wins():
    # a constant LRF makes every node equally good: the corner node (index
    # 0) wins every iteration, the path is deterministic and TIE is flagged
    sxy = W.hex_array(2, 30.0)
    lrf = W.axial_lrf(sxy)
    lrf.coef = np.ones_like(lrf.coef)
    lrf.hi = (1000.0, 0.0)       # constant far beyond every node
    g = W.GridCfg((9, 9, 1), 4, 0.5, (2.0, 2.0, 0.0), 0.0)
    sig = np.random.default_rng(9).poisson(40.0, size=(3, 19)).astype(np.float64)
    r = oracle.reconstruct(lrf, g, sig)
    start = oracle.reconstruct(lrf, W.GridCfg(**{**g.__dict__, "iterations": 0}), sig)
    assert np.all(r["path"] == 0)
    assert np.all(r["status"] & 32)
    shift = 4 * 2.0 * (1 + 0.5 + 0.25 + 0.125)
    np.testing.assert_allclose(r["x"], start["x"] - shift, atol=1e-12)
    np.testing.assert_allclose(r["y"], start["y"] - shift, atol=1e-12)


def test_single_sensor_likelihood_is_flat():
    # one sensor: A = n/L and l = n ln n - n at every node with L > 0
    lrf = W.axial_lrf(np.array([[0.0, 0.0]]))
    g = W.GridCfg((9, 9, 1), 2, 0.5, (5.0, 5.0, 0.0), 0.0)
    r = oracle.reconstruct(lrf, g, np.array([[57.0]]))
    assert np.all(r["path"][0] == 0) and r["status"][0] & 32
    assert r["lnl"][0] == pytest.approx(57 * math.log(57) - 57, rel=1e-13)


def test_single_sensor_ring_of_ties_lowest_valid_index():
    # one sensor, a grid reaching past the LRF domain (r <= 150 mm): every
    # node inside the domain ties (A g L = N at each of them), the nodes
    # outside are invalid, so the winner is the lowest index inside the disc
    lrf = W.axial_lrf(np.array([[0.0, 0.0]]))
    for stat in (0, 1):
        g = W.GridCfg((9, 9, 1), 1, 0.5, (32.0, 32.0, 0.0), 0.0, stat=stat)
        r = oracle.reconstruct(lrf, g, np.array([[57.0]]))
        off = (np.arange(81) % 9 - 4) * 32.0, (np.arange(81) // 9 - 4) * 32.0
        inside = np.hypot(*off) <= 150.0
        j = int(np.argmax(inside))
        assert j == 2 and r["path"][0, 0] == j and r["status"][0] & 32
        assert r["x"][0] == off[0][j] and r["y"][0] == off[1][j]


# ---------------------------------------------------------- per-event status


def test_status_flags_and_passive_sensors():
    wl, pos, etot, mu, sig = _event(0, noiseless=False, n=6)
    sig = sig.copy()
    sig[1] = 0.0
    sig[2, 3] = np.nan
    sig[3, 4] = -1.0
    r = oracle.reconstruct(wl.lrf, wl.grid, sig)
    assert list(r["status"][:4]) == [r["status"][0], 1, 2, 2]
    assert r["status"][0] in (0, 32)
    assert np.isnan(r["x"][1]) and np.isnan(r["E"][2])
    assert r["ndf"][0] == 19 - 3
    # Sec. 5.3: passive sensors are ignored; a passive sensor's value, even
    # NaN, changes nothing, and the result equals the detector without it
    lrf_p = W.axial_lrf(wl.lrf.sxy)
    lrf_p.active = np.ones(19, np.uint8)
    lrf_p.active[5] = 0
    s2 = sig[[0, 4, 5]].copy()
    s2[:, 5] = np.nan
    a = oracle.reconstruct(lrf_p, wl.grid, s2)
    keep = [i for i in range(19) if i != 5]
    lrf_r = W.axial_lrf(wl.lrf.sxy[keep])
    b = oracle.reconstruct(lrf_r, wl.grid, sig[[0, 4, 5]][:, keep])
    for key in ("x", "y", "E", "lnl", "chi2"):
        np.testing.assert_array_equal(a[key], b[key])
    assert a["ndf"][0] == 18 - 3
    # all passive
    lrf_p.active[:] = 0
    assert oracle.reconstruct(lrf_p, wl.grid, sig[:1])["status"][0] == 4


# ---------------------------------------------------------- whole pipeline


def test_resolution_reaches_cramer_rao_bound():
    # an efficient estimator at these photon counts: the rms error over many
    # events matches the mean Cramer-Rao bound computed from the LRF
    # derivatives (a closed form independent of the search)
    wl, pos, etot, mu, sig = _event(0, noiseless=False, n=3000, seed_offset=3)
    rad = np.hypot(pos[:, 0], pos[:, 1])
    r = oracle.reconstruct(wl.lrf, wl.grid, sig)
    S = (oracle.lrf_values(wl.lrf, pos) * wl.lrf.gain).sum(1)
    var = oracle.crb(wl.lrf, 2, pos, etot / S)
    fid = rad < 45
    err2 = (r["x"] - pos[:, 0]) ** 2 + (r["y"] - pos[:, 1]) ** 2
    ratio = math.sqrt(err2[fid].mean() / var[fid].sum(1).mean())
    assert 0.95 < ratio < 1.2, ratio
