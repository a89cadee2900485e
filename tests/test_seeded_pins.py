"""Pins of the oracle's seeded refinement, its chi2/ndf fallback, the tie
rule and the LRF clamp.

* Seeded refinement (learned seed, Sec. 5.1.3, refined by the contracting
  grid of Sec. 5.1.2.2): the event's iteration count K comes from the
  seed's predicted spread.  Pinned by equivalence: every seeded event must
  equal the plain seed-started grid with K iterations that starts from the
  step s_f * shrink^-(K-1) and ends on the configured final step s_f, and
  K must equal the closed form clamp(1 + ceil(log_{1/shrink}(kappa sigma /
  s_f)), kmin, kmax) (a logarithm, not the oracle's loop).  Shrink 0.5 keeps
  every step exact in binary, so the equivalences are bitwise.
* Fallback: events whose chi2/ndf at the refined node exceeds the threshold
  (or is not finite, or ndf <= 0) are reconstructed again by the fallback
  grid.  Pinned by the two limits (threshold 0, threshold +inf) and by the
  boundary value (chi2/ndf equal to the threshold stays).
* Ties (the paper does not order equally good nodes; reading: statistics
  within 1e-12 N are equal and the lowest node index wins): mirror-image
  nodes of a mirror-symmetric event are mathematically equal but their sums
  run in different sensor orders; the lower index must win and TIE must be
  set.  A relative asymmetry of 1e-9 in the signals must decide the other
  way.
* LRF clamp (reading: L = max(spline, 0) inside the domain): checked
  against the independent Cox-de Boor evaluator and through the node sums.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import workloads as W

SF = 7.5 * 0.5 ** 7      # final step of the 8-iteration refinement grid below


def _refine(kmin=2, kmax=6, kappa=1.0, scale=(3.0, 3.0, 0.0)):
    return W.GridCfg((3, 3, 1), 8, 0.5, (7.5, 7.5, 0.0), 0.0, start=2, seed_steps=1,
                     seed_kappa=kappa, seed_kmin=kmin, seed_kmax=kmax, seed_scale=scale)


def _events(n, seed=0):
    wl = W.workload(0)
    sig, truth = oracle.make_events(wl.lrf, wl.events, n, W.streams(700 + seed))
    rng = np.random.default_rng(seed)
    seeds = np.zeros((n, 4))
    seeds[:, :2] = truth["pos"][:, :2] + rng.normal(0.0, 1.5, (n, 2))
    return wl, sig, seeds


def _plain_equivalent(K):
    # seed-started grid with K iterations ending on the final step SF
    return W.GridCfg((3, 3, 1), K, 0.5, (SF * 2.0 ** (K - 1), SF * 2.0 ** (K - 1), 0.0), 0.0,
                     start=2)


def _iterations(out):
    return (out["path"] >= 0).sum(1)


def _same_event(a, b, e, ea=None):
    ea = e if ea is None else ea
    for k in ("x", "y", "z", "E", "lnl", "chi2"):
        np.testing.assert_array_equal(a[k][ea], b[k][e], err_msg=k)
    assert a["ndf"][ea] == b["ndf"][e] and a["status"][ea] == b["status"][e]


def _closed_form_K(s, kappa, scale, kmin, kmax):
    need = math.exp(0.5 * s) * kappa * scale
    if not math.isfinite(need):
        return kmax
    if need <= SF:
        return kmin
    return int(min(max(1 + math.ceil(math.log2(need / SF)), kmin), kmax))


def test_iteration_count_follows_the_closed_form_and_equals_the_plain_grid():
    wl, sig, seeds = _events(60)
    # spreads from well below the kmin step to well above the kmax step
    seeds[:, 3] = np.linspace(2 * math.log(0.01), 2 * math.log(40.0), 60)
    R = _refine()
    got = oracle.reconstruct(wl.lrf, R, sig, seeds=seeds)
    Ks = _iterations(got)
    expect = [_closed_form_K(s, 1.0, 3.0, 2, 6) for s in seeds[:, 3]]
    np.testing.assert_array_equal(Ks, expect)
    assert set(Ks) == {2, 3, 4, 5, 6}
    for K in set(Ks):
        idx = np.where(Ks == K)[0]
        ref = oracle.reconstruct(wl.lrf, _plain_equivalent(K), sig[idx], seeds=seeds[idx])
        for i, e in enumerate(idx):
            _same_event(got, ref, i, e)
            np.testing.assert_array_equal(got["path"][e, :K], ref["path"][i])
            assert np.all(got["path"][e, K:] == -1)


@pytest.mark.parametrize("s,K", [(math.inf, 6), (math.nan, 6), (-math.inf, 2)])
def test_non_finite_spread(s, K):
    wl, sig, seeds = _events(8, seed=1)
    seeds[:, 3] = s
    got = oracle.reconstruct(wl.lrf, _refine(), sig, seeds=seeds)
    assert np.all(_iterations(got) == K)
    ref = oracle.reconstruct(wl.lrf, _plain_equivalent(K), sig, seeds=seeds)
    for e in range(len(sig)):
        _same_event(got, ref, e)


@pytest.mark.parametrize("j", [1, 2, 3, 4])
def test_spread_on_a_step_boundary(j):
    # s = 0 gives sigma = 1 exactly; kappa * sigma * scale = SF * 2^j lands
    # on the first step of the (j+1)-iteration grid, which is long enough
    wl, sig, seeds = _events(4, seed=2)
    seeds[:, 3] = 0.0
    on = SF * 2.0 ** j
    got = oracle.reconstruct(wl.lrf, _refine(scale=(on, on, 0.0)), sig, seeds=seeds)
    assert np.all(_iterations(got) == j + 1)
    above = np.nextafter(on, np.inf)
    got = oracle.reconstruct(wl.lrf, _refine(scale=(above, above, 0.0)), sig, seeds=seeds)
    assert np.all(_iterations(got) == j + 2)
    # one axis is enough to need the longer grid
    got = oracle.reconstruct(wl.lrf, _refine(scale=(on, above, 0.0)), sig, seeds=seeds)
    assert np.all(_iterations(got) == j + 2)


def test_threshold_zero_equals_the_fallback_grid():
    wl, sig, seeds = _events(40, seed=3)
    seeds[:, 3] = 2 * math.log(1.5)
    got = oracle.reconstruct_seeded(wl.lrf, _refine(), wl.grid, 0.0, sig, seeds)
    ref = oracle.reconstruct(wl.lrf, wl.grid, sig)
    for e in range(len(sig)):
        for k in ("x", "y", "z", "E", "lnl", "chi2"):
            assert got[k][e] == ref[k][e], k
        assert got["status"][e] == ref["status"][e] | 16


def test_infinite_threshold_keeps_every_finite_refinement():
    wl, sig, seeds = _events(40, seed=4)
    seeds[:, 3] = 2 * math.log(1.5)
    seeds[5, :2] = (1000.0, 0.0)      # refinement far outside: chi2 not finite
    got = oracle.reconstruct_seeded(wl.lrf, _refine(), wl.grid, math.inf, sig, seeds)
    ref = oracle.reconstruct(wl.lrf, _refine(), sig, seeds=seeds)
    fb = oracle.reconstruct(wl.lrf, wl.grid, sig)
    assert not np.isfinite(ref["chi2"][5])
    for e in range(len(sig)):
        src = fb if e == 5 else ref
        for k in ("x", "y", "E", "lnl", "chi2"):
            assert got[k][e] == src[k][e], (e, k)
        assert got["status"][e] == (src["status"][e] | (16 if e == 5 else 0))


def test_fallback_boundary_keeps_chi2_per_ndf_equal_to_the_threshold():
    wl, sig, seeds = _events(12, seed=5)
    seeds[:, 3] = 2 * math.log(1.5)
    ref = oracle.reconstruct(wl.lrf, _refine(), sig, seeds=seeds)
    for e in (0, 7):
        thr = ref["chi2"][e] / ref["ndf"][e]
        at = oracle.reconstruct_seeded(wl.lrf, _refine(), wl.grid, thr, sig[e:e + 1],
                                       seeds[e:e + 1])
        assert at["status"][0] & 16 == 0 and at["x"][0] == ref["x"][e]
        below = oracle.reconstruct_seeded(wl.lrf, _refine(), wl.grid, np.nextafter(thr, 0.0),
                                          sig[e:e + 1], seeds[e:e + 1])
        assert below["status"][0] & 16


def test_no_degrees_of_freedom_always_falls_back():
    wl, sig, seeds = _events(6, seed=6)
    lrf = dataclasses.replace(wl.lrf, active=np.zeros(19, np.uint8))
    lrf.active[[8, 9, 10]] = 1                   # 3 sensors: ndf = 3 - 3 = 0
    seeds[:, 3] = 2 * math.log(1.5)
    got = oracle.reconstruct_seeded(lrf, _refine(), wl.grid, math.inf, sig, seeds)
    assert np.all(got["ndf"] == 0)
    assert np.all(got["status"] & 16)


# ------------------------------------------------------------------ ties


def _mirror_perm(sxy):
    # index of the sensor at (-X, Y)
    key = {(round(x, 6), round(y, 6)): i for i, (x, y) in enumerate(sxy)}
    return np.array([key[(round(-x, 6), round(y, 6))] for x, y in sxy])


def test_mirror_image_nodes_tie_and_the_lower_index_wins():
    # a source pair at (+-d, y0): the likelihood of one source is symmetric
    # in x with its minima at x = +-d; the grid is centred at x = 0
    wl = W.workload(0)
    sxy = wl.lrf.sxy
    perm = _mirror_perm(sxy)
    g = W.GridCfg((9, 9, 1), 1, 0.5, (7.5, 7.5, 0.0), 0.0, start=2)
    n_ties = n_rounded = 0
    for d, y0 in [(30.0, 0.0), (37.5, 15.0), (30.0, 3.3), (26.1, -4.2), (33.3, 11.1)]:
        pos = np.array([[d, y0, 0.0], [-d, y0, 0.0]])
        mu = oracle.expected_counts(wl.lrf, pos, np.array([1500.0, 1500.0]))
        sig = (0.5 * (mu[0] + mu[1]))[None, :]
        np.testing.assert_allclose(sig[0], sig[0][perm], rtol=1e-12)
        sig = 0.5 * (sig + sig[:, perm])          # exactly symmetric
        seed = np.array([[0.0, y0, 0.0, 0.0]])
        st = oracle.lattice_stats(wl.lrf, g, sig[0], (0.0, y0, 0.0), (7.5, 7.5, 0.0), (9, 9, 1))
        j = int(np.argmin(st))
        jm = (j // 9) * 9 + (8 - j % 9)           # mirror node
        if j % 9 == 4:
            continue                              # single minimum on the axis
        n_ties += 1
        n_rounded += st[j] != st[jm]              # equal values, different rounding
        r = oracle.reconstruct(wl.lrf, g, sig, seeds=seed)
        assert r["path"][0, 0] == min(j, jm) and r["path"][0, 0] % 9 < 4
        assert r["status"][0] & 32
        # a 1e-9 relative excess on the +x side (a gap of about 1e-9 N in the
        # statistic, 1000 times the tolerance) decides for the +x node
        tilt = sig.copy()
        tilt[0, sxy[:, 0] > 0] *= 1.0 + 1e-9
        r2 = oracle.reconstruct(wl.lrf, g, tilt, seeds=seed)
        assert r2["path"][0, 0] == max(j, jm) and not r2["status"][0] & 32
    assert n_ties == 5 and n_rounded >= 2


# ------------------------------------------------------------- LRF clamp


def _lobed_lrf():
    # a shared axial spline with a negative lobe between r = 40 and 70 mm
    lrf = W.axial_lrf(W.hex_array(2, 30.0))
    c = lrf.coef.reshape(-1).copy()
    c[7:11] = -0.05
    lrf.coef = c.reshape(1, 1, -1)
    return lrf


def test_negative_spline_is_clamped_to_zero():
    lrf = _lobed_lrf()
    c = lrf.coef.reshape(-1)
    r = np.linspace(0.0, 150.0, 1501)
    spline = oracle.deboor1(c, 20, 0.0, 150.0, r)
    assert spline.min() < -0.01
    pos = np.stack([lrf.sxy[4, 0] + r, np.full_like(r, lrf.sxy[4, 1]), np.zeros_like(r)], 1)
    L = oracle.lrf_values(lrf, pos)[:, 4]
    np.testing.assert_allclose(L, np.maximum(spline, 0.0), rtol=0, atol=1e-13)
    assert np.all(L[spline < -1e-12] == 0.0)


def test_clamped_sensors_leave_the_node_sums():
    lrf = _lobed_lrf()
    g = W.GridCfg()
    x, y = 3.0, -2.0
    rr = np.hypot(lrf.sxy[:, 0] - x, lrf.sxy[:, 1] - y)
    spline = oracle.deboor1(lrf.coef.reshape(-1), 20, 0.0, 150.0, rr)
    assert (spline < 0).sum() >= 3
    n = np.random.default_rng(3).poisson(30.0, 19).astype(np.float64)
    stat, S, A, lnl, chi2 = oracle.node_eval(lrf, g, n, x, y)
    Lc = np.maximum(spline, 0.0)
    assert S == pytest.approx(Lc.sum(), rel=1e-13)
    mu = A * Lc
    ref = np.sum(np.where(n > 0, n * np.log(A * np.maximum(Lc, 1e-9)), 0.0) - mu)
    assert lnl == pytest.approx(ref, rel=1e-12)
