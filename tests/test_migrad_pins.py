"""Pins of the oracle's variable-metric search (Sec. 5.1.2.1: Minuit2's
Migrad minimiser, a variable-metric method with numerical derivatives;
here the BFGS inverse update, central-difference gradients, a halving
line search with the Armijo condition and the EDM stop).

* SciPy's BFGS (an independent implementation of the same update, with
  its own gradient differences and line search) started at the same point
  on the same objective (the oracle's node statistic) reaches the same
  minimiser.
* The statistic never increases: the result is at least as good as the
  start on every event.
* Noiseless events: the minimiser is the true position (Gibbs' inequality
  makes the truth the global minimum), reached to 1e-4 mm; the
  central-difference gradient vanishes there.
* A wrong update would still descend but slowly: the mean number of
  accepted steps on noiseless events stays small.
* Iteration cap 0 returns the start after the start's value and its
  gradient (1 + 2 d evaluations); status flags as for the grid.
"""
import numpy as np
import pytest

import oracle
import workloads as W

scipy_opt = pytest.importorskip("scipy.optimize")


def _events(n, seed=0, noiseless=False):
    wl = W.workload(2)
    sig, truth = oracle.make_events(wl.lrf, wl.events, n, W.streams(950 + seed),
                                    noiseless=noiseless)
    return wl, sig, truth


def _cfg(**kw):
    base = dict(dims=3, stat=0, step0=(10.0, 10.0, 8.0), z_start=25.0, edm_tol=1e-10,
                max_iter=200)
    base.update(kw)
    return W.MigradCfg(**base)


def _f(wl, mc, row):
    g = W.GridCfg(stat=mc.stat, l_floor=mc.l_floor, v_floor=mc.v_floor)

    def f(p):
        z = p[2] if mc.dims == 3 else mc.z_start
        return oracle.node_eval(wl.lrf, g, row, p[0], p[1], z)[0]
    return f


def test_noiseless_events_reach_the_truth():
    wl, sig, truth = _events(400, 1, noiseless=True)
    mc = _cfg(edm_tol=1e-12)
    r = oracle.reconstruct_migrad(wl.lrf, mc, sig)
    err = np.max(np.abs(np.stack([r["x"], r["y"], r["z"]], 1) - truth["pos"]), 1)
    assert (err < 1e-4).mean() >= 0.98, np.quantile(err, [0.5, 0.98])
    ok = err < 1e-4
    assert r["iters"][ok].mean() <= 15, r["iters"][ok].mean()
    # the central-difference gradient vanishes at the result
    for e in np.where(ok)[0][:20]:
        f = _f(wl, mc, sig[e])
        p = np.array([r["x"][e], r["y"][e], r["z"][e]])
        for a in range(3):
            h = np.eye(3)[a] * 1e-3
            assert abs(f(p + h) - f(p - h)) / 2e-3 < 1e-3


@pytest.mark.parametrize("stat,dims", [(0, 3), (1, 3), (0, 2)])
def test_matches_scipy_bfgs(stat, dims):
    wl, sig, truth = _events(120, 2 + stat + dims)
    mc = _cfg(stat=stat, dims=dims, edm_tol=1e-10)
    r = oracle.reconstruct_migrad(wl.lrf, mc, sig)
    start = oracle.reconstruct(wl.lrf, W.GridCfg(iterations=0), sig)   # the centroid
    agree = clean = 0
    for e in range(len(sig)):
        f = _f(wl, mc, sig[e])
        x0 = np.array([start["x"][e], start["y"][e], mc.z_start][:dims])
        s = scipy_opt.minimize(f, x0, method="BFGS", jac="3-point",
                               options={"gtol": 1e-4, "maxiter": 400})
        got = np.array([r["x"][e], r["y"][e], r["z"][e]][:dims])
        same = np.max(np.abs(s.x - got)) < 1e-3 or abs(s.fun - f(got)) < 1e-7 * abs(s.fun)
        interior = dims == 2 or 0.5 < s.x[2] < 49.5
        if s.status == 0 and interior:
            # SciPy converged (gradient norm below gtol) inside the LRF's
            # domain: the same minimiser.  (At the domain's z wall the
            # statistic jumps to infinity and both methods stall short of
            # it at different points.)
            clean += 1
            agree += same
    # both are local methods: a few events may end in different local minima
    assert clean >= 0.4 * len(sig) and agree >= 0.95 * clean, (agree, clean)


def test_never_worse_than_the_start():
    wl, sig, truth = _events(300, 7)
    for stat in (0, 1):
        mc = _cfg(stat=stat, edm_tol=1e-6)
        r = oracle.reconstruct_migrad(wl.lrf, mc, sig)
        start = oracle.reconstruct(wl.lrf, W.GridCfg(iterations=0), sig)
        for e in range(len(sig)):
            f = _f(wl, mc, sig[e])
            assert f([r["x"][e], r["y"][e], r["z"][e]]) <= f([start["x"][e], start["y"][e],
                                                              mc.z_start])


def test_iteration_cap_zero_and_status():
    wl, sig, truth = _events(50, 8)
    mc = _cfg(max_iter=0)
    r = oracle.reconstruct_migrad(wl.lrf, mc, sig)
    start = oracle.reconstruct(wl.lrf, W.GridCfg(iterations=0), sig)
    np.testing.assert_array_equal(r["x"], start["x"])
    np.testing.assert_array_equal(r["y"], start["y"])
    assert (r["z"] == mc.z_start).all() and (r["iters"] == 0).all()
    assert (r["evals"] == 1 + 2 * mc.dims).all()
    bad = sig[:4].copy()
    bad[0, :] = 0.0                                   # empty
    bad[1, 3] = -1.0                                  # bad input
    bad[2, 5] = np.nan
    g = oracle.reconstruct(wl.lrf, wl.grid, bad)
    r = oracle.reconstruct_migrad(wl.lrf, _cfg(), bad)
    np.testing.assert_array_equal(r["status"][:3], g["status"][:3])
    assert np.isnan(r["x"][:3]).all() and r["status"][3] == 0


def test_limits_keep_the_search_in_the_domain_and_match_scipy_in_internal_coordinates():
    # z of an r-z LRF is limited to the spline's domain [0, 50] as Minuit
    # limits a parameter: z = lo + (hi - lo) (sin u + 1) / 2.  SciPy's BFGS
    # on the same objective written in (x, y, u) reaches the same minimiser,
    # also for events whose minimum lies against a wall of the domain.
    wl, sig, truth = _events(300, 11)
    mc = _cfg(edm_tol=1e-10)
    r = oracle.reconstruct_migrad(wl.lrf, mc, sig)
    lo, hi = wl.lrf.lo[1], wl.lrf.hi[1]
    assert ((r["z"] >= lo) & (r["z"] <= hi)).all()
    start = oracle.reconstruct(wl.lrf, W.GridCfg(iterations=0), sig)
    half = 0.5 * (hi - lo)
    agree = clean = walls = 0
    for e in range(len(sig)):
        f = _f(wl, mc, sig[e])

        def fu(v):
            return f([v[0], v[1], lo + half * (np.sin(v[2]) + 1.0)])
        u0 = np.array([start["x"][e], start["y"][e],
                       np.arcsin(np.clip((mc.z_start - lo) / half - 1.0, -1.0, 1.0))])
        s = scipy_opt.minimize(fu, u0, method="BFGS", jac="3-point",
                               options={"gtol": 1e-4, "maxiter": 400})
        zs = lo + half * (np.sin(s.x[2]) + 1.0)
        got = np.array([r["x"][e], r["y"][e], r["z"][e]])
        if s.status != 0:
            continue
        clean += 1
        walls += zs < lo + 0.5 or zs > hi - 0.5
        same = np.max(np.abs(np.array([s.x[0], s.x[1], zs]) - got)) < 2e-3 or \
            abs(s.fun - f(got)) < 1e-8 * abs(s.fun)
        agree += same
    assert clean >= 0.8 * len(sig) and walls >= 3, (clean, walls)
    assert agree >= 0.95 * clean, (agree, clean)
