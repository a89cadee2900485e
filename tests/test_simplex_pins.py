"""Pins of the oracle's simplex search (Sec. 5.1.2.1: Minuit2's Simplex
minimiser over the position, from the centroid or the strongest sensor;
here the Nelder-Mead method of Lagarias et al. 1998 with coefficients
1, 2, 1/2, 1/2).

* SciPy's Nelder-Mead, an independent implementation of the same published
  method, started from the same simplex with the same stopping rule
  (every vertex within tol of the best, per axis), reaches the same
  minimiser on the same objective (the oracle's node statistic).
* The same path: after k iterations SciPy holds the same best vertex, and
  it stops after the same number of iterations.
* The best value never increases: the result after k iterations has a
  statistic at least as good as after k - 1.
* Noiseless events: the minimiser is the true position (Gibbs' inequality
  makes the truth the global minimum).
* One sensor: the likelihood is flat, every comparison ties, so the method
  only shrinks towards the start vertex: the result is the start exactly,
  after ceil(log2(step0 / tol)) shrinks.
* Iteration cap 0 returns the best vertex of the initial simplex; status
  flags as for the grid.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

scipy_opt = pytest.importorskip("scipy.optimize")


def _events(k, n, seed=0, noiseless=False):
    wl = W.workload(k)
    sig, truth = oracle.make_events(wl.lrf, wl.events, n, W.streams(900 + seed),
                                    noiseless=noiseless)
    return wl, sig, truth


def _start(wl, sig):
    # the centroid start (the grid with no iteration returns it)
    return oracle.reconstruct(wl.lrf, W.GridCfg(iterations=0), sig)


def _scipy_nm(wl, sc, sig_row, start):
    d = sc.dims
    gcfg = W.GridCfg(stat=sc.stat, l_floor=sc.l_floor, v_floor=sc.v_floor)

    def f(p):
        z = p[2] if d == 3 else sc.z_start
        return oracle.node_eval(wl.lrf, gcfg, sig_row, p[0], p[1], z)[0]

    x0 = np.array(start[:d], np.float64)
    sim = np.array([x0] + [x0 + np.eye(d)[i] * sc.step0[i] for i in range(d)])
    r = scipy_opt.minimize(f, x0, method="Nelder-Mead",
                           options={"initial_simplex": sim, "xatol": sc.tol, "fatol": math.inf,
                                    "maxiter": sc.max_iter, "maxfev": 100 * sc.max_iter})
    return r.x, r.fun, r.nit


@pytest.mark.parametrize("k,stat", [(0, 0), (0, 1), (1, 0)])
def test_same_minimiser_as_scipy_nelder_mead(k, stat):
    wl, sig, truth = _events(k, 40, seed=k)
    step = 7.5 if k == 0 else 1.5
    sc = W.SimplexCfg(dims=2, stat=stat, step0=(step, step, 0.0), tol=1e-4, max_iter=400)
    got = oracle.reconstruct_simplex(wl.lrf, sc, sig)
    start = _start(wl, sig)
    gcfg = W.GridCfg(stat=stat)
    same = 0
    for e in range(len(sig)):
        x, fun, nit = _scipy_nm(wl, sc, sig[e].astype(np.float64), (start["x"][e], start["y"][e]))
        mine = oracle.node_eval(wl.lrf, gcfg, sig[e].astype(np.float64), got["x"][e], got["y"][e])[0]
        # the same minimiser: positions within a few tol and the value equal
        # to the rounding of a converged simplex.  SciPy writes the trial
        # points in another algebraic form, so on a rare event the two paths
        # part by rounding and may end in different local minima.
        dpos = max(abs(x[0] - got["x"][e]), abs(x[1] - got["y"][e]))
        same += dpos <= 5e-4 and abs(mine - fun) <= 1e-7 * max(1.0, abs(fun))
    assert same >= 0.95 * len(sig), same


@pytest.mark.parametrize("far", [False, True])
def test_same_path_as_scipy_nelder_mead(far):
    # after k iterations both implementations hold the same best vertex,
    # and they stop after the same number of iterations; from the centroid,
    # and from seeds 25 mm off (long expansion runs)
    wl, sig, truth = _events(0, 30, seed=11)
    sc = W.SimplexCfg(dims=2, step0=(7.5, 7.5, 0.0), tol=1e-3, max_iter=400)
    seeds = None
    if far:
        seeds = np.zeros((len(sig), 4))
        seeds[:, :2] = truth["pos"][:, :2] + np.array([25.0, -25.0])
        sc = W.SimplexCfg(**{**sc.__dict__, "start": 2, "step0": (2.0, 2.0, 0.0)})
        start = {"x": seeds[:, 0], "y": seeds[:, 1]}
    else:
        start = _start(wl, sig)
    full = oracle.reconstruct_simplex(wl.lrf, sc, sig, seeds=seeds)
    # SciPy counts from 1 (its result reports one more than the loop passes)
    # and runs maxiter - 1 passes
    same_it = 0
    for e in range(len(sig)):
        x, fun, nit = _scipy_nm(wl, sc, sig[e].astype(np.float64), (start["x"][e], start["y"][e]))
        same_it += nit - 1 == full["iters"][e]
    assert same_it >= 0.9 * len(sig), same_it
    for k in (2, 5, 9, 14):
        got = oracle.reconstruct_simplex(wl.lrf, W.SimplexCfg(**{**sc.__dict__, "max_iter": k}),
                                         sig, seeds=seeds)
        same = 0
        for e in range(len(sig)):
            x, fun, nit = _scipy_nm(wl, W.SimplexCfg(**{**sc.__dict__, "max_iter": k + 1}),
                                    sig[e].astype(np.float64), (start["x"][e], start["y"][e]))
            same += max(abs(x[0] - got["x"][e]), abs(x[1] - got["y"][e])) <= 1e-9
        assert same >= 0.9 * len(sig), (k, same)


def test_rz_three_axes_same_minimiser_as_scipy():
    wl, sig, truth = _events(2, 6, seed=7)
    sc = W.SimplexCfg(dims=3, step0=(10.0, 10.0, 50.0 / 6), z_start=25.0, tol=1e-4, max_iter=600)
    got = oracle.reconstruct_simplex(wl.lrf, sc, sig)
    start = _start(wl, sig)
    gcfg = W.GridCfg(stat=0)
    for e in range(len(sig)):
        x, fun, nit = _scipy_nm(wl, sc, sig[e].astype(np.float64),
                                (start["x"][e], start["y"][e], 25.0))
        mine = oracle.node_eval(wl.lrf, gcfg, sig[e].astype(np.float64), got["x"][e],
                                got["y"][e], got["z"][e])[0]
        assert abs(mine - fun) <= 1e-7 * max(1.0, abs(fun)), (e, mine, fun)


def test_best_value_never_increases():
    wl, sig, truth = _events(0, 25, seed=3)
    gcfg = W.GridCfg()
    prev = None
    for k in range(0, 60, 3):
        r = oracle.reconstruct_simplex(wl.lrf, W.SimplexCfg(max_iter=k), sig)
        st = np.array([oracle.node_eval(wl.lrf, gcfg, sig[e].astype(np.float64), r["x"][e],
                                        r["y"][e])[0] for e in range(len(sig))])
        if prev is not None:
            assert np.all(st <= prev + 1e-9 * np.abs(prev)), k
        prev = st


def test_noiseless_events_reach_the_truth():
    wl, sig, truth = _events(0, 200, seed=4, noiseless=True)
    r = oracle.reconstruct_simplex(wl.lrf, W.SimplexCfg(tol=1e-5, max_iter=400), sig)
    pos = truth["pos"]
    d = np.maximum(np.abs(r["x"] - pos[:, 0]), np.abs(r["y"] - pos[:, 1]))
    inner = np.hypot(pos[:, 0], pos[:, 1]) < 45.0
    assert np.mean(d[inner] <= 1e-3) >= 0.99, np.sort(d[inner])[-5:]
    np.testing.assert_allclose(r["E"][inner], truth["A"][inner], rtol=1e-5)


def test_flat_likelihood_shrinks_onto_the_start():
    lrf = W.axial_lrf(np.array([[3.0, -2.0]]))
    sc = W.SimplexCfg(step0=(7.5, 7.5, 0.0), tol=1e-3)
    r = oracle.reconstruct_simplex(lrf, sc, np.array([[57.0]]))
    assert r["x"][0] == 3.0 and r["y"][0] == -2.0
    k = math.ceil(math.log2(7.5 / 1e-3))
    # each iteration: reflection, inside contraction, shrink of two vertices
    assert r["iters"][0] == k and r["evals"][0] == 3 + 4 * k
    assert r["lnl"][0] == pytest.approx(57 * math.log(57) - 57, rel=1e-13)


def test_zero_iterations_and_status_flags():
    wl, sig, truth = _events(0, 6, seed=5)
    # no iteration: the best vertex of the initial simplex (start, start +
    # step0 along x, start + step0 along y; lowest value, earliest on ties)
    r0 = oracle.reconstruct_simplex(wl.lrf, W.SimplexCfg(max_iter=0), sig)
    g0 = oracle.reconstruct(wl.lrf, W.GridCfg(iterations=0), sig)
    gcfg = W.GridCfg()
    for e in range(len(sig)):
        vs = [(g0["x"][e], g0["y"][e]), (g0["x"][e] + 7.5, g0["y"][e]),
              (g0["x"][e], g0["y"][e] + 7.5)]
        f = [oracle.node_eval(wl.lrf, gcfg, sig[e].astype(np.float64), *v)[0] for v in vs]
        assert (r0["x"][e], r0["y"][e]) == vs[int(np.argmin(f))]
    assert np.all(r0["iters"] == 0)
    bad = sig.astype(np.float64).copy()
    bad[0] = 0.0
    bad[1, 3] = np.nan
    bad[2, 4] = -1.0
    r = oracle.reconstruct_simplex(wl.lrf, W.SimplexCfg(), bad)
    assert r["status"][0] == 1 and r["status"][1] == 2 and r["status"][2] == 2
    assert np.isnan(r["x"][:3]).all() and (r["status"][3:] == 0).all()
    assert (r["ndf"] == 19 - 3).all()
