"""GPU parity of the variable-metric search (Sec. 5.1.2.1: the Migrad-style
method, FP64) against the FP64 oracle: 99.9% of the events that end within one sensor
spacing of the array (99.5% of all) with every coordinate within 1e-3 mm,
E, lnL and chi2 within 1e-5 of their scale, equal status and ndf, and the same step and evaluation counts on 95% of events;
plus the status cases and argument errors.  Calls go through the
C ABI."""
import numpy as np
import pytest

import oracle
import workloads as W

from parity import compare, summary, to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ants():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_07247_amd import ants as A
    return A


def _run(ants, lrf, mc, sig, seeds=None):
    print(f"[gpu] migrad n={len(sig)} dims={mc.dims} stat={mc.stat} start={mc.start}",
          flush=True)
    L = ants.LrfSet(lrf)
    d = torch.from_numpy(np.ascontiguousarray(sig, np.float32)).cuda()
    s = torch.from_numpy(np.ascontiguousarray(seeds, np.float32)).cuda() if seeds is not None \
        else None
    out = ants.reconstruct_migrad(L, ants.migrad_cfg(mc), d, seeds=s, n_eval=True)
    torch.cuda.synchronize()
    return to_np(out)


CASES = [  # workload, n, dims, stat, start, step0, z_start
    (0, 3000, 2, 0, 0, (7.5, 7.5, 0.0), 0.0),
    (0, 2000, 2, 1, 1, (7.5, 7.5, 0.0), 0.0),
    (1, 1500, 2, 0, 0, (1.5, 1.5, 0.0), 0.0),
    (1, 1000, 2, 1, 0, (1.5, 1.5, 0.0), 0.0),
    (2, 2000, 3, 0, 0, (10.0, 10.0, 8.0), 25.0),
    (2, 1000, 3, 1, 0, (10.0, 10.0, 8.0), 25.0),
    (2, 2000, 2, 0, 0, (10.0, 10.0, 0.0), 25.0),
]


@pytest.mark.parametrize("k,n,dims,stat,start,step0,z0", CASES)
def test_migrad_matches_oracle(ants, k, n, dims, stat, start, step0, z0):
    wl = W.workload(k)
    sig, truth = oracle.make_events(wl.lrf, wl.events, n, W.streams(k + 6100))
    # a tight EDM tolerance: the two searches then stop close enough that the
    # energy and statistics at their end points agree to the output
    # tolerances (near a wall of the z domain the energy moves by ~1e-4 per
    # micrometre of z)
    mc = W.MigradCfg(dims=dims, stat=stat, start=start, step0=step0, z_start=z0, edm_tol=1e-10,
                     max_iter=200)
    ref = oracle.reconstruct_migrad(wl.lrf, mc, sig)
    gpu = _run(ants, wl.lrf, mc, sig)
    res = compare(ref, gpu, sig, stat, three_d=dims == 3)
    same_it = (gpu["iters"] == ref["iters"]) & (gpu["n_fp64"] == ref["evals"])
    # events whose search ends more than one sensor spacing beyond the array
    # lie where the statistic is nearly flat: paths there are long and
    # last-bit differences of the statistic take the two searches apart
    sxy = np.asarray(wl.lrf.sxy, np.float64)
    c = sxy.mean(0)
    spacing = np.min([np.hypot(*(sxy[i] - sxy[j])) for i in range(len(sxy))
                      for j in range(i)])
    reach = np.max(np.hypot(*(sxy - c).T)) + spacing
    with np.errstate(invalid="ignore"):
        inside = ~(np.hypot(ref["x"] - c[0], ref["y"] - c[1]) > reach)
    frac_in = res["ok"][inside].mean()
    print(summary(res), "| inside the array", inside.mean(), frac_in, "| steps equal",
          same_it.mean(), "mean", ref["iters"].mean(), "evals", ref["evals"].mean())
    assert frac_in >= 0.999 and res["frac"] >= 0.995, summary(res)
    # the step count follows comparisons of FP64 statistics summed in a
    # different order (EDM against its tolerance, the line search's
    # sufficient decrease): near a threshold a last-bit difference moves
    # the stop by a step, within the position tolerance above
    assert (same_it | ~res["ok"]).mean() >= 0.95
    np.testing.assert_array_equal(gpu["ndf"], ref["ndf"])


def test_seed_start_status_cases_and_errors(ants):
    wl = W.workload(2)
    sig, truth = oracle.make_events(wl.lrf, wl.events, 400, W.streams(6200))
    sig = sig.copy()
    sig[0, :] = 0.0
    sig[1, 2] = -1.0
    sig[2, 4] = np.nan
    seeds = np.zeros((400, 4))
    seeds[:, :3] = truth["pos"] + np.random.default_rng(1).normal(0.0, 2.0, (400, 3))
    seeds[:, 2] = np.clip(seeds[:, 2], 1.0, 49.0)
    mc = W.MigradCfg(dims=3, stat=0, start=2, step0=(10.0, 10.0, 8.0), z_start=25.0,
                     edm_tol=1e-10)
    ref = oracle.reconstruct_migrad(wl.lrf, mc, sig, seeds=seeds)
    gpu = _run(ants, wl.lrf, mc, sig, seeds)
    np.testing.assert_array_equal(gpu["status"][:3], ref["status"][:3])
    assert np.isnan(gpu["x"][:3]).all()
    res = compare(ref, gpu, sig, 0, three_d=True)
    assert res["frac"] >= 0.995, summary(res)
    L = ants.LrfSet(wl.lrf)
    d = torch.from_numpy(np.ascontiguousarray(sig, np.float32)).cuda()
    ds = torch.from_numpy(np.ascontiguousarray(seeds, np.float32)).cuda()
    for bad in (dict(h=0.0), dict(edm_tol=-1.0), dict(dims=4), dict(max_iter=-1),
                dict(step0=(0.0, 1.0, 1.0)), dict(stat=7)):
        c = W.MigradCfg(**{**mc.__dict__, **bad})
        with pytest.raises(ants.AntsError) as ei:
            ants.reconstruct_migrad(L, ants.migrad_cfg(c), d, seeds=ds)
        assert ei.value.code == ants.E_ARG, bad
    with pytest.raises(ants.AntsError):                 # seed start without seeds
        ants.reconstruct_migrad(L, ants.migrad_cfg(mc), d, seeds=None)
