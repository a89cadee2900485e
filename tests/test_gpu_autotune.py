"""Per-set launch plans of the contracting grid (ants_autotune /
ants_set_plan): every plan gives the same reconstruction bit for bit, the
tuner stores its choice in the set and reconstruct uses it, and invalid
plans are rejected.  Calls go through the C ABI."""
import itertools

import numpy as np
import pytest

import oracle
import workloads as W

from parity import to_np

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ants():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_07247_amd import ants as A
    return A


KEYS = ("x", "y", "z", "E", "lnl", "chi2", "ndf", "status", "path")


def _case(k, n, refine=False, stat=0):
    wl = W.workload(k)
    sig, truth = oracle.make_events(wl.lrf, wl.events, n, W.streams(k + 9500))
    g = W.GridCfg(**{**wl.grid.__dict__, "stat": stat})
    seeds = None
    if refine:
        g = W.seeded_refine_grid()
        rng = np.random.default_rng(3)
        seeds = np.zeros((n, 4), np.float32)
        seeds[:, :3] = truth["pos"] + rng.normal(0.0, 1.6, (n, 3))
        seeds[:, 3] = 2 * np.log(1.6 / 90.0)
    return wl, sig, seeds, g


# XY (workload 1): the screen from y-collapsed rows staged in LDS against
# the per-node screen reading the coefficients through the cache; both are
# sound, so every decision and output agrees
@pytest.mark.parametrize("k,n,refine,stat", [(0, 3000, False, 0), (2, 1500, False, 0),
                                             (2, 4000, True, 0), (1, 1500, False, 0),
                                             (1, 1000, False, 1)])
def test_every_plan_reconstructs_identically(ants, k, n, refine, stat):
    wl, sig, seeds, g = _case(k, n, refine, stat)
    print(f"[gpu] plans workload {k} n={n} refine={refine} stat={stat}", flush=True)
    L = ants.LrfSet(wl.lrf)
    cfg = ants.grid_cfg(g)
    d = torch.from_numpy(sig).cuda()
    s = torch.from_numpy(seeds).cuda() if seeds is not None else None
    ref = to_np(ants.reconstruct(L, cfg, d, seeds=s, path=True))
    for wpb, bpc, screen in itertools.product((4, 2, 1), (0, 2, 5), (0, 1)):
        ants.set_plan(L, cfg, ants.GridPlan(wpb, bpc, screen))
        got = to_np(ants.reconstruct(L, cfg, d, seeds=s, path=True))
        for key in KEYS:
            np.testing.assert_array_equal(got[key], ref[key], err_msg=f"{key} {wpb} {bpc} {screen}")
    ants.set_plan(L, cfg, None)
    best, ms = ants.autotune(L, cfg, d, seeds=s)
    print("tuned", best.waves_per_block, best.blocks_per_cu, best.screen, np.round(ms, 3).tolist())
    cands = 12 if (k == 2 and stat == 0) or k == 1 else 6
    assert (ms[:cands] > 0).all() and (ms[cands:] == 0).all()
    got = to_np(ants.reconstruct(L, cfg, d, seeds=s, path=True))
    for key in KEYS:
        np.testing.assert_array_equal(got[key], ref[key], err_msg=key)


def test_seeded_path_uses_the_stored_plans(ants):
    wl, sig, seeds, g = _case(2, 3000, True)
    L = ants.LrfSet(wl.lrf)
    refine, plain = ants.grid_cfg(g), ants.grid_cfg(wl.grid)
    d = torch.from_numpy(sig).cuda()
    s = torch.from_numpy(seeds).cuda()
    a, na_ = ants.reconstruct_seeded(L, None, refine, plain, 2.0, d, seeds=s)
    a = to_np(a)
    ants.set_plan(L, refine, ants.GridPlan(1, 2, 1))
    ants.set_plan(L, plain, ants.GridPlan(2, 0, 1))
    b, nb_ = ants.reconstruct_seeded(L, None, refine, plain, 2.0, d, seeds=s)
    b = to_np(b)
    assert na_.item() == nb_.item()
    for key in KEYS[:-1]:
        np.testing.assert_array_equal(a[key], b[key], err_msg=key)


def test_invalid_plans_are_rejected(ants):
    wl = W.workload(0)
    L = ants.LrfSet(wl.lrf)
    cfg = ants.grid_cfg(wl.grid)
    for bad in ((3, 0, 0), (0, 0, 0), (4, -1, 0), (4, 33, 0), (4, 0, 2)):
        with pytest.raises(ants.AntsError) as ei:
            ants.set_plan(L, cfg, ants.GridPlan(*bad))
        assert ei.value.code == ants.E_ARG
