"""GPU parity: the HIP contracting-grid library against the FP64 oracle on
the same seeded inputs (Sec. 5.1.2.2).  Bar: 99.9% of events with every
coordinate within 1e-3 mm and lnL / chi2 within 1e-5 of their scale,
identical status bits and ndf; mismatches are classified as near ties or
other.  Calls go through the C ABI (ctypes binding)."""
import math

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


def _events(k, n, seed_off=0, noiseless=False):
    wl = W.workload(k)
    sig, truth = oracle.make_events(wl.lrf, wl.events, n, W.streams(k + 1000 * seed_off),
                                    noiseless=noiseless)
    return wl, sig, truth


def _run(ants, wl, sig, grid=None, seeds=None, screen_scale=0.0, lrf=None):
    grid = grid or wl.grid
    print(f"[gpu] {wl.name} n={len(sig)} stat={grid.stat} nodes={grid.nodes} K={grid.iterations}",
          flush=True)
    L = lrf or ants.LrfSet(wl.lrf)
    d = torch.from_numpy(np.ascontiguousarray(sig, np.float32)).cuda()
    s = torch.from_numpy(np.ascontiguousarray(seeds, np.float32)).cuda() if seeds is not None else None
    out = ants.reconstruct(L, ants.grid_cfg(grid, screen_scale), d, seeds=s, path=True,
                           n_fp64=True)
    torch.cuda.synchronize()
    return to_np(out)


@pytest.mark.parametrize("k,n,stat", [(0, 10_000, 0), (0, 3_000, 1), (1, 2_000, 0),
                                      (1, 2_000, 1), (2, 3_000, 0), (2, 1_000, 1)])
def test_parity_against_oracle(ants, k, n, stat):
    wl, sig, truth = _events(k, n)
    grid = W.GridCfg(**{**wl.grid.__dict__, "stat": stat})
    ref = oracle.reconstruct(wl.lrf, grid, sig)
    gpu = _run(ants, wl, sig, grid)
    res = compare(ref, gpu, sig, stat, three_d=grid.nodes[2] > 1)
    print(summary(res), "| mean FP64 nodes/event", gpu["n_fp64"].mean())
    assert res["frac"] >= 0.999, summary(res)
    np.testing.assert_array_equal(gpu["ndf"], ref["ndf"])


@pytest.mark.parametrize("k,nodes,stat,n", [(0, (5, 5, 1), 0, 3_000), (0, (5, 5, 1), 1, 2_000),
                                             (0, (3, 3, 1), 0, 2_000), (1, (5, 5, 1), 0, 1_000),
                                             (1, (3, 3, 1), 1, 1_000), (2, (3, 3, 3), 0, 2_000),
                                             (2, (3, 3, 3), 1, 1_000), (2, (5, 5, 1), 0, 1_000),
                                             (2, (5, 5, 3), 0, 1_000), (2, (3, 3, 9), 0, 1_000),
                                             (2, (9, 9, 3), 0, 500), (0, (7, 11, 1), 0, 2_000),
                                             (1, (11, 11, 1), 0, 1_000), (1, (9, 9, 1), 1, 1_000)])
def test_parity_small_grids_split_sensor_loop(ants, k, nodes, stat, n):
    # grids of <= 32 nodes run the screen with the sensors split between the
    # two halves of a wave (odd and even sensor counts, both statistics);
    # r-z grids with 2..8 planes run the column-factored screen (sensor
    # groups per column for 3x3 and 5x5 columns, two passes for 9x9), more
    # planes the per-node screen; several tiles with at most 32 nodes in the
    # last one (7x11, 9x9 with 3 planes) split only the last tile (ML)
    wl, sig, truth = _events(k, n, seed_off=2)
    grid = W.GridCfg(**{**wl.grid.__dict__, "nodes": nodes, "stat": stat,
                        "iterations": wl.grid.iterations + 2})
    ref = oracle.reconstruct(wl.lrf, grid, sig)
    gpu = _run(ants, wl, sig, grid)
    res = compare(ref, gpu, sig, stat, three_d=nodes[2] > 1)
    print(summary(res), "| mean FP64 nodes/event", gpu["n_fp64"].mean())
    assert res["frac"] >= 0.999, summary(res)
    full = _run(ants, wl, sig[:500], grid, screen_scale=1e30)
    np.testing.assert_array_equal(gpu["path"][:500], full["path"])


def test_screen_is_sound_full_fp64_gives_same_answers(ants):
    # with an unbounded screening margin every valid node is decided in FP64;
    # the default margin must reach exactly the same decisions
    wl, sig, truth = _events(2, 1500, seed_off=1)
    a = _run(ants, wl, sig)
    b = _run(ants, wl, sig, screen_scale=1e30)
    assert (b["n_fp64"] > 50 * a["n_fp64"].mean()).mean() > 0.9
    np.testing.assert_array_equal(a["path"], b["path"])
    for key in ("x", "y", "z", "E", "lnl", "chi2"):
        np.testing.assert_array_equal(a[key], b[key])


def test_noiseless_events_land_within_final_step(ants):
    wl, sig, truth = _events(2, 1000, seed_off=2, noiseless=True)
    gpu = _run(ants, wl, sig)
    sf = wl.grid.final_step
    pos = truth["pos"]
    d = np.abs(np.stack([gpu["x"] - pos[:, 0], gpu["y"] - pos[:, 1], gpu["z"] - pos[:, 2]], 1))
    inside = (d <= np.array(sf) + 1e-4).all(1)
    assert inside.mean() >= 0.995, inside.mean()


def test_ragged_batches_and_start_options(ants):
    wl, sig, truth = _events(0, 1000, seed_off=3)
    L = ants.LrfSet(wl.lrf)
    for n in (1, 3, 63, 64, 65, 257):
        ref = oracle.reconstruct(wl.lrf, wl.grid, sig[:n])
        gpu = _run(ants, wl, sig[:n], lrf=L)
        res = compare(ref, gpu, sig[:n])
        assert res["ok"].all(), (n, summary(res))
    g = W.GridCfg(**{**wl.grid.__dict__, "start": 1})
    ref = oracle.reconstruct(wl.lrf, g, sig)
    res = compare(ref, _run(ants, wl, sig, g, lrf=L), sig)
    assert res["frac"] >= 0.999, summary(res)
    seeds = np.zeros((len(sig), 4))
    seeds[:, :2] = truth["pos"][:, :2] + 0.8
    g = W.GridCfg(**{**wl.grid.__dict__, "start": 2, "step0": (1.0, 1.0, 0.0)})
    ref = oracle.reconstruct(wl.lrf, g, sig, seeds=seeds)
    res = compare(ref, _run(ants, wl, sig, g, seeds=seeds, lrf=L), sig)
    assert res["frac"] >= 0.999, summary(res)
    for K in (0, 1):
        g = W.GridCfg(**{**wl.grid.__dict__, "iterations": K})
        ref = oracle.reconstruct(wl.lrf, g, sig[:300])
        res = compare(ref, _run(ants, wl, sig[:300], g, lrf=L), sig[:300])
        assert res["ok"].all(), (K, summary(res))


def test_empty_batch_and_bad_events(ants):
    wl, sig, truth = _events(0, 40, seed_off=4)
    L = ants.LrfSet(wl.lrf)
    empty = torch.empty((0, 19), dtype=torch.float32, device="cuda")
    out = ants.reconstruct(L, ants.grid_cfg(wl.grid), empty)
    torch.cuda.synchronize()
    assert out["x"].numel() == 0
    sig = sig.copy()
    sig[3] = 0.0
    sig[5, 2] = np.nan
    sig[7, 11] = -2.0
    sig[9, 0] = np.inf
    ref = oracle.reconstruct(wl.lrf, wl.grid, sig)
    gpu = _run(ants, wl, sig, lrf=L)
    assert list(gpu["status"][[3, 5, 7, 9]]) == [1, 2, 2, 2]
    res = compare(ref, gpu, sig)
    assert res["ok"].all(), summary(res)


def test_passive_sensors(ants):
    wl, sig, truth = _events(2, 800, seed_off=5)
    lrf = W.rz_lrf(wl.lrf.sxy)
    lrf.active = np.ones(37, np.uint8)
    lrf.active[[0, 18, 30]] = 0
    sig = sig.copy()
    sig[:, 18] = np.nan           # ignored: passive
    wlp = W.Workload(2, "hex37-rz-passive", lrf, wl.grid, wl.events, 800)
    ref = oracle.reconstruct(lrf, wl.grid, sig)
    gpu = _run(ants, wlp, sig)
    res = compare(ref, gpu, sig, three_d=True)
    assert res["frac"] >= 0.999, summary(res)
    assert (gpu["ndf"] == 34 - 4).all()
    lrf.active[:] = 0
    gpu = _run(ants, W.Workload(2, "all-passive", lrf, wl.grid, wl.events, 10), sig[:10])
    assert (gpu["status"] == 4).all()


def test_degenerate_ties_follow_lowest_index(ants):
    # a constant LRF makes every node equally good: the FP64 values differ
    # only by rounding, within the tie tolerance, so the corner node (index 0)
    # wins every iteration, as in the oracle, and TIE is set
    sxy = W.hex_array(2, 30.0)
    lrf = W.axial_lrf(sxy)
    lrf.coef = np.ones_like(lrf.coef)
    lrf.hi = (1000.0, 0.0)
    for stat in (0, 1):
        g = W.GridCfg((9, 9, 1), 4, 0.5, (2.0, 2.0, 0.0), 0.0, stat=stat)
        sig = np.random.default_rng(9).poisson(40.0, size=(70, 19)).astype(np.float32)
        ref = oracle.reconstruct(lrf, g, sig)
        gpu = _run(ants, W.Workload(0, "constant-lrf", lrf, g, None, 70), sig, g)
        assert np.all(ref["path"] == 0) and np.all(ref["status"] & 32)
        np.testing.assert_array_equal(gpu["path"], ref["path"])
        np.testing.assert_array_equal(gpu["status"], ref["status"])
        res = compare(ref, gpu, sig, stat)
        assert res["ok"].all(), summary(res)


@pytest.mark.parametrize("stat", [0, 1])
def test_single_sensor_ring_of_ties(ants, stat):
    # one sensor: every node inside the LRF domain ties; the grid reaches
    # past the domain, so each iteration's winner is the lowest index inside
    # the disc r <= 150 mm around the sensor (a node on the far side of the
    # FP32 screen's error bound included)
    lrf = W.axial_lrf(np.array([[0.0, 0.0]]))
    g = W.GridCfg((9, 9, 1), 3, 0.5, (32.0, 32.0, 0.0), 0.0, stat=stat)
    sig = np.random.default_rng(11).poisson(60.0, size=(40, 1)).astype(np.float32) + 1
    ref = oracle.reconstruct(lrf, g, sig)
    gpu = _run(ants, W.Workload(0, "one-sensor", lrf, g, None, 40), sig, g)
    assert np.all(ref["path"][:, 0] == 2) and np.all(ref["status"] & 32)
    np.testing.assert_array_equal(gpu["path"], ref["path"])
    np.testing.assert_array_equal(gpu["status"], ref["status"])
    res = compare(ref, gpu, sig, stat)
    assert res["ok"].all(), summary(res)


def test_full_size_r_z_batch_sampled_against_oracle(ants):
    # 10 M events, the benchmark's launch: rows repeat a 99,991-event base set
    wl, base, truth = _events(2, 99_991, seed_off=6)
    n = 10_000_000
    print("[gpu] full-size r-z batch", n, flush=True)
    dbase = torch.from_numpy(base).cuda()
    reps = -(-n // len(base))
    d = dbase.repeat(reps, 1)[:n].contiguous()
    del dbase
    L = ants.LrfSet(wl.lrf)
    out = ants.reconstruct(L, ants.grid_cfg(wl.grid), d)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    idx = np.unique(np.concatenate([rng.integers(0, n, 12_000), [0, n - 1, n // 2]]))
    got = {k: v[torch.from_numpy(idx).cuda()].cpu().numpy() for k, v in out.items()}
    rows = base[idx % len(base)]
    ref = oracle.reconstruct(wl.lrf, wl.grid, rows)
    res = compare(ref, got, rows, three_d=True)
    assert res["frac"] >= 0.999, summary(res)
    del d, out
    torch.cuda.empty_cache()
