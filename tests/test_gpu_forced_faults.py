"""Host-forced conditions of the seeded path, checked against the oracle:
a chi2/ndf threshold of 0 (every event falls back to the plain grid) and of
infinity (none does), seeds far outside the detector and not-a-number seeds
(the refinement finds no valid node; the fallback recovers the event), a
network whose input count does not match the detector, and a truncated
network file."""
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


@pytest.fixture(scope="module")
def case(ants):
    wl = W.workload(2)
    n = 600
    sig, truth = oracle.make_events(wl.lrf, wl.events, n, W.streams(2 + 7000))
    rng = np.random.default_rng(70)
    seeds = np.zeros((n, 4), np.float32)
    seeds[:, :3] = truth["pos"][:n] + rng.normal(0, 2.0, (n, 3))
    seeds[:, 3] = 2 * math.log(2.0 / 90.0)
    return wl, ants.LrfSet(wl.lrf), sig, seeds


def _seeded(ants, L, refine, fallback, thr, sig, seeds):
    out, nfb = ants.reconstruct_seeded(L, None, ants.grid_cfg(refine), ants.grid_cfg(fallback),
                                       thr, torch.from_numpy(sig).cuda(),
                                       seeds=torch.from_numpy(seeds).cuda())
    torch.cuda.synchronize()
    return to_np(out), int(nfb.item())


def test_threshold_zero_sends_every_event_to_the_fallback(ants, case):
    wl, L, sig, seeds = case
    refine = W.seeded_refine_grid()
    print("[gpu] forced fallback, threshold 0", flush=True)
    got, nfb = _seeded(ants, L, refine, wl.grid, 0.0, sig, seeds)
    assert nfb == len(sig)
    assert np.all(got["status"] & 16)
    plain = to_np(ants.reconstruct(L, ants.grid_cfg(wl.grid), torch.from_numpy(sig).cuda()))
    torch.cuda.synchronize()
    for k in ("x", "y", "z", "E", "lnl", "chi2", "ndf"):
        np.testing.assert_array_equal(got[k], plain[k])
    ref = oracle.reconstruct_seeded(wl.lrf, refine, wl.grid, 0.0, sig, seeds.astype(np.float64))
    res = compare(ref, got, sig, three_d=True)
    assert res["frac"] >= 0.999, summary(res)


def test_infinite_threshold_keeps_every_finite_refinement(ants, case):
    # only refinements without a finite chi2 (seeds with z outside the LRF
    # domain leave the small grid without a valid node) still fall back
    wl, L, sig, seeds = case
    refine = W.seeded_refine_grid()
    got, nfb = _seeded(ants, L, refine, wl.grid, float("inf"), sig, seeds)
    only = to_np(ants.reconstruct(L, ants.grid_cfg(refine), torch.from_numpy(sig).cuda(),
                                  seeds=torch.from_numpy(seeds).cuda()))
    torch.cuda.synchronize()
    bad = ~np.isfinite(only["chi2"]) | (only["ndf"] <= 0)
    assert nfb == int(bad.sum())
    np.testing.assert_array_equal((got["status"] & 16) != 0, bad)
    for k in ("x", "y", "z", "E", "lnl", "chi2", "ndf", "status"):
        np.testing.assert_array_equal(got[k][~bad], only[k][~bad])
    ref = oracle.reconstruct_seeded(wl.lrf, refine, wl.grid, float("inf"), sig,
                                    seeds.astype(np.float64))
    res = compare(ref, got, sig, three_d=True)
    assert res["frac"] >= 0.999, summary(res)


def test_seeds_outside_the_detector_and_nan_seeds(ants, case):
    wl, L, sig, seeds = case
    s = seeds.copy()
    s[:40, :2] = (1.0e4, -1.0e4)          # far outside every LRF domain
    s[40:60, :] = np.nan                  # no seed at all
    refine = W.seeded_refine_grid()
    got, nfb = _seeded(ants, L, refine, wl.grid, 2.0, sig, s)
    ref = oracle.reconstruct_seeded(wl.lrf, refine, wl.grid, 2.0, sig, s.astype(np.float64))
    res = compare(ref, got, sig, three_d=True)
    print(summary(res), "fallbacks", nfb)
    assert res["frac"] >= 0.999, summary(res)
    assert np.all(got["status"][:60] & 16) and np.all(ref["status"][:60] & 16)
    assert np.all(np.isfinite(got["x"][:60]))


def test_network_input_count_must_match_the_detector(ants, case):
    wl, L, sig, seeds = case
    net = ants.Mlp(19, 256, 2, seed=1)
    with pytest.raises(ants.AntsError) as e:
        ants.reconstruct_seeded(L, net, ants.grid_cfg(W.seeded_refine_grid()),
                                ants.grid_cfg(wl.grid), 2.0, torch.from_numpy(sig).cuda())
    assert e.value.code == ants.E_ARG


def test_truncated_network_file(ants, tmp_path):
    net = ants.Mlp(37, 256, 2, seed=1)
    p = tmp_path / "net.bin"
    net.save(p)
    data = p.read_bytes()
    p.write_bytes(data[: len(data) // 2])
    with pytest.raises(ants.AntsError) as e:
        ants.Mlp.load(p)
    assert e.value.code == ants.E_FORMAT
    p.write_bytes(b"NOTANET!" + data[8:])
    with pytest.raises(ants.AntsError) as e:
        ants.Mlp.load(p)
    assert e.value.code == ants.E_FORMAT
    q = tmp_path / "ok.bin"
    net.save(q)
    again = ants.Mlp.load(q)
    np.testing.assert_array_equal(again.get_params(), net.get_params())
