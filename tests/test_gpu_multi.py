"""Persistent multi-detector launch: chunks from 19-, 61- and 127-sensor
hexagonal detectors (axial LRFs) in one launch must give exactly what one
launch per chunk gives, for every plan, and match the oracle."""
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
def stream(ants):
    geoms = W.mixed_geometries()
    grid = W.workload(3).grid
    rng = np.random.default_rng(33)
    sets = [ants.LrfSet(lrf) for lrf, _ in geoms]
    chunks, host, off = [], [], 0
    for c in range(40):
        g = int(rng.integers(0, 3))
        n = int(np.clip(rng.lognormal(np.log(300), 1.0), 20, 3000))
        lrf, rec = geoms[g]
        sig, _ = oracle.make_events(lrf, rec, n, W.streams(4000 + c))
        host.append((g, sig, off))
        chunks.append((g, torch.from_numpy(sig).cuda(), off))
        off += n
    cfg = ants.grid_cfg(grid)
    return geoms, grid, sets, [cfg, cfg, cfg], chunks, host, off


def test_multi_equals_per_chunk_launches_and_oracle(ants, stream):
    geoms, grid, sets, cfgs, chunks, host, total = stream
    print(f"[gpu] multi-detector {len(chunks)} chunks, {total} events", flush=True)
    out = to_np(ants.reconstruct_multi(sets, cfgs, chunks, total))
    torch.cuda.synchronize()
    for g, sig, off in chunks:
        one = to_np(ants.reconstruct(sets[g], cfgs[g], sig))
        for k in ("x", "y", "z", "E", "lnl", "chi2", "ndf", "status"):
            np.testing.assert_array_equal(one[k], out[k][off:off + sig.shape[0]])
    fr = []
    for g, sig, off in host:
        ref = oracle.reconstruct(geoms[g][0], grid, sig)
        got = {k: v[off:off + len(sig)] for k, v in out.items()}
        res = compare(ref, got, sig)
        fr.append(res["ok"])
    ok = np.concatenate(fr)
    assert ok.mean() >= 0.999, ok.mean()


def test_every_plan_gives_identical_results(ants, stream):
    geoms, grid, sets, cfgs, chunks, host, total = stream
    ref = to_np(ants.reconstruct_multi(sets, cfgs, chunks, total))
    for T, B, lds in ((1, 1, 1), (8, 4, 0), (128, 16, 1), (4096, 2, 0), (32, 32, 1)):
        plan = ants.Plan(T, B, lds)
        got = to_np(ants.reconstruct_multi(sets, cfgs, chunks, total, plan=plan))
        for k in ("x", "y", "E", "lnl", "status"):
            np.testing.assert_array_equal(got[k], ref[k])
    best, ms = ants.autotune_multi(sets, cfgs, chunks, min(total, 20000))
    print("autotuned plan", best.events_per_item, best.blocks_per_cu, best.table_in_lds,
          "ms", np.round(ms, 3).tolist())
    assert np.all(ms > 0) and len(ms) == 3 + 6 * len(sets)
    got = to_np(ants.reconstruct_multi(sets, cfgs, chunks, total, plan=best))
    np.testing.assert_array_equal(got["x"], ref["x"])
    # no plan: each set runs its own stored part of the tuned plan
    for _ in range(2):
        got = to_np(ants.reconstruct_multi(sets, cfgs, chunks, total))
        for k in ("x", "y", "z", "E", "lnl", "chi2", "ndf", "status"):
            np.testing.assert_array_equal(got[k], ref[k])


def test_rejects_mixed_kinds(ants, stream):
    geoms, grid, sets, cfgs, chunks, host, total = stream
    rz = ants.LrfSet(W.workload(2).lrf)
    with pytest.raises(ants.AntsError):
        ants.reconstruct_multi([sets[0], rz], [cfgs[0], ants.grid_cfg(W.workload(2).grid)],
                               chunks[:1], total)
