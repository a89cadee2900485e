"""The allocation-free seeded entry point (ants_reconstruct_seeded_noalloc)
against the allocating one, through the C ABI: network seeds and explicit
seeds, two calls in a row with the second on a smaller batch (the fixed
workspace keeps the last call's contents), and the size limit."""
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


def _same(a, b):
    for k in ("x", "y", "z", "E", "lnl", "chi2", "ndf", "status"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_noalloc_equals_allocating_entry_point(ants):
    wl = W.workload(2)
    sig, truth = oracle.make_events(wl.lrf, wl.events, 6000, W.streams(2 + 9000))
    L = ants.LrfSet(wl.lrf)
    net = ants.Mlp(37, 256, 3, seed=4, pos_scale=W.SEED_POS_SCALE, pos_offset=W.SEED_POS_OFFSET)
    refine = ants.grid_cfg(W.seeded_refine_grid())
    plain = ants.grid_cfg(wl.grid)
    d = torch.from_numpy(sig).cuda()
    rng = np.random.default_rng(5)
    seeds = np.zeros((len(sig), 4), np.float32)
    seeds[:, :3] = truth["pos"] + rng.normal(0.0, 1.6, (len(sig), 3))
    seeds[:, 3] = 2 * np.log(1.6 / 90.0)
    seeds[:30, :2] += 45.0                     # a few fallbacks
    ds = torch.from_numpy(seeds).cuda()
    # the untrained network puts seeds anywhere: many fallbacks, large lists
    for n, use_seeds in ((6000, False), (2500, False), (6000, True), (1700, True)):
        print(f"[gpu] noalloc vs allocating, n={n} seeds={use_seeds}", flush=True)
        s = ds[:n].contiguous() if use_seeds else None
        m = None if use_seeds else net
        a, na_ = ants.reconstruct_seeded(L, m, refine, plain, 2.0, d[:n].contiguous(), seeds=s)
        b, nb_ = ants.reconstruct_seeded(L, m, refine, plain, 2.0, d[:n].contiguous(), seeds=s,
                                         noalloc=True)
        torch.cuda.synchronize()
        assert na_.item() == nb_.item() and na_.item() > 0
        _same(to_np(a), to_np(b))


def test_noalloc_rejects_batches_beyond_its_workspace(ants):
    wl = W.workload(2)
    L = ants.LrfSet(wl.lrf)
    refine = ants.grid_cfg(W.seeded_refine_grid())
    plain = ants.grid_cfg(wl.grid)
    n = ants.NOALLOC_MAX_EVENTS + 1
    d = torch.zeros((n, 37), dtype=torch.float32, device="cuda")
    s = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(ants.AntsError) as ei:
        ants.reconstruct_seeded(L, None, refine, plain, 2.0, d, seeds=s, noalloc=True)
    assert ei.value.code == ants.E_ARG and "workspace" in str(ei.value)
