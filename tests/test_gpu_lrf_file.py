"""LRF-set files through the C ABI on the GPU: a set saved and loaded again,
and a descriptor written by ants_lrf_write and loaded, reconstruct the same
events bit for bit as the set they came from (passive sensors kept)."""
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


@pytest.mark.parametrize("k", [0, 1, 2])
def test_saved_and_loaded_sets_reconstruct_identically(ants, k, tmp_path):
    wl = W.workload(k)
    m = wl.lrf
    m.active = np.ones(m.sxy.shape[0], np.uint8)
    m.active[2] = 0
    sig, _ = oracle.make_events(m, wl.events, 700, W.streams(k + 4000))
    d = torch.from_numpy(sig).cuda()
    cfg = ants.grid_cfg(wl.grid)
    print(f"[gpu] lrf file round trip, workload {k}", flush=True)
    L = ants.LrfSet(m)
    ref = to_np(ants.reconstruct(L, cfg, d))
    L.save(str(tmp_path / "a.lrf"))
    ants.write_lrf(m, str(tmp_path / "b.lrf"))
    assert (tmp_path / "a.lrf").read_bytes() == (tmp_path / "b.lrf").read_bytes()
    for f in ("a.lrf", "b.lrf"):
        L2 = ants.LrfSet.load(str(tmp_path / f))
        assert (L2.n_sensors, L2.n_active, L2.kind) == (L.n_sensors, L.n_active, L.kind)
        got = to_np(ants.reconstruct(L2, cfg, d))
        torch.cuda.synchronize()
        for key in ("x", "y", "z", "E", "lnl", "chi2", "ndf", "status"):
            np.testing.assert_array_equal(got[key], ref[key], err_msg=key)
