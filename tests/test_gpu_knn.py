"""GPU k-NN reconstruction (Sec. 5.1.4) against the oracle: the same
neighbours (indices bit-exact, single-precision distances bit-exact) and
positions to single-precision rounding, on the axial, XY and r-z
detectors; ties from duplicated calibration rows; invalid events; ragged
batches.  Calls go through the C ABI."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ants():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_07247_amd import ants as A
    return A


def _case(k, m, n, seed):
    wl = W.workload(k)
    cs, ct = oracle.make_events(wl.lrf, wl.events, m, W.streams(k + 7000 + seed))
    qs, qt = oracle.make_events(wl.lrf, wl.events, n, W.streams(k + 7100 + seed))
    return wl, cs, ct["pos"].astype(np.float32), qs


def _gpu(ants, wl, cs, cpos, qs, k):
    print(f"[gpu] knn m={len(cs)} n={len(qs)} k={k} sensors={cs.shape[1]}", flush=True)
    L = ants.LrfSet(wl.lrf)
    K = ants.Knn(L, torch.from_numpy(np.ascontiguousarray(cs, np.float32)).cuda(),
                 torch.from_numpy(cpos).cuda())
    out = K.reconstruct(k, torch.from_numpy(np.ascontiguousarray(qs, np.float32)).cuda(),
                        neighbours=True)
    torch.cuda.synchronize()
    return {key: v.cpu().numpy() for key, v in out.items()}


def _check(ref, got, k):
    np.testing.assert_array_equal(got["status"], ref["status"])
    np.testing.assert_array_equal(got["idx"], ref["idx"].astype(np.int32))
    np.testing.assert_array_equal(got["dist"], ref["dist"])
    ok = ref["status"] == 0
    ref3 = np.stack([ref["x"], ref["y"], ref["z"]], 1)
    np.testing.assert_allclose(got["xyz"][ok], ref3[ok], rtol=0, atol=1e-4)
    assert np.isnan(got["xyz"][~ok]).all()


@pytest.mark.parametrize("k,m,n,kk", [(0, 20000, 1500, 16), (1, 8000, 700, 8), (2, 9000, 900, 32),
                                      (2, 5003, 257, 1)])
def test_knn_matches_oracle(ants, k, m, n, kk):
    wl, cs, cpos, qs = _case(k, m, n, kk)
    cal = oracle.KnnCal(wl.lrf, cs, cpos.astype(np.float64))
    ref = oracle.knn_reconstruct(cal, kk, qs)
    got = _gpu(ants, wl, cs, cpos, qs, kk)
    _check(ref, got, kk)


def test_knn_ties_invalid_and_ragged(ants):
    wl, cs, cpos, qs = _case(0, 1500, 300, 3)
    cs = np.concatenate([cs, cs[:700]])               # exact ties with lower indices
    cpos = np.concatenate([cpos, cpos[:700] + 1.0])
    cs[20] = 0.0
    cs[21, 4] = np.nan
    qs = qs.copy()
    qs[0] = 0.0
    qs[1, 2] = -1.0
    cal = oracle.KnnCal(wl.lrf, cs, cpos.astype(np.float64))
    ref = oracle.knn_reconstruct(cal, 12, qs)
    got = _gpu(ants, wl, cs, cpos, qs, 12)
    _check(ref, got, 12)
    assert list(got["status"][:2]) == [1, 2]
    for n in (1, 255, 257):
        part = _gpu(ants, wl, cs, cpos, qs[:n], 12)
        for key in ("xyz", "status", "idx", "dist"):
            np.testing.assert_array_equal(part[key], got[key][:n])
