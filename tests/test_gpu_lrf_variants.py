"""GPU parity of the composite and sliced LRFs (Sec. 6.1.1, 6.1.2) in the
same kernels as the other kinds: the contracting grid (ML and chi2, 2-D
composite, 3-D sliced) and the simplex search, against the FP64 oracle at
the parity bar (99.9% of events; 100% for the simplex), status bits and
ndf exact.  Calls go through the C ABI."""
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


def _composite():
    return W.composite_lrf(W.hex_array(2, 30.0)), W.EventRecipe("disc", 60.0, 500.0, 2000.0)


def _sliced():
    return (W.sliced_lrf(W.hex_array(3, 30.0), n_planes=6, nb=20, ext=130.0),
            W.EventRecipe("disc", 90.0, 500.0, 2000.0, 0.0, 50.0, True))


def _grid(ants, lrf, g, sig):
    print(f"[gpu] kind {lrf.kind} grid n={len(sig)} nodes={g.nodes} stat={g.stat}", flush=True)
    L = ants.LrfSet(lrf)
    out = ants.reconstruct(L, ants.grid_cfg(g), torch.from_numpy(sig).cuda(), path=True,
                           n_fp64=True)
    torch.cuda.synchronize()
    return to_np(out)


@pytest.mark.parametrize("which,stat,n", [("composite", 0, 3000), ("composite", 1, 1500),
                                          ("sliced", 0, 800), ("sliced", 1, 300)])
def test_grid_matches_oracle(ants, which, stat, n):
    if which == "composite":
        lrf, rec = _composite()
        g = W.GridCfg((9, 9, 1), 6, 0.5, (7.5, 7.5, 0.0), 0.0, stat=stat)
    else:
        lrf, rec = _sliced()
        g = W.GridCfg((7, 7, 7), 8, 0.5, (10.0, 10.0, 50.0 / 6.0), 25.0, stat=stat)
    sig, truth = oracle.make_events(lrf, rec, n, W.streams(8000 + lrf.kind + stat))
    ref = oracle.reconstruct(lrf, g, sig)
    gpu = _grid(ants, lrf, g, sig)
    res = compare(ref, gpu, sig, stat, three_d=g.nodes[2] > 1)
    print(summary(res), "| mean FP64 nodes/event", gpu["n_fp64"].mean())
    assert res["frac"] >= 0.999, summary(res)
    np.testing.assert_array_equal(gpu["ndf"], ref["ndf"])


def test_grid_decisions_equal_all_fp64(ants):
    # the FP32 screen's bound holds for the new kinds: unbounded margin
    # (every node in FP64) gives the same results
    for lrf, rec, g in ((*_composite(), W.GridCfg((9, 9, 1), 6, 0.5, (7.5, 7.5, 0.0), 0.0)),
                        (*_sliced(), W.GridCfg((7, 7, 7), 8, 0.5, (10.0, 10.0, 50.0 / 6.0),
                                               25.0))):
        sig, _ = oracle.make_events(lrf, rec, 400, W.streams(8100 + lrf.kind))
        L = ants.LrfSet(lrf)
        d = torch.from_numpy(sig).cuda()
        a = to_np(ants.reconstruct(L, ants.grid_cfg(g), d, path=True))
        b = to_np(ants.reconstruct(L, ants.grid_cfg(g, 1e30), d, path=True))
        torch.cuda.synchronize()
        for k in ("path", "x", "y", "z", "E", "lnl", "chi2", "status"):
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.mark.parametrize("which", ["composite", "sliced"])
def test_simplex_matches_oracle(ants, which):
    if which == "composite":
        lrf, rec = _composite()
        sc = W.SimplexCfg(dims=2, step0=(7.5, 7.5, 0.0), tol=1e-3, max_iter=300)
    else:
        lrf, rec = _sliced()
        sc = W.SimplexCfg(dims=3, step0=(10.0, 10.0, 50.0 / 6.0), z_start=25.0, tol=1e-3,
                          max_iter=400)
    sig, truth = oracle.make_events(lrf, rec, 600, W.streams(8200 + lrf.kind))
    ref = oracle.reconstruct_simplex(lrf, sc, sig)
    print(f"[gpu] simplex kind {lrf.kind}", flush=True)
    L = ants.LrfSet(lrf)
    gpu = to_np(ants.reconstruct_simplex(L, ants.simplex_cfg(sc), torch.from_numpy(sig).cuda()))
    torch.cuda.synchronize()
    res = compare(ref, gpu, sig, 0, three_d=sc.dims == 3)
    assert res["ok"].all(), summary(res)
    np.testing.assert_array_equal(gpu["iters"], ref["iters"])


def test_generator_draws_from_the_new_kinds(ants):
    # device generator against the oracle's twin (same Philox streams)
    for lrf, rec in (_composite(), _sliced()):
        L = ants.LrfSet(lrf)
        print(f"[gpu] generator kind {lrf.kind}", flush=True)
        sig, truth = ants.generate(L, ants.gen_cfg(rec), 500, 99)
        torch.cuda.synchronize()
        ext = rec.extent
        ref_sig, ref_truth = oracle.generate(lrf, 0, ext, rec.z_lo, rec.z_hi if rec.three_d else
                                             rec.z_lo, rec.e_lo, rec.e_hi, 500, 99)
        np.testing.assert_allclose(truth.cpu().numpy(), ref_truth, rtol=1e-6, atol=1e-4)
        same = sig.cpu().numpy() == ref_sig.astype(np.float32)
        assert same.mean() >= 0.999, same.mean()
