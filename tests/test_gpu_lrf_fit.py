"""LRF fit from events on the GPU (Sec. 6, 6.2, 8) against the FP64 oracle
fit on the same inputs, and the iterative procedure (reconstruct, refit,
repeat) started from a wrong LRF.  Calls go through the C ABI."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import lrf_fit as F

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ants():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_07247_amd import ants as A
    return A


def _inputs(g, n, seed, noiseless=False):
    """Oracle-drawn events, true positions and LRF scale (E_tot / S) as the
    reconstruction record, rounded to FP32 as the library's outputs are."""
    lrf, rec = W.mixed_geometries()[g]
    sig, truth = oracle.generate(lrf, 0, rec.extent, 0.0, 0.0, rec.e_lo, rec.e_hi, n, seed,
                                 noiseless=noiseless)
    S = oracle.lrf_values(lrf, truth[:, :3]) @ np.asarray(lrf.gain, np.float64)
    rng = np.random.default_rng(seed)
    r = {"x": truth[:, 0].astype(np.float32), "y": truth[:, 1].astype(np.float32),
         "E": (truth[:, 3] / S).astype(np.float32),
         "chi2": rng.uniform(0.0, 60.0, n).astype(np.float32),
         "ndf": np.full(n, lrf.sxy.shape[0] - 3, np.int32),
         "status": np.where(rng.uniform(size=n) < 0.05, 8, 0).astype(np.int32)}
    return lrf, sig.astype(np.float32), r


def _dev(ants, r):
    n = len(r["x"])
    d = {k: torch.from_numpy(v).cuda() for k, v in r.items()}
    for k in ("z", "lnl"):
        d[k] = torch.zeros(n, dtype=torch.float32, device="cuda")
    return d


@pytest.mark.parametrize("g,chi2cut", [(1, 0.0), (1, 1.5), (2, 0.0), (0, 0.0)])
def test_fit_matches_oracle(ants, g, chi2cut):
    lrf, sig, r = _inputs(g, 20_000, 40 + g)
    print(f"[gpu] LRF fit, {lrf.sxy.shape[0]} sensors, chi2/ndf cut {chi2cut}", flush=True)
    L = ants.LrfSet(lrf)
    nb, lo, hi = lrf.nb[0], lrf.lo[0], lrf.hi[0]
    coef, counts = ants.fit_axial_lrf(L, ants.fit_cfg(nb, lo, hi, 1e-9, chi2cut),
                                      torch.from_numpy(sig).cuda(), _dev(ants, r))
    torch.cuda.synchronize()
    use = F.event_mask(r["E"], r["status"], r["chi2"], r["ndf"], chi2cut if chi2cut > 0 else None)
    x64 = {k: r[k].astype(np.float64) for k in ("x", "y", "E")}
    ref = F.fit_axial_shared(lrf.sxy, lrf.gain, lrf.active, sig.astype(np.float64), x64["x"],
                             x64["y"], x64["E"], use, nb, lo, hi, ridge=1e-9)
    _, _, npairs = F.normal_equations(lrf.sxy, lrf.gain, lrf.active, sig.astype(np.float64),
                                      x64["x"], x64["y"], x64["E"], use, nb, lo, hi)
    got = coef.cpu().numpy()
    # FP64 sums in another order: relative agreement far below the fit's noise
    assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref)), np.max(np.abs(got - ref))
    assert counts.cpu().tolist() == [int(use.sum()), npairs]
    # same inputs, same bits
    again, _ = ants.fit_axial_lrf(L, ants.fit_cfg(nb, lo, hi, 1e-9, chi2cut),
                                  torch.from_numpy(sig).cuda(), _dev(ants, r))
    np.testing.assert_array_equal(again.cpu().numpy(), got)


def test_fit_recovers_spline_from_noiseless_events(ants):
    lrf, sig, r = _inputs(1, 20_000, 7, noiseless=True)
    r["status"][:] = 0
    L = ants.LrfSet(lrf)
    coef, _ = ants.fit_axial_lrf(L, ants.fit_cfg(lrf.nb[0], lrf.lo[0], lrf.hi[0], 0.0),
                                 torch.from_numpy(sig).cuda(), _dev(ants, r))
    ref = np.asarray(lrf.coef).reshape(-1)
    # inputs rounded to FP32 (positions, scale, signals): agreement to ~1e-6
    assert np.max(np.abs(coef.cpu().numpy() - ref)) < 2e-5 * np.max(np.abs(ref))


def test_empty_fit_gives_nan(ants):
    lrf, sig, r = _inputs(0, 64, 9)
    r["status"][:] = 8
    L = ants.LrfSet(lrf)
    coef, counts = ants.fit_axial_lrf(L, ants.fit_cfg(lrf.nb[0], 0.0, 150.0, 0.0),
                                      torch.from_numpy(sig).cuda(), _dev(ants, r))
    assert np.all(np.isnan(coef.cpu().numpy()))
    assert counts.cpu().tolist() == [0, 0]


def test_iterative_procedure_converges_from_wrong_lrf(ants):
    # Sec. 8 on the GPU: 100 k events of the 61-sensor detector, start from
    # an LRF for a 13 mm source height (truth: 10 mm), four refits
    true_lrf, rec = W.mixed_geometries()[1]
    Lt = ants.LrfSet(true_lrf)
    sig, truth = ants.generate(Lt, ants.gen_cfg(rec), 100_000, 5)
    grid = ants.grid_cfg(W.workload(3).grid)
    wrong = W.axial_lrf(true_lrf.sxy, h=13.0)
    start = ants.AxialModel(wrong.sxy, wrong.gain, wrong.active, wrong.nb[0], wrong.lo[0],
                            wrong.hi[0], np.asarray(wrong.coef).reshape(-1))
    models, last = ants.iterate_axial_lrf(start, grid, sig, 4)
    t = truth.cpu().numpy()
    errs = []
    for m in models:
        L = ants.LrfSet(m)
        o = ants.reconstruct(L, grid, sig)
        torch.cuda.synchronize()
        inner = np.hypot(t[:, 0], t[:, 1]) < 90
        dx = o["x"].cpu().numpy() - t[:, 0]
        dy = o["y"].cpu().numpy() - t[:, 1]
        errs.append(float(np.sqrt(0.5 * np.mean(dx[inner] ** 2 + dy[inner] ** 2))))
        L.close()
    ref = ants.reconstruct(Lt, grid, sig)
    torch.cuda.synchronize()
    dx = ref["x"].cpu().numpy() - t[:, 0]
    dy = ref["y"].cpu().numpy() - t[:, 1]
    best = float(np.sqrt(0.5 * np.mean(dx[inner] ** 2 + dy[inner] ** 2)))
    print("sigma_xy per iteration", np.round(errs, 3).tolist(), "with the true LRF", round(best, 3))
    # the procedure can need tens of iterations (Sec. 8): every refit must
    # improve the resolution, and four must close a third of the gap to the
    # resolution with the true LRF
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] - best < 0.67 * (errs[0] - best), (errs, best)
