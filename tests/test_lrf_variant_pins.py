"""Pins of the oracle's composite and sliced LRFs (Sec. 6.1.1: an axial LRF
plus an XY LRF of the residual; Sec. 6.1.2: XY LRFs on z planes with linear
interpolation between the two closest planes).

* Composite with a zero residual is the axial LRF, and with a zero axial
  part it is the XY LRF of the residual tables: values bit for bit, and so
  is every reconstruction (same path, same outputs).
* Composite = max(axial + residual, 0) against an independent evaluation
  (Cox-de Boor recursion for the axial spline and, row by row then
  column, for the tensor-product residual).
* Sliced on a plane is that plane's XY LRF bit for bit, and so is a 2-D
  reconstruction at that depth; between planes the value is affine in z
  (the quarter points lie on the chord); outside the planes' z range it is
  0; identical planes give the XY LRF at every depth.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import workloads as W


def _events(lrf, recipe, n, seed):
    sig, truth = oracle.make_events(lrf, recipe, n, W.streams(seed))
    return sig


def _same(a, b):
    for k in ("x", "y", "z", "E", "lnl", "chi2", "ndf", "status", "path"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_composite_reduces_to_axial_and_to_xy():
    sxy = W.hex_array(2, 30.0)
    comp = W.composite_lrf(sxy)
    axial = W.axial_lrf(sxy, nb=comp.nb[0], hi=comp.hi[0])
    pos = np.random.default_rng(1).uniform(-80, 80, (300, 3))
    pos[:, 2] = 0.0
    no_res = dataclasses.replace(comp, xy_coef=np.zeros_like(comp.xy_coef))
    np.testing.assert_array_equal(oracle.lrf_values(no_res, pos), oracle.lrf_values(axial, pos))
    xy = W.LRFSet(W.KIND_XY, sxy, comp.gain, comp.active, 0, comp.xy_nb, comp.xy_lo, comp.xy_hi,
                  comp.xy_coef)
    no_ax = dataclasses.replace(comp, coef=np.zeros_like(comp.coef))
    np.testing.assert_array_equal(oracle.lrf_values(no_ax, pos), oracle.lrf_values(xy, pos))
    rec = W.EventRecipe("disc", 60.0, 500.0, 2000.0)
    g = W.GridCfg((9, 9, 1), 6, 0.5, (7.5, 7.5, 0.0), 0.0)
    sig = _events(axial, rec, 60, 3)
    _same(oracle.reconstruct(no_res, g, sig), oracle.reconstruct(axial, g, sig))
    sig = _events(xy, rec, 60, 4)
    _same(oracle.reconstruct(no_ax, g, sig), oracle.reconstruct(xy, g, sig))


def test_composite_is_the_clamped_sum():
    sxy = W.hex_array(2, 30.0)
    comp = W.composite_lrf(sxy, amp=-0.3)           # negative residual: the clamp acts
    rng = np.random.default_rng(2)
    pos = np.zeros((200, 3))
    pos[:, :2] = rng.uniform(-100, 100, (200, 2))
    got = oracle.lrf_values(comp, pos)
    nb, (lo,), (hi,) = comp.nb[0], comp.lo[:1], comp.hi[:1]
    xnb, xlo, xhi = comp.xy_nb, comp.xy_lo, comp.xy_hi
    clamped = 0
    for p in range(len(pos)):
        for i in range(len(sxy)):
            r = np.hypot(pos[p, 0] - sxy[i, 0], pos[p, 1] - sxy[i, 1])
            a = oracle.deboor1(comp.coef.reshape(-1), nb, lo, hi, r)[0] if r <= hi else 0.0
            tab = comp.xy_coef[i]
            b = 0.0
            if xlo[0] <= pos[p, 0] <= xhi[0] and xlo[1] <= pos[p, 1] <= xhi[1]:
                rows = np.array([oracle.deboor1(tab[j], xnb[0], xlo[0], xhi[0], pos[p, 0])[0]
                                 for j in range(tab.shape[0])])
                b = oracle.deboor1(rows, xnb[1], xlo[1], xhi[1], pos[p, 1])[0]
            want = max(a + b, 0.0)
            clamped += a + b < 0
            assert got[p, i] == pytest.approx(want, rel=1e-12, abs=1e-15), (p, i)
    assert clamped > 50


def _plane_xy(sl, p):
    return W.LRFSet(W.KIND_XY, sl.sxy, sl.gain, sl.active, 0, sl.nb, sl.lo, sl.hi,
                    np.ascontiguousarray(sl.coef[:, p]))


def test_sliced_on_a_plane_is_that_planes_xy_lrf():
    sxy = W.hex_array(2, 30.0)
    sl = W.sliced_lrf(sxy, n_planes=6, nb=16, ext=110.0)
    rng = np.random.default_rng(5)
    xy = rng.uniform(-80, 80, (200, 2))
    rec = W.EventRecipe("disc", 60.0, 500.0, 2000.0)
    for p, z in enumerate(np.linspace(0.0, 50.0, 6)):
        pos = np.column_stack([xy, np.full(200, z)])
        np.testing.assert_array_equal(oracle.lrf_values(sl, pos),
                                      oracle.lrf_values(_plane_xy(sl, p), pos))
    # a 2-D reconstruction at the depth of plane 2 equals the XY one
    sig = _events(_plane_xy(sl, 2), rec, 50, 6)
    g = W.GridCfg((9, 9, 1), 6, 0.5, (7.5, 7.5, 0.0), 20.0)
    a = oracle.reconstruct(sl, g, sig)
    b = oracle.reconstruct(_plane_xy(sl, 2), g, sig)
    for k in ("x", "y", "E", "lnl", "chi2", "ndf", "status", "path"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_sliced_is_affine_between_planes_and_zero_outside():
    sxy = W.hex_array(2, 30.0)
    sl = W.sliced_lrf(sxy, n_planes=6, nb=16, ext=110.0)
    rng = np.random.default_rng(7)
    xy = rng.uniform(-60, 60, (100, 2))
    for zp in (0.0, 10.0, 40.0):
        ends = [oracle.lrf_values(sl, np.column_stack([xy, np.full(100, zp + s)]))
                for s in (0.0, 10.0)]
        for s in (2.5, 5.0, 7.5):
            mid = oracle.lrf_values(sl, np.column_stack([xy, np.full(100, zp + s)]))
            chord = ends[0] + (ends[1] - ends[0]) * (s / 10.0)
            np.testing.assert_allclose(mid, chord, rtol=1e-12, atol=1e-15)
    for z in (-0.5, 50.5, 80.0):
        assert not oracle.lrf_values(sl, np.column_stack([xy, np.full(100, z)])).any()
    # each plane's LRF is clamped before the interpolation: a plane whose
    # spline is negative contributes 0
    neg = sl.coef.copy()
    neg[:, 2] *= -1.0
    sln = dataclasses.replace(sl, coef=neg)
    up = oracle.lrf_values(sl, np.column_stack([xy, np.full(100, 30.0)]))
    for s_ in (2.5, 5.0):
        got = oracle.lrf_values(sln, np.column_stack([xy, np.full(100, 20.0 + s_)]))
        np.testing.assert_allclose(got, (s_ / 10.0) * up, rtol=1e-12, atol=1e-15)
    same = dataclasses.replace(sl, coef=np.repeat(sl.coef[:, :1], 6, axis=1))
    for z in (3.0, 27.5, 49.0):
        np.testing.assert_allclose(oracle.lrf_values(same, np.column_stack([xy, np.full(100, z)])),
                                   oracle.lrf_values(_plane_xy(sl, 0),
                                                     np.column_stack([xy, np.zeros(100)])),
                                   rtol=1e-15, atol=0)
