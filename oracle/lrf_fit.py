"""FP64 reference of the LRF fit from events (ANTS2, arXiv:1602.07247).

TEST INFRASTRUCTURE ONLY: nothing in the library imports or runs this.

The LRF module computes LRFs from signals and event positions (Sec. 6),
here for the axial parameterisation (Sec. 6.1.1) with one LRF shared by all
sensors and per-sensor relative gains (Sec. 6.2, "one group for all
sensors").  The iterative procedure of Sec. 8 alternates it with the
position reconstruction, keeping only events that pass a filter.

Readings (the paper prints no fit formula):
  * model: signal n_ie = E_e * g_i * L(r_ie), L a uniform cubic B-spline
    on [lo, hi] with nb breakpoints (nb + 2 coefficients, coefficient j
    centred on breakpoint j - 1, as the reconstruction reads it);
  * linear least squares in the coefficients: every (event, active sensor)
    pair with lo <= r <= hi (relative slack 1e-9 of the span) gives one
    estimate n_ie / (E_e g_i) of L(r_ie), all weighted 1 (so a sensor's
    signals and gain scaled together leave the fit unchanged);
  * a ridge of `ridge` times the mean diagonal of the normal matrix keeps
    coefficients without data defined (they go to zero);
  * events enter when their reconstruction status is 0, E > 0 and finite,
    and chi2/ndf <= chi2ndf_max (when given).
"""
from __future__ import annotations

import numpy as np


def bspline_weights(t):
    """Uniform cubic B-spline weights of the four coefficients m..m+3 at
    local coordinate t in [0, 1] (the textbook blending functions)."""
    t = np.asarray(t, np.float64)
    s = 1.0 - t
    return np.stack([s * s * s / 6.0,
                     (3.0 * t ** 3 - 6.0 * t * t + 4.0) / 6.0,
                     (-3.0 * t ** 3 + 3.0 * t * t + 3.0 * t + 1.0) / 6.0,
                     t ** 3 / 6.0], axis=-1)


def event_mask(E, status=None, chi2=None, ndf=None, chi2ndf_max=None):
    """Events used by the fit (the filter of the iterative procedure, Sec. 8)."""
    E = np.asarray(E, np.float64)
    use = np.isfinite(E) & (E > 0.0)
    if status is not None:
        use &= np.asarray(status) == 0
    if chi2ndf_max is not None and chi2ndf_max > 0:
        c = np.asarray(chi2, np.float64)
        d = np.asarray(ndf, np.float64)
        with np.errstate(divide="ignore", invalid="ignore"):
            use &= (d > 0) & (c / d <= chi2ndf_max)
    return use


def normal_equations(sxy, gain, active, signals, x, y, E, use, nb, lo, hi):
    """Normal matrix M [(nb+2)^2] and right-hand side v [nb+2] of the
    least-squares fit, and the number of (event, sensor) pairs in it."""
    nc = nb + 2
    d = (hi - lo) / (nb - 1)
    tol = 1e-9 * (hi - lo)
    M = np.zeros((nc, nc))
    v = np.zeros(nc)
    sig = np.asarray(signals, np.float64)[use]
    xe = np.asarray(x, np.float64)[use]
    ye = np.asarray(y, np.float64)[use]
    Ee = np.asarray(E, np.float64)[use]
    npairs = 0
    for i in range(len(sxy)):
        if not active[i]:
            continue
        r = np.sqrt((xe - sxy[i][0]) ** 2 + (ye - sxy[i][1]) ** 2)
        inside = (r >= lo - tol) & (r <= hi + tol)
        r = r[inside]
        target = sig[inside, i] / (Ee[inside] * gain[i])
        u = (r - lo) / d
        m = np.clip(np.floor(u).astype(np.int64), 0, nb - 2)
        t = u - m
        b = bspline_weights(t)
        for k in range(4):
            np.add.at(v, m + k, b[:, k] * target)
            for l in range(4):
                np.add.at(M, (m + k, m + l), b[:, k] * b[:, l])
        npairs += int(inside.sum())
    return M, v, npairs


def fit_axial_shared(sxy, gain, active, signals, x, y, E, use, nb, lo, hi, ridge=1e-9):
    """Coefficients [nb+2] of the shared axial LRF fitted to the events."""
    M, v, _ = normal_equations(sxy, gain, active, signals, x, y, E, use, nb, lo, hi)
    lam = ridge * float(np.mean(np.diag(M)))
    return np.linalg.solve(M + lam * np.eye(len(v)), v)
