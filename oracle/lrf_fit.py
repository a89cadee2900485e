"""FP64 reference of the LRF fit from events (ANTS2, arXiv:1602.07247).

TEST INFRASTRUCTURE ONLY: nothing in the library imports or runs this.

The LRF module computes LRFs from signals and event positions (Sec. 6),
here for the axial parameterisation (Sec. 6.1.1) with per-sensor relative
gains and the sensors in groups that share one LRF (Sec. 6.2: one group
for all sensors, groups by distance from the array centre or by symmetry,
or every sensor its own); the relative gains can be re-calculated within
fixed groups without changing the LRF profiles (Sec. 6.3).  The iterative
procedure of Sec. 8 alternates the fit with the position reconstruction,
keeping only events that pass a filter, optionally with a small random
shift of the reconstructed positions (its draws are inputs here).

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
  * events enter when their reconstruction status has none of the failure
    bits (empty, bad input, no active sensor, no valid node: 1|2|4|8; the
    tie and fallback bits describe how a valid position was found), E > 0
    and finite, and chi2/ndf <= chi2ndf_max (when given);
  * groups: one table per group, fitted to the pairs of its member sensors
    only; a group without pairs has no solution (NaN);
  * shift: the fit reads (x + dx, y + dy) for each event, the shift drawn
    by the caller;
  * gains within groups: the least-squares scale of n_ie / E_e against the
    group's fixed L(r_ie) over the sensor's pairs in the domain,
    g_i = sum (n/E) L / sum L^2;
  * composite LRFs (Sec. 6.1.1: an axial LRF shared by every sensor plus an
    XY residual per sensor or shared; the LRF is max(axial + residual, 0),
    each part 0 outside its own domain) are fitted in two stages: the
    shared axial fit above, then the XY residual fitted to the estimates
    n_ie / (E_e g_i) minus the fitted axial spline at r_ie (not clamped);
  * sliced LRFs (Sec. 6.1.2: XY LRFs on n_planes z planes, interpolated
    linearly between the two closest): each plane's tables are fitted as
    XY LRFs to the events whose reconstructed z is nearest that plane,
    z in [z_p - d/2, z_p + d/2) for plane spacing d (the first plane's
    window open below, the last's open above).
"""
from __future__ import annotations

import numpy as np

# reconstruction status bits that mark a failed event: empty, bad input,
# no active sensor, no valid node
FAILED = 1 | 2 | 4 | 8


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
        use &= (np.asarray(status) & FAILED) == 0
    if chi2ndf_max is not None and chi2ndf_max > 0:
        c = np.asarray(chi2, np.float64)
        d = np.asarray(ndf, np.float64)
        with np.errstate(divide="ignore", invalid="ignore"):
            use &= (d > 0) & (c / d <= chi2ndf_max)
    return use


def _positions(x, y, use, shift):
    xe = np.asarray(x, np.float64)
    ye = np.asarray(y, np.float64)
    if shift is not None:
        sh = np.asarray(shift, np.float64)
        xe = xe + sh[:, 0]
        ye = ye + sh[:, 1]
    return xe[use], ye[use]


def normal_equations(sxy, gain, active, signals, x, y, E, use, nb, lo, hi, members=None,
                     shift=None):
    """Normal matrix M [(nb+2)^2] and right-hand side v [nb+2] of the
    least-squares fit over the pairs of the sensors in `members` (default:
    every active sensor), and the number of (event, sensor) pairs in it.
    `shift` [n][2]: added to the event positions."""
    nc = nb + 2
    d = (hi - lo) / (nb - 1)
    tol = 1e-9 * (hi - lo)
    M = np.zeros((nc, nc))
    v = np.zeros(nc)
    sig = np.asarray(signals, np.float64)[use]
    xe, ye = _positions(x, y, use, shift)
    Ee = np.asarray(E, np.float64)[use]
    npairs = 0
    if members is None:
        members = range(len(sxy))
    for i in members:
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


def _solve(M, v, ridge):
    lam = ridge * float(np.mean(np.diag(M)))
    try:
        return np.linalg.solve(M + lam * np.eye(len(v)), v)
    except np.linalg.LinAlgError:
        return np.full(len(v), np.nan)


def fit_axial_grouped(sxy, gain, active, signals, x, y, E, use, nb, lo, hi, groups,
                      ridge=1e-9, shift=None):
    """One axial table per sensor group (Sec. 6.2).  `groups` [n_sensors]:
    the group of each sensor (0..G-1), -1 for sensors not fitted.  Returns
    the coefficients [G][nb+2] (NaN rows for groups without pairs) and the
    pair count of each group [G]."""
    groups = np.asarray(groups, np.int64)
    G = int(groups.max()) + 1 if len(groups) and groups.max() >= 0 else 0
    coef = np.full((G, nb + 2), np.nan)
    pairs = np.zeros(G, np.int64)
    for g in range(G):
        members = [i for i in range(len(sxy)) if groups[i] == g and active[i]]
        M, v, npairs = normal_equations(sxy, gain, active, signals, x, y, E, use, nb, lo, hi,
                                        members, shift)
        pairs[g] = npairs
        if npairs > 0:
            coef[g] = _solve(M, v, ridge)
    return coef, pairs


def axial_value(coef, nb, lo, hi, r):
    """The reconstruction's axial LRF at distances r: max(spline, 0) inside
    [lo, hi] (relative slack 1e-9), 0 outside."""
    r = np.asarray(r, np.float64)
    d = (hi - lo) / (nb - 1)
    tol = 1e-9 * (hi - lo)
    inside = (r >= lo - tol) & (r <= hi + tol)
    u = (np.clip(r, lo, hi) - lo) / d
    m = np.clip(np.floor(u).astype(np.int64), 0, nb - 2)
    b = bspline_weights(u - m)
    c = np.asarray(coef, np.float64)
    val = sum(b[..., k] * c[m + k] for k in range(4))
    return np.where(inside, np.maximum(val, 0.0), 0.0)


def fit_gains(sxy, active, signals, x, y, E, use, nb, lo, hi, tables, table_of, shift=None):
    """Relative gains re-calculated within fixed groups (Sec. 6.3): for each
    active sensor i with a table (table_of[i] >= 0), the least-squares
    scale g_i of n_ie / E_e against L_{table_of[i]}(r_ie) over its pairs in
    the domain.  Returns gains [n_sensors] (NaN where there is no pair or
    sum L^2 = 0) and the pair counts."""
    d = (hi - lo) / (nb - 1)
    tol = 1e-9 * (hi - lo)
    sig = np.asarray(signals, np.float64)[use]
    xe, ye = _positions(x, y, use, shift)
    Ee = np.asarray(E, np.float64)[use]
    n = len(sxy)
    gains = np.full(n, np.nan)
    pairs = np.zeros(n, np.int64)
    for i in range(n):
        if not active[i] or table_of[i] < 0:
            continue
        r = np.sqrt((xe - sxy[i][0]) ** 2 + (ye - sxy[i][1]) ** 2)
        inside = (r >= lo - tol) & (r <= hi + tol)
        L = axial_value(tables[table_of[i]], nb, lo, hi, r[inside])
        t = sig[inside, i] / Ee[inside]
        pairs[i] = int(inside.sum())
        den = float(np.sum(L * L))
        if pairs[i] > 0 and den > 0.0:
            gains[i] = float(np.sum(t * L)) / den
    return gains, pairs


# ---- two-dimensional LRFs: r-z (Sec. 6.1.1, r and depth) and XY (Sec.
# 6.1.1, per-sensor bicubic in the detector plane)
#
# Readings: the same least squares as the axial fit, on the tensor-product
# cubic B-spline of the reconstruction (coefficient (j1, j0) centred on
# breakpoints (j1 - 1, j0 - 1), table [nb1 + 2][nb0 + 2]); a pair enters when
# both spline arguments lie in their domains (relative slack 1e-9); the
# arguments are (r, z) for "rz" and (x, y) for "xy"; a ridge of `ridge`
# times the mean diagonal; groups, shifts and the event filter as above.

def axial_spline(coef, nb, lo, hi, r):
    """The axial spline at distances r inside [lo, hi] (relative slack
    1e-9), not clamped, 0 outside: the axial part of a composite LRF."""
    r = np.asarray(r, np.float64)
    d = (hi - lo) / (nb - 1)
    tol = 1e-9 * (hi - lo)
    inside = (r >= lo - tol) & (r <= hi + tol)
    u = (np.clip(r, lo, hi) - lo) / d
    m = np.clip(np.floor(u).astype(np.int64), 0, nb - 2)
    b = bspline_weights(u - m)
    c = np.asarray(coef, np.float64)
    val = sum(b[..., k] * c[m + k] for k in range(4))
    return np.where(inside, val, 0.0)


def _args2d(kind, sx, sy, xe, ye, ze):
    if kind == "rz":
        return np.sqrt((xe - sx) ** 2 + (ye - sy) ** 2), ze
    return xe, ye


def _locate(u, nb, lo, hi):
    d = (hi - lo) / (nb - 1)
    tol = 1e-9 * (hi - lo)
    inside = (u >= lo - tol) & (u <= hi + tol)
    v = (u - lo) / d
    m = np.clip(np.floor(v).astype(np.int64), 0, nb - 2)
    return inside, m, v - m


def normal_equations_2d(kind, sxy, gain, active, signals, x, y, z, E, use, nb, lo, hi,
                        members=None, shift=None, base=None):
    """Normal matrix [nc][nc], right side [nc] (nc = (nb0 + 2)(nb1 + 2),
    coefficient (j1, j0) at index j1 (nb0 + 2) + j0) and pair count of the
    least-squares fit of a 2-D LRF over the pairs of the sensors in
    `members` (default: every active sensor).  base = (coef, nb, lo, hi) of
    an axial spline subtracted from every estimate at the pair's distance
    (the residual of a composite LRF), or None."""
    nc0, nc1 = nb[0] + 2, nb[1] + 2
    nc = nc0 * nc1
    M = np.zeros((nc, nc))
    v = np.zeros(nc)
    sig = np.asarray(signals, np.float64)[use]
    xe, ye = _positions(x, y, use, shift)
    ze = np.asarray(z, np.float64)[use]
    Ee = np.asarray(E, np.float64)[use]
    npairs = 0
    if members is None:
        members = range(len(sxy))
    for i in members:
        if not active[i]:
            continue
        u, w = _args2d(kind, sxy[i][0], sxy[i][1], xe, ye, ze)
        in0, m0, t0 = _locate(u, nb[0], lo[0], hi[0])
        in1, m1, t1 = _locate(w, nb[1], lo[1], hi[1])
        ok = in0 & in1
        b0 = bspline_weights(t0[ok])
        b1 = bspline_weights(t1[ok])
        m0, m1 = m0[ok], m1[ok]
        target = sig[ok, i] / (Ee[ok] * gain[i])
        if base is not None:
            r = np.sqrt((xe[ok] - sxy[i][0]) ** 2 + (ye[ok] - sxy[i][1]) ** 2)
            target = target - axial_spline(base[0], base[1], base[2], base[3], r)
        idx = [(m1 + q) * nc0 + (m0 + p) for q in range(4) for p in range(4)]
        wts = [b1[:, q] * b0[:, p] for q in range(4) for p in range(4)]
        for a in range(16):
            np.add.at(v, idx[a], wts[a] * target)
            for b in range(16):
                np.add.at(M, (idx[a], idx[b]), wts[a] * wts[b])
        npairs += int(ok.sum())
    return M, v, npairs


def fit_2d_grouped(kind, sxy, gain, active, signals, x, y, z, E, use, nb, lo, hi, groups,
                   ridge=1e-9, shift=None, base=None):
    """One 2-D table per sensor group: coefficients [G][nb1 + 2][nb0 + 2]
    (NaN for groups without pairs) and pair counts [G]."""
    groups = np.asarray(groups, np.int64)
    G = int(groups.max()) + 1 if len(groups) and groups.max() >= 0 else 0
    nc0, nc1 = nb[0] + 2, nb[1] + 2
    coef = np.full((G, nc1, nc0), np.nan)
    pairs = np.zeros(G, np.int64)
    for g in range(G):
        members = [i for i in range(len(sxy)) if groups[i] == g and active[i]]
        M, v, npairs = normal_equations_2d(kind, sxy, gain, active, signals, x, y, z, E, use,
                                           nb, lo, hi, members, shift, base)
        pairs[g] = npairs
        if npairs > 0:
            coef[g] = _solve(M, v, ridge).reshape(nc1, nc0)
    return coef, pairs


def value_2d(coef, nb, lo, hi, u, w):
    """The reconstruction's 2-D LRF max(spline, 0) at (u, w), 0 outside."""
    coef = np.asarray(coef, np.float64)
    in0, m0, t0 = _locate(np.asarray(u, np.float64), nb[0], lo[0], hi[0])
    in1, m1, t1 = _locate(np.asarray(w, np.float64), nb[1], lo[1], hi[1])
    b0, b1 = bspline_weights(t0), bspline_weights(t1)
    val = sum(b1[..., q] * b0[..., p] * coef[m1 + q, m0 + p] for q in range(4) for p in range(4))
    return np.where(in0 & in1, np.maximum(val, 0.0), 0.0)


def spline_2d(coef, nb, lo, hi, u, w):
    """A 2-D spline at (u, w) inside its domain, not clamped, 0 outside: the
    XY residual of a composite LRF."""
    coef = np.asarray(coef, np.float64)
    in0, m0, t0 = _locate(np.asarray(u, np.float64), nb[0], lo[0], hi[0])
    in1, m1, t1 = _locate(np.asarray(w, np.float64), nb[1], lo[1], hi[1])
    b0, b1 = bspline_weights(t0), bspline_weights(t1)
    val = sum(b1[..., q] * b0[..., p] * coef[m1 + q, m0 + p] for q in range(4) for p in range(4))
    return np.where(in0 & in1, val, 0.0)


def composite_value(axial_coef, nb, lo, hi, xy_coef, xy_nb, xy_lo, xy_hi, r, x, y):
    """A composite LRF max(axial(r) + residual(x, y), 0), each part 0
    outside its own domain."""
    return np.maximum(axial_spline(axial_coef, nb, lo, hi, r)
                      + spline_2d(xy_coef, xy_nb, xy_lo, xy_hi, x, y), 0.0)


def fit_composite(sxy, gain, active, signals, x, y, E, use, nb, lo, hi, xy_nb, xy_lo, xy_hi,
                  xy_groups, ridge=1e-9, shift=None):
    """Two-stage composite fit: the shared axial table [nb + 2], then one XY
    residual table per group of xy_groups [G][xy_nb1 + 2][xy_nb0 + 2]
    fitted to the estimates minus that axial spline; (axial, residuals,
    residual pair counts)."""
    members = [i for i in range(len(sxy)) if active[i]]
    M, v, _ = normal_equations(sxy, gain, active, signals, x, y, E, use, nb, lo, hi, members,
                               shift)
    axial = _solve(M, v, ridge)
    z = np.zeros(len(np.asarray(x)))
    res, pairs = fit_2d_grouped("xy", sxy, gain, active, signals, x, y, z, E, use, xy_nb, xy_lo,
                                xy_hi, xy_groups, ridge, shift, (axial, nb, lo, hi))
    return axial, res, pairs


def slice_windows(n_planes, z_lo, z_hi):
    """Depth window [a, b) of each plane: the events nearest that plane."""
    d = (z_hi - z_lo) / (n_planes - 1)
    cuts = [z_lo + (p + 0.5) * d for p in range(n_planes - 1)]
    lows = [-np.inf] + cuts
    highs = cuts + [np.inf]
    return list(zip(lows, highs))


def fit_sliced(sxy, gain, active, signals, x, y, z, E, use, nb, lo, hi, n_planes, z_lo, z_hi,
               groups, ridge=1e-9, shift=None):
    """Per-plane XY fits of a sliced LRF: tables [G][n_planes][nb1 + 2]
    [nb0 + 2] and pair counts [n_planes][G]."""
    zz = np.asarray(z, np.float64)
    tabs, pairs = [], []
    for a, b in slice_windows(n_planes, z_lo, z_hi):
        u = np.asarray(use, bool) & (zz >= a) & (zz < b)
        c, n = fit_2d_grouped("xy", sxy, gain, active, signals, x, y, z, E, u, nb, lo, hi,
                              groups, ridge, shift)
        tabs.append(c)
        pairs.append(n)
    return np.stack(tabs, 1), np.stack(pairs)
