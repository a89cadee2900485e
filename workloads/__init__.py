"""Seeded synthetic workloads: detector geometry, the LRF coefficient recipe
and the random draws for flood-field events.

This module holds no reconstruction arithmetic.  It is the one place that
both the oracle-side tests and the library-side benchmark take their inputs
from:

* sensor arrays (regular hexagonal or square packing, Sec. 3.3);
* the light response that the detector is assumed to have, the solid-angle
  form h^3 / (h^2 + r^2)^(3/2), and B-spline coefficients for it built by a
  cubic quasi-interpolant that only samples that function (Sec. 6: LRFs are
  parameterised by cubic B-splines);
* flood-field source positions, event energies and relative gains
  (Sec. 4.1.1 "flood field"; Sec. 5.1.1 relative gains), and Poisson draws
  for counts whose means the caller supplies.

Random numbers come from NumPy PCG64 seeded with SeedSequence(160207247 + k)
for workload k, spawned into independent streams for positions, energies,
gains and counts.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 160207247

# ---------------------------------------------------------------- geometry


def hex_array(rings: int, pitch: float) -> np.ndarray:
    """Hexagonal packing with `rings` rings around a centre sensor.

    Sensors sit at pitch*(i + j/2, j*sqrt(3)/2) for integers with
    max(|i|, |j|, |i+j|) <= rings, ordered by j (rows of constant y) then i.
    Returns [n][2] float64 (19, 37, 61, 127 sensors for 2, 3, 4, 6 rings).
    """
    pts = []
    for j in range(-rings, rings + 1):
        for i in range(-rings, rings + 1):
            if max(abs(i), abs(j), abs(i + j)) <= rings:
                pts.append((pitch * (i + 0.5 * j), pitch * j * math.sqrt(3.0) / 2.0))
    return np.asarray(pts, dtype=np.float64)


def square_array(n: int, pitch: float) -> np.ndarray:
    """n x n square packing centred on the origin, index = n*row + col."""
    off = -(n - 1) * pitch / 2.0
    pts = [(off + pitch * c, off + pitch * r) for r in range(n) for c in range(n)]
    return np.asarray(pts, dtype=np.float64)


# ------------------------------------------------ detector light response


def solid_angle(h, r2):
    """Relative light seen by a sensor at squared lateral distance r2 from a
    point source at height h: h^3 / (h^2 + r2)^(3/2) (1 at r = 0)."""
    h = np.asarray(h, dtype=np.float64)
    return h ** 3 / (h * h + r2) ** 1.5


_QI = np.array([-1.0, 8.0, -1.0]) / 6.0


def quasi_interp_1d(f, lo: float, hi: float, nb: int) -> np.ndarray:
    """Coefficients of a uniform cubic B-spline (nb breakpoints on [lo, hi],
    nb+2 coefficients, coefficient j centred on breakpoint j-1) for f, by
    the cubic quasi-interpolant c_j = (-f(u_{j-2}) + 8 f(u_{j-1}) - f(u_j))/6,
    which reproduces cubic polynomials exactly.  f is sampled only."""
    d = (hi - lo) / (nb - 1)
    u = lo + d * (np.arange(-2, nb + 2))          # u_{-2} .. u_{nb+1}
    fu = np.asarray(f(u), dtype=np.float64)
    return _QI[0] * fu[:-2] + _QI[1] * fu[1:-1] + _QI[2] * fu[2:]


def quasi_interp_2d(f, lo, hi, nb) -> np.ndarray:
    """Tensor-product quasi-interpolant: table [nb1+2][nb0+2] for f(u0, u1)."""
    d0 = (hi[0] - lo[0]) / (nb[0] - 1)
    d1 = (hi[1] - lo[1]) / (nb[1] - 1)
    u0 = lo[0] + d0 * np.arange(-2, nb[0] + 2)
    u1 = lo[1] + d1 * np.arange(-2, nb[1] + 2)
    F = np.asarray(f(u0[None, :], u1[:, None]), dtype=np.float64)  # [n1][n0]
    G = _QI[0] * F[:, :-2] + _QI[1] * F[:, 1:-1] + _QI[2] * F[:, 2:]
    return _QI[0] * G[:-2, :] + _QI[1] * G[1:-1, :] + _QI[2] * G[2:, :]


# ----------------------------------------------------------- descriptors

KIND_AXIAL, KIND_XY, KIND_RZ, KIND_COMPOSITE, KIND_SLICED = 1, 2, 3, 4, 5


@dataclass
class LRFSet:
    """Detector model: sensors, gains, activity mask and LRF coefficients."""
    kind: int
    sxy: np.ndarray            # [n][2] float64
    gain: np.ndarray           # [n] float64
    active: np.ndarray         # [n] uint8
    shared: int
    nb: tuple                  # (nb0, nb1); nb1 = 1 for axial
    lo: tuple
    hi: tuple
    coef: np.ndarray           # [n_lrf][nb1+2][nb0+2] float64 (axial: [n_lrf][1][nb0+2];
                               # sliced: [n_lrf][n_planes][nb1+2][nb0+2])
    # composite: the XY residual added to the (shared) axial part
    xy_nb: tuple = (0, 0)
    xy_lo: tuple = (0.0, 0.0)
    xy_hi: tuple = (0.0, 0.0)
    xy_coef: np.ndarray = None  # [n_xy][xy_nb1+2][xy_nb0+2]
    xy_shared: int = 1
    # sliced: XY LRFs on n_planes z planes from z_lo to z_hi
    n_planes: int = 0
    z_lo: float = 0.0
    z_hi: float = 0.0

    @property
    def n_sensors(self) -> int:
        return int(self.sxy.shape[0])


@dataclass
class GridCfg:
    nodes: tuple = (9, 9, 1)
    iterations: int = 6
    shrink: float = 0.5
    step0: tuple = (7.5, 7.5, 0.0)
    z_start: float = 0.0
    stat: int = 0              # 0 ML, 1 chi2
    start: int = 0             # 0 CoG, 1 strongest sensor, 2 seed
    l_floor: float = 1e-9
    v_floor: float = 1.0
    seed_steps: int = 0
    seed_kappa: float = 1.0
    seed_kmin: int = 1
    seed_kmax: int = 1
    seed_scale: tuple = (0.0, 0.0, 0.0)
    cut_signal: float = 0.0    # ignore sensors with a signal below this (0 = off)
    cut_distance: float = 0.0  # ignore sensors farther than this from the start, mm (0 = off)

    @property
    def final_step(self):
        f = self.shrink ** (self.iterations - 1)
        return tuple(s * f for s in self.step0)


@dataclass
class SimplexCfg:
    """Simplex (Nelder-Mead) search settings: searched axes, statistic,
    start, initial simplex edge per axis, convergence size, iteration cap."""
    dims: int = 2              # 2: x, y; 3: x, y, z
    stat: int = 0              # 0 ML, 1 chi2
    start: int = 0             # 0 CoG, 1 strongest sensor, 2 seed
    step0: tuple = (7.5, 7.5, 0.0)
    z_start: float = 0.0
    tol: float = 1e-3          # mm: every vertex within tol of the best, per axis
    max_iter: int = 200
    l_floor: float = 1e-9
    v_floor: float = 1.0


@dataclass
class MigradCfg:
    """Variable-metric (Migrad-style) search settings: searched axes,
    statistic, start, per-axis scale (fallback curvature), central-difference
    step, EDM tolerance, iteration cap."""
    dims: int = 2              # 2: x, y; 3: x, y, z
    stat: int = 0              # 0 ML, 1 chi2
    start: int = 0             # 0 CoG, 1 strongest sensor, 2 seed
    step0: tuple = (7.5, 7.5, 0.0)
    z_start: float = 0.0
    h: float = 1e-3            # mm
    edm_tol: float = 1e-6      # statistic units
    max_iter: int = 100
    l_floor: float = 1e-9
    v_floor: float = 1.0


@dataclass
class EventRecipe:
    region: str                # "disc" or "square"
    extent: float              # disc radius or square half-width (mm)
    e_lo: float
    e_hi: float
    z_lo: float = 0.0
    z_hi: float = 0.0
    three_d: bool = False


@dataclass
class Workload:
    index: int
    name: str
    lrf: LRFSet
    grid: GridCfg
    events: EventRecipe
    n_events: int
    extra: dict = field(default_factory=dict)


def axial_lrf(sxy, h=10.0, nb=20, lo=0.0, hi=150.0, gain=None) -> LRFSet:
    c = quasi_interp_1d(lambda r: solid_angle(h, r * r), lo, hi, nb)
    n = sxy.shape[0]
    return LRFSet(KIND_AXIAL, sxy, np.ones(n) if gain is None else gain,
                  np.ones(n, np.uint8), 1, (nb, 1), (lo, 0.0), (hi, 0.0),
                  c.reshape(1, 1, -1))


def rz_lrf(sxy, nbr=24, nbz=16, rlo=0.0, rhi=200.0, zlo=0.0, zhi=50.0) -> LRFSet:
    c = quasi_interp_2d(lambda r, z: solid_angle(z + 10.0, r * r),
                        (rlo, zlo), (rhi, zhi), (nbr, nbz))
    n = sxy.shape[0]
    return LRFSet(KIND_RZ, sxy, np.ones(n), np.ones(n, np.uint8), 1, (nbr, nbz),
                  (rlo, zlo), (rhi, zhi), c.reshape(1, nbz + 2, nbr + 2))


def xy_lrf(sxy, gain, h=5.0, nb=32, lo=-24.0, hi=24.0) -> LRFSet:
    tabs = []
    for X, Y in sxy:
        tabs.append(quasi_interp_2d(
            lambda x, y, X=X, Y=Y: solid_angle(h, (x - X) ** 2 + (y - Y) ** 2),
            (lo, lo), (hi, hi), (nb, nb)))
    n = sxy.shape[0]
    return LRFSet(KIND_XY, sxy, gain, np.ones(n, np.uint8), 0, (nb, nb),
                  (lo, lo), (hi, hi), np.stack(tabs))


def composite_lrf(sxy, h=10.0, nb=24, hi=200.0, xy_nb=24, ext=90.0, amp=0.04,
                  shift=6.0, width=14.0) -> LRFSet:
    """Composite LRF (axial part + XY residual per sensor): the axial
    solid-angle response of axial_lrf plus, per sensor, a non-axial bump
    amp * exp(-((x - X - shift)^2 + (y - Y)^2) / (2 width^2)) (light
    scattered towards +x) on a uniform XY grid over [-ext, ext]^2."""
    base = axial_lrf(sxy, h=h, nb=nb, hi=hi)
    tabs = []
    for X, Y in sxy:
        tabs.append(quasi_interp_2d(
            lambda x, y, X=X, Y=Y: amp * np.exp(-((x - X - shift) ** 2 + (y - Y) ** 2)
                                                / (2 * width ** 2)),
            (-ext, -ext), (ext, ext), (xy_nb, xy_nb)))
    return LRFSet(KIND_COMPOSITE, base.sxy, base.gain, base.active, 1, base.nb, base.lo,
                  base.hi, base.coef, xy_nb=(xy_nb, xy_nb), xy_lo=(-ext, -ext),
                  xy_hi=(ext, ext), xy_coef=np.stack(tabs), xy_shared=0)


def sliced_lrf(sxy, n_planes=6, z_lo=0.0, z_hi=50.0, nb=20, ext=130.0) -> LRFSet:
    """Sliced LRF: per sensor, XY LRFs on n_planes z planes, each the
    solid-angle response with h = z + 10 mm of that plane (as the r-z
    workload), on a uniform XY grid over [-ext, ext]^2."""
    zs = np.linspace(z_lo, z_hi, n_planes)
    tabs = []
    for X, Y in sxy:
        tabs.append(np.stack([quasi_interp_2d(
            lambda x, y, X=X, Y=Y, h=z + 10.0: solid_angle(h, (x - X) ** 2 + (y - Y) ** 2),
            (-ext, -ext), (ext, ext), (nb, nb)) for z in zs]))
    n = sxy.shape[0]
    return LRFSet(KIND_SLICED, sxy, np.ones(n), np.ones(n, np.uint8), 0, (nb, nb),
                  (-ext, -ext), (ext, ext), np.stack(tabs), n_planes=n_planes, z_lo=z_lo,
                  z_hi=z_hi)


def streams(k: int, n: int = 4):
    """Independent generators for workload k: positions, energy, gains, counts."""
    ss = np.random.SeedSequence(SEED_BASE + k).spawn(n)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss]


def workload(k: int) -> Workload:
    """The five workloads: 0 axial 19-hex, 1 XY 8x8 square, 2 r-z 37-hex,
    3 mixed 19/61/127-hex stream, 4 learned-seed r-z (same detector as 2)."""
    if k == 0:
        sxy = hex_array(2, 30.0)
        return Workload(0, "hex19-axial", axial_lrf(sxy),
                        GridCfg((9, 9, 1), 6, 0.5, (7.5, 7.5, 0.0), 0.0),
                        EventRecipe("disc", 60.0, 500.0, 2000.0), 10_000)
    if k == 1:
        sxy = square_array(8, 6.0)
        gain = streams(1)[2].uniform(0.8, 1.2, size=sxy.shape[0])
        return Workload(1, "square64-xy", xy_lrf(sxy, gain),
                        GridCfg((9, 9, 1), 6, 0.5, (1.5, 1.5, 0.0), 0.0),
                        EventRecipe("square", 24.0, 200.0, 1000.0), 1_000_000)
    if k in (2, 4):
        sxy = hex_array(3, 30.0)
        g = GridCfg((7, 7, 7), 8, 0.5, (10.0, 10.0, 50.0 / 6.0), 25.0)
        return Workload(k, "hex37-rz" if k == 2 else "hex37-rz-seeded", rz_lrf(sxy), g,
                        EventRecipe("disc", 90.0, 500.0, 2000.0, 0.0, 50.0, True), 10_000_000,
                        {} if k == 2 else {"n_train": 5_000_000, "n_val": 500_000,
                                           "chi2ndf_max": 2.0})
    if k == 3:
        return Workload(3, "hex19-61-127-axial-stream", axial_lrf(hex_array(2, 30.0)),
                        GridCfg((9, 9, 1), 6, 0.5, (7.5, 7.5, 0.0), 0.0),
                        EventRecipe("disc", 60.0, 500.0, 2000.0), 20_000_000,
                        {"rings": (2, 4, 6), "chunk_median": 1e4, "chunk_sigma_ln": 1.0,
                         "chunk_min": 1_000, "chunk_max": 100_000})
    raise ValueError(f"no workload {k}")


def mixed_geometries():
    """The three detectors of the mixed stream: 19, 61 and 127 hex sensors,
    pitch 30 mm, axial LRFs as in workload 0; events fill r < 30*rings."""
    out = []
    for rings in (2, 4, 6):
        out.append((axial_lrf(hex_array(rings, 30.0)),
                    EventRecipe("disc", 30.0 * rings, 500.0, 2000.0)))
    return out


# -------------------------------------------------------------- draws


def draw_sources(recipe: EventRecipe, n: int, rng_pos, rng_e):
    """Flood-field sources: positions [n][3] and total expected
    photoelectrons E_tot [n] (uniform in [e_lo, e_hi])."""
    pos = np.zeros((n, 3), dtype=np.float64)
    if recipe.region == "disc":
        u = rng_pos.random(n)
        v = rng_pos.random(n)
        r = recipe.extent * np.sqrt(u)
        phi = 2.0 * np.pi * v
        pos[:, 0] = r * np.cos(phi)
        pos[:, 1] = r * np.sin(phi)
    else:
        pos[:, 0] = rng_pos.uniform(-recipe.extent, recipe.extent, n)
        pos[:, 1] = rng_pos.uniform(-recipe.extent, recipe.extent, n)
    if recipe.three_d:
        pos[:, 2] = rng_pos.uniform(recipe.z_lo, recipe.z_hi, n)
    etot = rng_e.uniform(recipe.e_lo, recipe.e_hi, n)
    return pos, etot


def poisson_counts(mu: np.ndarray, rng) -> np.ndarray:
    """Poisson draws with the given means, returned as float32 counts."""
    return rng.poisson(mu).astype(np.float32)


def chunk_stream(total: int, seed_offset: int = 0, median=1e4, sigma_ln=1.0,
                 lo=1_000, hi=100_000, n_geom=3):
    """Chunk sizes (lognormal, clipped) and a geometry id per chunk, summing
    to `total` events (the last chunk is trimmed)."""
    rng = streams(3 + seed_offset, 5)[4]
    sizes, geoms, acc = [], [], 0
    while acc < total:
        s = int(np.clip(round(rng.lognormal(math.log(median), sigma_ln)), lo, hi))
        s = min(s, total - acc)
        sizes.append(s)
        geoms.append(int(rng.integers(0, n_geom)))
        acc += s
    return np.asarray(sizes, np.int64), np.asarray(geoms, np.int32)


# Network targets: (position - offset) / scale.  One scale on every axis, so
# that the single predicted log-variance describes all three (the seeds'
# errors are about equal in x, y and z for the 37-sensor r-z detector).
SEED_POS_SCALE = (90.0, 90.0, 90.0)
SEED_POS_OFFSET = (0.0, 0.0, 25.0)


def seeded_refine_grid(kappa: float = 0.5, kmin: int = 2, kmax: int = 8,
                       shrink: float = 0.4) -> GridCfg:
    """Refinement grid of the learned-seed path: 3 x 3 x 3 nodes started at
    the seed, ending on the plain grid's final step (workload 2: 10, 10,
    50/6 mm halved over 8 iterations), with the iteration count chosen per
    event from the seed's predicted spread (kappa * sigma).  Steps shrink by
    0.4 per iteration (a 3-node grid keeps the minimum within reach for any
    factor >= 1/3: the next grid spans c / (1 - c) >= 1/2 of the step)."""
    final = [10.0 * 0.5 ** 7, 10.0 * 0.5 ** 7, 50.0 / 6.0 * 0.5 ** 7]
    step0 = tuple(f / shrink ** (kmax - 1) for f in final)
    return GridCfg((3, 3, 3), kmax, shrink, step0, 25.0, stat=0, start=2,
                   seed_steps=1, seed_kappa=kappa, seed_kmin=kmin, seed_kmax=kmax,
                   seed_scale=SEED_POS_SCALE)
