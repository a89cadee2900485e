"""FP64 CPU oracle for contracting-grid reconstruction (ANTS2, arXiv:1602.07247).

TEST INFRASTRUCTURE ONLY.  Nothing in the library (paper_1602_07247_amd/)
imports, links or runs anything here; only tests/, the smoke check and the
CPU-baseline leg of bench.py do.  The grid search itself is plain C
(ants_oracle.c, double precision, one event at a time); the learned-seed
network reference is NumPy float64 (mlp.py), and so is the LRF fit from
events used by the iterative procedure (lrf_fit.py).  The two share no code with the
HIP path.

Sections of the paper each function follows are cited in ants_oracle.c.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ants_oracle.c")
_LIB = os.path.join(_HERE, "libants_oracle.so")


# -O3 for the timed CPU baseline; x86-64-v3 (AVX2) rather than -march=native
# because the library is built on one host and loaded on another.  No FMA
# contraction and no reassociation: each operation rounds as written, so the
# results do not depend on these flags.
BUILD_FLAGS = "gcc -O3 -march=x86-64-v3 -ffp-contract=off -fopenmp"


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (flags above)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-ffp-contract=off",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Lrf(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_sensors", C.c_int), ("sxy", C.POINTER(C.c_double)),
                ("gain", C.POINTER(C.c_double)), ("active", C.POINTER(C.c_uint8)),
                ("shared", C.c_int), ("nb", C.c_int * 2), ("lo", C.c_double * 2),
                ("hi", C.c_double * 2), ("coef", C.POINTER(C.c_double)),
                ("xy_nb", C.c_int * 2), ("xy_lo", C.c_double * 2), ("xy_hi", C.c_double * 2),
                ("xy_coef", C.POINTER(C.c_double)), ("xy_shared", C.c_int),
                ("n_planes", C.c_int), ("z_lo", C.c_double), ("z_hi", C.c_double)]


class _Cfg(C.Structure):
    _fields_ = [("nodes", C.c_int * 3), ("iterations", C.c_int), ("shrink", C.c_double),
                ("step0", C.c_double * 3), ("z_start", C.c_double), ("stat", C.c_int),
                ("start", C.c_int), ("l_floor", C.c_double), ("v_floor", C.c_double),
                ("seed_steps", C.c_int), ("seed_kappa", C.c_double), ("seed_kmin", C.c_int),
                ("seed_kmax", C.c_int), ("seed_scale", C.c_double * 3),
                ("cut_signal", C.c_double), ("cut_distance", C.c_double)]


class _SCfg(C.Structure):
    _fields_ = [("dims", C.c_int), ("stat", C.c_int), ("start", C.c_int),
                ("step0", C.c_double * 3), ("z_start", C.c_double), ("tol", C.c_double),
                ("max_iter", C.c_int), ("l_floor", C.c_double), ("v_floor", C.c_double)]


class _VCfg(C.Structure):
    _fields_ = [("dims", C.c_int), ("stat", C.c_int), ("start", C.c_int),
                ("step0", C.c_double * 3), ("z_start", C.c_double), ("h", C.c_double),
                ("edm_tol", C.c_double), ("max_iter", C.c_int), ("l_floor", C.c_double),
                ("v_floor", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        d, i64 = C.c_double, C.c_int64
        P = C.POINTER
        _lib.o_spline1.restype = d
        _lib.o_spline1.argtypes = [P(d), C.c_int, d, d, d]
        _lib.o_spline1_du.restype = d
        _lib.o_spline1_du.argtypes = [P(d), C.c_int, d, d, d]
        _lib.o_deboor1.restype = d
        _lib.o_deboor1.argtypes = [P(d), C.c_int, d, d, d]
        _lib.o_spline2.restype = d
        _lib.o_spline2.argtypes = [P(d), P(C.c_int), P(d), P(d), d, d, P(d), P(d)]
        _lib.o_basis.argtypes = [d, P(d)]
        _lib.o_reconstruct.argtypes = [P(_Lrf), P(_Cfg), i64, P(d), P(d), P(d), P(C.c_int),
                                       P(C.c_int), P(C.c_int), P(d), C.c_int]
        _lib.o_lattice_stats.argtypes = [P(_Lrf), P(_Cfg), P(d), P(d), P(d), P(C.c_int), P(d),
                                         C.c_int]
        _lib.o_node_eval_ext.argtypes = [P(_Lrf), P(_Cfg), P(d), d, d, d, P(d)]
        _lib.o_lrf_values.argtypes = [P(_Lrf), i64, P(d), P(d), C.c_int]
        _lib.o_expected_counts.argtypes = [P(_Lrf), i64, P(d), P(d), P(d), C.c_int]
        _lib.o_crb.argtypes = [P(_Lrf), C.c_int, i64, P(d), P(d), P(d)]
        _lib.o_reconstruct_seeded.argtypes = [P(_Lrf), P(_Cfg), P(_Cfg), d, i64, P(d), P(d),
                                              P(d), P(C.c_int), P(C.c_int), C.c_int]
        _lib.o_knn_prepare.argtypes = [P(_Lrf), i64, P(d), P(C.c_float), P(C.c_uint8), C.c_int]
        _lib.o_knn_reconstruct.argtypes = [P(_Lrf), i64, P(C.c_float), P(C.c_uint8), P(d),
                                           C.c_int, i64, P(d), P(d), P(C.c_int), P(i64),
                                           P(C.c_float), C.c_int]
        _lib.o_reconstruct_simplex.argtypes = [P(_Lrf), P(_SCfg), i64, P(d), P(d), P(d),
                                               P(C.c_int), P(C.c_int), P(C.c_int), P(C.c_int),
                                               C.c_int]
        _lib.o_reconstruct_migrad.argtypes = [P(_Lrf), P(_VCfg), i64, P(d), P(d), P(d),
                                               P(C.c_int), P(C.c_int), P(C.c_int), P(C.c_int),
                                               C.c_int]
        u32 = C.c_uint32
        _lib.o_philox4x32_10.argtypes = [P(u32), P(u32), P(u32)]
        _lib.o_poisson.restype = d
        _lib.o_poisson.argtypes = [d, C.c_uint64, u32, P(u32)]
        _lib.o_generate.argtypes = [P(_Lrf), C.c_int, d, d, d, d, d, C.c_int, C.c_uint64,
                                    C.c_uint64, i64, P(d), P(d), C.c_int]
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _threads(n):
    return int(n) if n else (os.cpu_count() or 1)


class Model:
    """Keeps C views of an LRF set (workloads.LRFSet) alive."""

    def __init__(self, lrf):
        self.sxy = np.ascontiguousarray(lrf.sxy, dtype=np.float64)
        self.gain = np.ascontiguousarray(lrf.gain, dtype=np.float64)
        self.active = np.ascontiguousarray(lrf.active, dtype=np.uint8)
        self.coef = np.ascontiguousarray(lrf.coef, dtype=np.float64)
        self.c = _Lrf()
        self.c.kind = lrf.kind
        self.c.n_sensors = self.sxy.shape[0]
        self.c.sxy = _dp(self.sxy)
        self.c.gain = _dp(self.gain)
        self.c.active = self.active.ctypes.data_as(C.POINTER(C.c_uint8))
        self.c.shared = lrf.shared
        self.c.nb[0], self.c.nb[1] = lrf.nb
        self.c.lo[0], self.c.lo[1] = lrf.lo
        self.c.hi[0], self.c.hi[1] = lrf.hi
        self.c.coef = _dp(self.coef)
        self.n_sensors = self.sxy.shape[0]
        # composite: XY residual; sliced: z planes (see workloads.LRFSet)
        xc = getattr(lrf, "xy_coef", None)
        if xc is not None:
            self.xy_coef = np.ascontiguousarray(xc, dtype=np.float64)
            self.c.xy_coef = _dp(self.xy_coef)
            self.c.xy_nb[0], self.c.xy_nb[1] = lrf.xy_nb
            self.c.xy_lo[0], self.c.xy_lo[1] = lrf.xy_lo
            self.c.xy_hi[0], self.c.xy_hi[1] = lrf.xy_hi
            self.c.xy_shared = int(lrf.xy_shared)
        self.c.n_planes = int(getattr(lrf, "n_planes", 0))
        self.c.z_lo = float(getattr(lrf, "z_lo", 0.0))
        self.c.z_hi = float(getattr(lrf, "z_hi", 0.0))


def _cfg(g):
    c = _Cfg()
    for k in range(3):
        c.nodes[k] = int(g.nodes[k])
        c.step0[k] = float(g.step0[k])
    c.iterations = int(g.iterations)
    c.shrink = float(g.shrink)
    c.z_start = float(g.z_start)
    c.stat = int(g.stat)
    c.start = int(g.start)
    c.l_floor = float(g.l_floor)
    c.v_floor = float(g.v_floor)
    c.seed_steps = int(getattr(g, "seed_steps", 0))
    c.seed_kappa = float(getattr(g, "seed_kappa", 1.0))
    c.seed_kmin = int(getattr(g, "seed_kmin", 1))
    c.seed_kmax = int(getattr(g, "seed_kmax", 1))
    for k, v in enumerate(getattr(g, "seed_scale", (0.0, 0.0, 0.0))):
        c.seed_scale[k] = float(v)
    c.cut_signal = float(getattr(g, "cut_signal", 0.0))
    c.cut_distance = float(getattr(g, "cut_distance", 0.0))
    return c


def reconstruct(lrf, grid, signals, seeds=None, threads=None):
    """Contracting-grid reconstruction of every event (FP64).

    Returns a dict: x, y, z, E, lnl, chi2 (float64), ndf, status (int32),
    path [n][K] (best node index per iteration) and gaps [n][K] (second-best
    minus best statistic per iteration)."""
    m = lrf if isinstance(lrf, Model) else Model(lrf)
    sig = np.ascontiguousarray(signals, dtype=np.float64)
    n = sig.shape[0]
    assert sig.shape[1] == m.n_sensors
    K = int(grid.iterations)
    out6 = np.empty((n, 6), np.float64)
    ndf = np.empty(n, np.int32)
    status = np.empty(n, np.int32)
    path = np.empty((n, K), np.int32)
    gaps = np.empty((n, K), np.float64)
    sd = None
    if seeds is not None:
        sd = np.ascontiguousarray(seeds, dtype=np.float64)
        assert sd.shape == (n, 4)
    cfg = _cfg(grid)
    lib().o_reconstruct(C.byref(m.c), C.byref(cfg), n, _dp(sig),
                        _dp(sd) if sd is not None else None, _dp(out6), _ip(ndf), _ip(status),
                        _ip(path), _dp(gaps), _threads(threads))
    return {"x": out6[:, 0], "y": out6[:, 1], "z": out6[:, 2], "E": out6[:, 3],
            "lnl": out6[:, 4], "chi2": out6[:, 5], "ndf": ndf, "status": status,
            "path": path, "gaps": gaps}


def lattice_stats(lrf, grid, n_event, center, step, nodes, threads=None):
    """Statistic (-lnL or chi2) at every node of a lattice, index
    (jz*ny + jy)*nx + jx."""
    m = lrf if isinstance(lrf, Model) else Model(lrf)
    n = np.ascontiguousarray(n_event, dtype=np.float64)
    c = np.ascontiguousarray(center, dtype=np.float64)
    s = np.ascontiguousarray(step, dtype=np.float64)
    nd = np.ascontiguousarray(nodes, dtype=np.int32)
    out = np.empty(int(np.prod(nodes)), np.float64)
    cfg = _cfg(grid)
    lib().o_lattice_stats(C.byref(m.c), C.byref(cfg), _dp(n), _dp(c), _dp(s), _ip(nd), _dp(out),
                          _threads(threads))
    return out


def node_eval(lrf, grid, n_event, x, y, z=0.0):
    """(stat, S, A, lnl, chi2) at one source position."""
    m = lrf if isinstance(lrf, Model) else Model(lrf)
    n = np.ascontiguousarray(n_event, dtype=np.float64)
    res = np.empty(5, np.float64)
    cfg = _cfg(grid)
    lib().o_node_eval_ext(C.byref(m.c), C.byref(cfg), _dp(n), float(x), float(y), float(z),
                          _dp(res))
    return res


def lrf_values(lrf, pos3, threads=None):
    """LRF of every sensor at every position: [n_pos][n_sensors]."""
    m = lrf if isinstance(lrf, Model) else Model(lrf)
    p = np.ascontiguousarray(pos3, dtype=np.float64)
    out = np.empty((p.shape[0], m.n_sensors), np.float64)
    lib().o_lrf_values(C.byref(m.c), p.shape[0], _dp(p), _dp(out), _threads(threads))
    return out


def expected_counts(lrf, pos3, etot, threads=None):
    """Means mu_i = A g_i L_i with sum_active mu_i = E_tot: [n_pos][n_sensors]."""
    m = lrf if isinstance(lrf, Model) else Model(lrf)
    p = np.ascontiguousarray(pos3, dtype=np.float64)
    e = np.ascontiguousarray(etot, dtype=np.float64)
    out = np.empty((p.shape[0], m.n_sensors), np.float64)
    lib().o_expected_counts(C.byref(m.c), p.shape[0], _dp(p), _dp(e), _dp(out), _threads(threads))
    return out


def crb(lrf, dim, pos3, A):
    """Cramer-Rao variances of the position parameters: [n_pos][dim]."""
    m = lrf if isinstance(lrf, Model) else Model(lrf)
    p = np.ascontiguousarray(pos3, dtype=np.float64)
    a = np.ascontiguousarray(A, dtype=np.float64)
    out = np.empty((p.shape[0], dim), np.float64)
    lib().o_crb(C.byref(m.c), int(dim), p.shape[0], _dp(p), _dp(a), _dp(out))
    return out


def spline1(coef, nb, lo, hi, u):
    c = np.ascontiguousarray(coef, dtype=np.float64)
    return np.array([lib().o_spline1(_dp(c), nb, lo, hi, float(x)) for x in np.atleast_1d(u)])


def spline1_du(coef, nb, lo, hi, u):
    c = np.ascontiguousarray(coef, dtype=np.float64)
    return np.array([lib().o_spline1_du(_dp(c), nb, lo, hi, float(x)) for x in np.atleast_1d(u)])


def deboor1(coef, nb, lo, hi, u):
    c = np.ascontiguousarray(coef, dtype=np.float64)
    return np.array([lib().o_deboor1(_dp(c), nb, lo, hi, float(x)) for x in np.atleast_1d(u)])


def spline2(coef, nb, lo, hi, u, w):
    c = np.ascontiguousarray(coef, dtype=np.float64)
    nbv = (C.c_int * 2)(*nb)
    lov = (C.c_double * 2)(*lo)
    hiv = (C.c_double * 2)(*hi)
    return np.array([lib().o_spline2(_dp(c), nbv, lov, hiv, float(a), float(b), None, None)
                     for a, b in zip(np.atleast_1d(u), np.atleast_1d(w))])


def basis(t):
    b = np.empty(4, np.float64)
    lib().o_basis(float(t), _dp(b))
    return b


def make_events(lrf, recipe, n, rngs, noiseless=False, threads=None):
    """Flood-field events from the LRF model itself: positions and E_tot
    from the workload streams, means from the oracle's LRF, Poisson counts
    (or the means themselves when noiseless).  Returns (signals float32
    [n][ns], truth dict)."""
    from workloads import draw_sources, poisson_counts
    pos, etot = draw_sources(recipe, n, rngs[0], rngs[1])
    mu = expected_counts(lrf, pos, etot, threads)
    if noiseless:
        sig = mu.astype(np.float32)
    else:
        sig = poisson_counts(mu, rngs[3])
    S = (lrf_values(lrf, pos, threads) * np.asarray(lrf.gain)[None, :]
         * np.asarray(lrf.active)[None, :]).sum(1)
    return sig, {"pos": pos, "etot": etot, "A": etot / S, "mu": mu}


def philox4x32_10(ctr, key):
    """Philox4x32-10 block: four 32-bit counter words, two key words."""
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().o_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def poisson(mu, event, stream, seed):
    k = (C.c_uint32 * 2)(seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return lib().o_poisson(float(mu), int(event), int(stream), k)


def generate(lrf, region, extent, z_lo, z_hi, e_lo, e_hi, n, seed, first=0, noiseless=False,
             threads=None):
    """Reference flood-field events (see the generator's definition in the
    library header).  Returns (signals [n][ns] float64, truth [n][4])."""
    m = lrf if isinstance(lrf, Model) else Model(lrf)
    truth = np.empty((n, 4), np.float64)
    sig = np.empty((n, m.n_sensors), np.float64)
    lib().o_generate(C.byref(m.c), int(region), float(extent), float(z_lo), float(z_hi),
                     float(e_lo), float(e_hi), int(bool(noiseless)), int(seed), int(first), int(n),
                     _dp(truth), _dp(sig), _threads(threads))
    return sig, truth


def reconstruct_seeded(lrf, refine, fallback, chi2ndf_max, signals, seeds, threads=None):
    """Seeded reconstruction: refine from seeds [n][4] = (x, y, z, log-variance)
    and re-run events with chi2/ndf above the threshold on the fallback grid."""
    m = lrf if isinstance(lrf, Model) else Model(lrf)
    sig = np.ascontiguousarray(signals, dtype=np.float64)
    sd = np.ascontiguousarray(seeds, dtype=np.float64)
    n = sig.shape[0]
    out6 = np.empty((n, 6), np.float64)
    ndf = np.empty(n, np.int32)
    status = np.empty(n, np.int32)
    r, f = _cfg(refine), _cfg(fallback)
    lib().o_reconstruct_seeded(C.byref(m.c), C.byref(r), C.byref(f), float(chi2ndf_max), n,
                               _dp(sig), _dp(sd), _dp(out6), _ip(ndf), _ip(status),
                               _threads(threads))
    return {"x": out6[:, 0], "y": out6[:, 1], "z": out6[:, 2], "E": out6[:, 3],
            "lnl": out6[:, 4], "chi2": out6[:, 5], "ndf": ndf, "status": status}


def _scfg(g):
    c = _SCfg()
    c.dims, c.stat, c.start = int(g.dims), int(g.stat), int(g.start)
    for k in range(3):
        c.step0[k] = float(g.step0[k])
    c.z_start, c.tol, c.max_iter = float(g.z_start), float(g.tol), int(g.max_iter)
    c.l_floor, c.v_floor = float(g.l_floor), float(g.v_floor)
    return c


def _vcfg(g):
    c = _VCfg()
    c.dims, c.stat, c.start = int(g.dims), int(g.stat), int(g.start)
    for k in range(3):
        c.step0[k] = float(g.step0[k])
    c.z_start, c.h, c.edm_tol = float(g.z_start), float(g.h), float(g.edm_tol)
    c.max_iter = int(g.max_iter)
    c.l_floor, c.v_floor = float(g.l_floor), float(g.v_floor)
    return c


def reconstruct_migrad(lrf, vcfg, signals, seeds=None, threads=None):
    """Variable-metric (Migrad-style) search per event (FP64).  Returns a
    dict: x, y, z, E, lnl, chi2, ndf, status, iters (accepted steps) and
    evals (statistic evaluations)."""
    m = lrf if isinstance(lrf, Model) else Model(lrf)
    sig = np.ascontiguousarray(signals, dtype=np.float64)
    n = sig.shape[0]
    assert sig.shape[1] == m.n_sensors
    out6 = np.empty((n, 6), np.float64)
    ndf = np.empty(n, np.int32)
    status = np.empty(n, np.int32)
    iters = np.empty(n, np.int32)
    evals = np.empty(n, np.int32)
    sd = None
    if seeds is not None:
        sd = np.ascontiguousarray(seeds, dtype=np.float64)
        assert sd.shape == (n, 4)
    c = _vcfg(vcfg)
    lib().o_reconstruct_migrad(C.byref(m.c), C.byref(c), n, _dp(sig),
                               _dp(sd) if sd is not None else None, _dp(out6), _ip(ndf),
                               _ip(status), _ip(iters), _ip(evals), _threads(threads))
    return {"x": out6[:, 0], "y": out6[:, 1], "z": out6[:, 2], "E": out6[:, 3],
            "lnl": out6[:, 4], "chi2": out6[:, 5], "ndf": ndf, "status": status,
            "iters": iters, "evals": evals}


def reconstruct_simplex(lrf, scfg, signals, seeds=None, threads=None):
    """Simplex (Nelder-Mead) search per event (FP64).  Returns a dict: x, y,
    z, E, lnl, chi2, ndf, status, iters (iterations run) and evals
    (statistic evaluations)."""
    m = lrf if isinstance(lrf, Model) else Model(lrf)
    sig = np.ascontiguousarray(signals, dtype=np.float64)
    n = sig.shape[0]
    assert sig.shape[1] == m.n_sensors
    out6 = np.empty((n, 6), np.float64)
    ndf = np.empty(n, np.int32)
    status = np.empty(n, np.int32)
    iters = np.empty(n, np.int32)
    evals = np.empty(n, np.int32)
    sd = None
    if seeds is not None:
        sd = np.ascontiguousarray(seeds, dtype=np.float64)
        assert sd.shape == (n, 4)
    c = _scfg(scfg)
    lib().o_reconstruct_simplex(C.byref(m.c), C.byref(c), n, _dp(sig),
                                _dp(sd) if sd is not None else None, _dp(out6), _ip(ndf),
                                _ip(status), _ip(iters), _ip(evals), _threads(threads))
    return {"x": out6[:, 0], "y": out6[:, 1], "z": out6[:, 2], "E": out6[:, 3],
            "lnl": out6[:, 4], "chi2": out6[:, 5], "ndf": ndf, "status": status,
            "iters": iters, "evals": evals}


class KnnCal:
    """Calibration set of the k-NN reconstruction: normalised signals of the
    active sensors (single precision, as defined in the oracle) and the
    known positions."""

    def __init__(self, lrf, signals, positions, threads=None):
        self.m = lrf if isinstance(lrf, Model) else Model(lrf)
        sig = np.ascontiguousarray(signals, dtype=np.float64)
        self.n = sig.shape[0]
        self.na = int(np.count_nonzero(self.m.active))
        self.cal = np.empty((self.n, max(self.na, 1)), np.float32)
        self.valid = np.empty(self.n, np.uint8)
        self.pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(self.n, 3)
        lib().o_knn_prepare(C.byref(self.m.c), self.n, _dp(sig),
                            self.cal.ctypes.data_as(C.POINTER(C.c_float)),
                            self.valid.ctypes.data_as(C.POINTER(C.c_uint8)), _threads(threads))


def knn_reconstruct(cal, k, signals, threads=None):
    """k-NN positions of events (Sec. 5.1.4).  Returns a dict: x, y, z,
    status, idx [n][k] (neighbours in order, -1 past the valid ones) and
    dist [n][k] (their single-precision squared distances)."""
    sig = np.ascontiguousarray(signals, dtype=np.float64)
    n = sig.shape[0]
    out3 = np.empty((n, 3), np.float64)
    status = np.empty(n, np.int32)
    idx = np.empty((n, k), np.int64)
    dist = np.empty((n, k), np.float32)
    lib().o_knn_reconstruct(C.byref(cal.m.c), cal.n,
                            cal.cal.ctypes.data_as(C.POINTER(C.c_float)),
                            cal.valid.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(cal.pos), int(k),
                            n, _dp(sig), _dp(out3), _ip(status),
                            idx.ctypes.data_as(C.POINTER(C.c_int64)),
                            dist.ctypes.data_as(C.POINTER(C.c_float)), _threads(threads))
    return {"x": out3[:, 0], "y": out3[:, 1], "z": out3[:, 2], "status": status, "idx": idx,
            "dist": dist}
