"""Thin ctypes binding of the C ABI in include/ants.h.

Argument marshalling only: every step of the reconstruction runs in the HIP
library libants.so built next to this file.  PyTorch provides device memory
and streams.  Importing this module fails loudly when the library is
missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libants.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as "
                      f"g; g.build()')")

_lib = C.CDLL(LIB_PATH)

OK, E_ARG, E_FORMAT, E_DEVICE, E_NOMEM, E_UNSUPPORTED, E_STATE = 0, -1, -2, -3, -4, -5, -6
EV_EMPTY, EV_BAD_INPUT, EV_NO_ACTIVE, EV_NO_VALID_NODE, EV_FALLBACK, EV_TIE = 1, 2, 4, 8, 16, 32
LRF_AXIAL, LRF_XY, LRF_RZ = 1, 2, 3
STAT_ML, STAT_CHI2 = 0, 1
START_COG, START_MAXSENSOR, START_SEED = 0, 1, 2


class AntsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ants error {code}: {msg}")
        self.code = code


class LrfDesc(C.Structure):
    _fields_ = [("n_sensors", C.c_int32), ("sensor_xy", C.POINTER(C.c_double)),
                ("gain", C.POINTER(C.c_double)), ("active", C.POINTER(C.c_uint8)),
                ("kind", C.c_int32), ("shared", C.c_int32), ("n_knots", C.c_int32 * 2),
                ("lo", C.c_double * 2), ("hi", C.c_double * 2), ("coef", C.POINTER(C.c_double))]


class GridCfg(C.Structure):
    _fields_ = [("nodes", C.c_int32 * 3), ("iterations", C.c_int32), ("shrink", C.c_double),
                ("step0", C.c_double * 3), ("z_start", C.c_double), ("stat", C.c_int32),
                ("start", C.c_int32), ("l_floor", C.c_double), ("v_floor", C.c_double),
                ("screen_scale", C.c_double)]


class GenCfg(C.Structure):
    _fields_ = [("region", C.c_int32), ("extent", C.c_double), ("z_lo", C.c_double),
                ("z_hi", C.c_double), ("e_lo", C.c_double), ("e_hi", C.c_double),
                ("noiseless", C.c_int32)]


class Out(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in
                ("x", "y", "z", "E", "lnl", "chi2", "ndf", "status", "path", "n_fp64")]


_vp = C.c_void_p
_lib.ants_last_error.restype = C.c_char_p
_lib.ants_version.restype = C.c_char_p
_lib.ants_lrfset_create.argtypes = [C.POINTER(LrfDesc), C.POINTER(_vp)]
_lib.ants_lrfset_destroy.argtypes = [_vp]
_lib.ants_lrfset_info.argtypes = [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int32)]
_lib.ants_reconstruct.argtypes = [_vp, C.POINTER(GridCfg), C.c_int64, _vp, _vp, Out, _vp]

_lib.ants_generate.argtypes = [_vp, C.POINTER(GenCfg), C.c_int64, C.c_uint64, C.c_uint64, _vp,
                               _vp, _vp]

EXPORTED = ("ants_last_error", "ants_version", "ants_lrfset_create", "ants_lrfset_destroy",
            "ants_lrfset_info", "ants_reconstruct", "ants_generate")


def _check(code):
    if code != OK:
        raise AntsError(code, _lib.ants_last_error().decode())


def version() -> str:
    return _lib.ants_version().decode()


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class LrfSet:
    """Device copy of a detector model.  `model` has the fields kind, sxy,
    gain, active, shared, nb, lo, hi, coef (see workloads.LRFSet)."""

    def __init__(self, model):
        self._h = _vp()
        sxy = np.ascontiguousarray(model.sxy, np.float64)
        gain = np.ascontiguousarray(model.gain, np.float64)
        active = np.ascontiguousarray(model.active, np.uint8)
        coef = np.ascontiguousarray(model.coef, np.float64)
        d = LrfDesc()
        d.n_sensors = sxy.shape[0]
        d.sensor_xy = _dptr(sxy)
        d.gain = _dptr(gain)
        d.active = active.ctypes.data_as(C.POINTER(C.c_uint8))
        d.kind = int(model.kind)
        d.shared = int(model.shared)
        d.n_knots[0], d.n_knots[1] = int(model.nb[0]), int(model.nb[1])
        d.lo[0], d.lo[1] = float(model.lo[0]), float(model.lo[1])
        d.hi[0], d.hi[1] = float(model.hi[0]), float(model.hi[1])
        d.coef = _dptr(coef)
        _check(_lib.ants_lrfset_create(C.byref(d), C.byref(self._h)))
        ns, na, kind = C.c_int32(), C.c_int32(), C.c_int32()
        _check(_lib.ants_lrfset_info(self._h, C.byref(ns), C.byref(na), C.byref(kind)))
        self.n_sensors, self.n_active, self.kind = ns.value, na.value, kind.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _lib.ants_lrfset_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def grid_cfg(g, screen_scale: float = 0.0) -> GridCfg:
    """GridCfg from an object with nodes, iterations, shrink, step0, z_start,
    stat, start, l_floor, v_floor (see workloads.GridCfg)."""
    c = GridCfg()
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
    c.screen_scale = float(screen_scale)
    return c


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def alloc_out(n, iterations=0, device="cuda", path=False, n_fp64=False):
    import torch
    f = dict(dtype=torch.float32, device=device)
    i = dict(dtype=torch.int32, device=device)
    out = {k: torch.empty(n, **f) for k in ("x", "y", "z", "E", "lnl", "chi2")}
    out["ndf"] = torch.empty(n, **i)
    out["status"] = torch.empty(n, **i)
    if path:
        out["path"] = torch.empty((n, max(iterations, 1)), **i)
    if n_fp64:
        out["n_fp64"] = torch.empty(n, **i)
    return out


def _out_struct(out):
    o = Out()
    for k in ("x", "y", "z", "E", "lnl", "chi2", "ndf", "status", "path", "n_fp64"):
        t = out.get(k)
        setattr(o, k, t.data_ptr() if t is not None else None)
    return o


def reconstruct(lrfset: LrfSet, cfg: GridCfg, signals, seeds=None, out=None, stream=None,
                path=False, n_fp64=False):
    """Contracting-grid reconstruction of `signals` ([n][n_sensors] float32,
    on the GPU).  Returns the dict of output tensors (asynchronous)."""
    import torch
    assert signals.dtype == torch.float32 and signals.is_cuda and signals.is_contiguous()
    n = signals.shape[0]
    assert signals.dim() == 2 and signals.shape[1] == lrfset.n_sensors, signals.shape
    if out is None:
        out = alloc_out(n, cfg.iterations, signals.device, path, n_fp64)
    sp = None
    if seeds is not None:
        assert seeds.dtype == torch.float32 and seeds.is_cuda and seeds.is_contiguous()
        assert seeds.shape == (n, 4)
        sp = seeds.data_ptr()
    _check(_lib.ants_reconstruct(lrfset.handle, C.byref(cfg), n, signals.data_ptr(), sp,
                                 _out_struct(out), _stream_handle(stream)))
    return out


def gen_cfg(recipe, noiseless=False) -> GenCfg:
    """GenCfg from an event recipe (region, extent, e_lo, e_hi, z_lo, z_hi,
    three_d; see workloads.EventRecipe)."""
    c = GenCfg()
    c.region = 0 if recipe.region == "disc" else 1
    c.extent = float(recipe.extent)
    c.z_lo = float(recipe.z_lo)
    c.z_hi = float(recipe.z_hi) if recipe.three_d else float(recipe.z_lo)
    c.e_lo = float(recipe.e_lo)
    c.e_hi = float(recipe.e_hi)
    c.noiseless = 1 if noiseless else 0
    return c


def generate(lrfset: LrfSet, cfg: GenCfg, n: int, seed: int, first: int = 0, signals=None,
             truth=True, stream=None):
    """Draw n flood-field events on the GPU.  Returns (signals [n][ns],
    truth [n][4] = x, y, z, E_tot or None)."""
    import torch
    if signals is None:
        signals = torch.empty((n, lrfset.n_sensors), dtype=torch.float32, device="cuda")
    t = torch.empty((n, 4), dtype=torch.float32, device=signals.device) if truth else None
    _check(_lib.ants_generate(lrfset.handle, C.byref(cfg), n, seed, first, signals.data_ptr(),
                              t.data_ptr() if t is not None else None, _stream_handle(stream)))
    return signals, t
