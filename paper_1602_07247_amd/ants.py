"""Thin ctypes binding of the C ABI in include/ants.h.

Argument marshalling only: every step of the reconstruction runs in the HIP
library libants.so built next to this file.  PyTorch provides device memory
and streams.  Importing this module fails loudly when the library is
missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
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
LRF_AXIAL, LRF_XY, LRF_RZ, LRF_COMPOSITE, LRF_SLICED = 1, 2, 3, 4, 5
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
                ("lo", C.c_double * 2), ("hi", C.c_double * 2), ("coef", C.POINTER(C.c_double)),
                ("xy_knots", C.c_int32 * 2), ("xy_lo", C.c_double * 2), ("xy_hi", C.c_double * 2),
                ("xy_coef", C.POINTER(C.c_double)), ("xy_shared", C.c_int32),
                ("n_planes", C.c_int32), ("z_lo", C.c_double), ("z_hi", C.c_double)]


class GridCfg(C.Structure):
    _fields_ = [("nodes", C.c_int32 * 3), ("iterations", C.c_int32), ("shrink", C.c_double),
                ("step0", C.c_double * 3), ("z_start", C.c_double), ("stat", C.c_int32),
                ("start", C.c_int32), ("l_floor", C.c_double), ("v_floor", C.c_double),
                ("screen_scale", C.c_double), ("seed_steps", C.c_int32),
                ("seed_kappa", C.c_double), ("seed_kmin", C.c_int32), ("seed_kmax", C.c_int32),
                ("seed_scale", C.c_double * 3), ("cut_signal", C.c_double),
                ("cut_distance", C.c_double)]


class GenCfg(C.Structure):
    _fields_ = [("region", C.c_int32), ("extent", C.c_double), ("z_lo", C.c_double),
                ("z_hi", C.c_double), ("e_lo", C.c_double), ("e_hi", C.c_double),
                ("noiseless", C.c_int32)]


class MlpCfg(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("hidden", C.c_int32), ("n_layers", C.c_int32),
                ("seed", C.c_uint64), ("pos_scale", C.c_double * 3),
                ("pos_offset", C.c_double * 3)]


class AdamCfg(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double)]


class TrainCfg(C.Structure):
    _fields_ = [("n_train", C.c_int64), ("n_val", C.c_int64), ("batch", C.c_int32),
                ("epochs", C.c_int32), ("adam", AdamCfg), ("lr_decay", C.c_double),
                ("seed", C.c_uint64), ("events", GenCfg)]


class Chunk(C.Structure):
    _fields_ = [("set", C.c_int32), ("n_events", C.c_int64), ("d_signals", C.c_void_p),
                ("out_offset", C.c_int64)]


class Plan(C.Structure):
    _fields_ = [("events_per_item", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("table_in_lds", C.c_int32)]


class GridPlan(C.Structure):
    _fields_ = [("waves_per_block", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("screen", C.c_int32)]


class Fit2dCfg(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nb", C.c_int32 * 2), ("lo", C.c_double * 2),
                ("hi", C.c_double * 2), ("ridge", C.c_double), ("chi2ndf_max", C.c_double),
                ("d_base", C.c_void_p), ("base_nb", C.c_int32), ("base_lo", C.c_double),
                ("base_hi", C.c_double), ("ev_z_lo", C.c_double), ("ev_z_hi", C.c_double)]


class MigradCfg(C.Structure):
    _fields_ = [("dims", C.c_int32), ("stat", C.c_int32), ("start", C.c_int32),
                ("step0", C.c_double * 3), ("z_start", C.c_double), ("h", C.c_double),
                ("edm_tol", C.c_double), ("max_iter", C.c_int32), ("l_floor", C.c_double),
                ("v_floor", C.c_double)]


class SimplexCfg(C.Structure):
    _fields_ = [("dims", C.c_int32), ("stat", C.c_int32), ("start", C.c_int32),
                ("step0", C.c_double * 3), ("z_start", C.c_double), ("tol", C.c_double),
                ("max_iter", C.c_int32), ("l_floor", C.c_double), ("v_floor", C.c_double)]


class FitCfg(C.Structure):
    _fields_ = [("nb", C.c_int32), ("lo", C.c_double), ("hi", C.c_double), ("ridge", C.c_double),
                ("chi2ndf_max", C.c_double)]


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
_lib.ants_lrf_write.argtypes = [C.POINTER(LrfDesc), C.c_char_p]
_lib.ants_lrfset_save.argtypes = [_vp, C.c_char_p]
_lib.ants_lrfset_load.argtypes = [C.c_char_p, C.POINTER(_vp)]

_lib.ants_generate.argtypes = [_vp, C.POINTER(GenCfg), C.c_int64, C.c_uint64, C.c_uint64, _vp,
                               _vp, _vp]

_lib.ants_mlp_create.argtypes = [C.POINTER(MlpCfg), C.POINTER(_vp)]
_lib.ants_mlp_destroy.argtypes = [_vp]
_lib.ants_mlp_num_params.argtypes = [_vp]
_lib.ants_mlp_num_params.restype = C.c_int64
_lib.ants_mlp_get_params.argtypes = [_vp, C.POINTER(C.c_float), C.c_int64]
_lib.ants_mlp_set_params.argtypes = [_vp, C.POINTER(C.c_float), C.c_int64]
_lib.ants_mlp_forward.argtypes = [_vp, _vp, C.c_int64, _vp, _vp, _vp]
_lib.ants_mlp_grad.argtypes = [_vp, _vp, C.c_int64, _vp, _vp, _vp, _vp, _vp]
_lib.ants_mlp_train_step.argtypes = [_vp, _vp, C.c_int64, _vp, _vp, C.POINTER(AdamCfg), _vp, _vp]
_lib.ants_mlp_train.argtypes = [_vp, _vp, C.POINTER(TrainCfg), C.POINTER(C.c_double), _vp]
_lib.ants_mlp_save.argtypes = [_vp, C.c_char_p]
_lib.ants_mlp_load.argtypes = [C.c_char_p, C.POINTER(_vp)]
_lib.ants_reconstruct_seeded.argtypes = [_vp, _vp, C.POINTER(GridCfg), C.POINTER(GridCfg),
                                         C.c_double, C.c_int64, _vp, _vp, Out, _vp, _vp]
_lib.ants_reconstruct_seeded_noalloc.argtypes = _lib.ants_reconstruct_seeded.argtypes
NOALLOC_MAX_EVENTS = 1 << 20

_lib.ants_reconstruct_multi.argtypes = [C.POINTER(_vp), C.POINTER(GridCfg), C.c_int32,
                                        C.POINTER(Chunk), C.c_int32, C.POINTER(Plan), Out, _vp]
_lib.ants_autotune_multi.argtypes = [C.POINTER(_vp), C.POINTER(GridCfg), C.c_int32,
                                     C.POINTER(Chunk), C.c_int32, C.c_int64, Out, C.POINTER(Plan),
                                     C.POINTER(C.c_double), _vp]

_lib.ants_autotune.argtypes = [_vp, C.POINTER(GridCfg), C.c_int64, _vp, _vp, Out,
                               C.POINTER(GridPlan), C.POINTER(C.c_double), _vp]
_lib.ants_set_plan.argtypes = [_vp, C.POINTER(GridCfg), C.POINTER(GridPlan)]
_lib.ants_reconstruct_simplex.argtypes = [_vp, C.POINTER(SimplexCfg), C.c_int64, _vp, _vp, Out,
                                          _vp, _vp]
_lib.ants_reconstruct_migrad.argtypes = [_vp, C.POINTER(MigradCfg), C.c_int64, _vp, _vp, Out,
                                          _vp, _vp]

_lib.ants_knn_create.argtypes = [_vp, C.c_int64, _vp, _vp, C.POINTER(_vp), _vp]
_lib.ants_knn_destroy.argtypes = [_vp]
_lib.ants_knn_reconstruct.argtypes = [_vp, C.c_int32, C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp]

_lib.ants_fit_axial_lrf.argtypes = [_vp, C.POINTER(FitCfg), C.c_int64, _vp, C.c_int64, Out, _vp,
                                    _vp, _vp]
_lib.ants_fit_axial_lrf_grouped.argtypes = [_vp, C.POINTER(FitCfg), C.c_int32, _vp, C.c_int64,
                                            _vp, C.c_int64, Out, _vp, _vp, _vp, _vp]
_lib.ants_fit_lrf2d_grouped.argtypes = [_vp, C.POINTER(Fit2dCfg), C.c_int32, _vp, C.c_int64, _vp,
                                        C.c_int64, Out, _vp, _vp, _vp, _vp]
_lib.ants_fit_axial_gains.argtypes = [_vp, C.POINTER(FitCfg), C.c_int32, _vp, _vp, C.c_int64,
                                      _vp, C.c_int64, Out, _vp, _vp, _vp, _vp]

EXPORTED = ("ants_last_error", "ants_version", "ants_lrfset_create", "ants_lrfset_destroy",
            "ants_lrfset_info", "ants_reconstruct", "ants_generate", "ants_mlp_create",
            "ants_mlp_destroy", "ants_mlp_num_params", "ants_mlp_get_params",
            "ants_mlp_set_params", "ants_mlp_forward", "ants_mlp_grad", "ants_mlp_train_step",
            "ants_mlp_train", "ants_mlp_save", "ants_mlp_load", "ants_reconstruct_seeded",
            "ants_reconstruct_seeded_noalloc",
            "ants_reconstruct_multi", "ants_autotune_multi", "ants_fit_axial_lrf",
            "ants_lrf_write", "ants_lrfset_save", "ants_lrfset_load",
            "ants_reconstruct_simplex", "ants_knn_create", "ants_knn_destroy",
            "ants_knn_reconstruct", "ants_autotune", "ants_set_plan",
            "ants_fit_axial_lrf_grouped", "ants_fit_axial_gains", "ants_reconstruct_migrad",
            "ants_fit_lrf2d_grouped")


def _check(code):
    if code != OK:
        raise AntsError(code, _lib.ants_last_error().decode())


def version() -> str:
    return _lib.ants_version().decode()


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def lrf_desc(model):
    """(LrfDesc, arrays it points into) for a detector model with the fields
    kind, sxy, gain, active, shared, nb, lo, hi, coef (see workloads.LRFSet)."""
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
    keep = [sxy, gain, active, coef]
    xc = getattr(model, "xy_coef", None)
    if xc is not None:
        xc = np.ascontiguousarray(xc, np.float64)
        keep.append(xc)
        d.xy_coef = _dptr(xc)
        d.xy_knots[0], d.xy_knots[1] = int(model.xy_nb[0]), int(model.xy_nb[1])
        d.xy_lo[0], d.xy_lo[1] = float(model.xy_lo[0]), float(model.xy_lo[1])
        d.xy_hi[0], d.xy_hi[1] = float(model.xy_hi[0]), float(model.xy_hi[1])
        d.xy_shared = int(model.xy_shared)
    d.n_planes = int(getattr(model, "n_planes", 0))
    d.z_lo = float(getattr(model, "z_lo", 0.0))
    d.z_hi = float(getattr(model, "z_hi", 0.0))
    return d, keep


def write_lrf(model, path):
    """Write a detector model as an LRF-set file (ants_lrf_write)."""
    d, keep = lrf_desc(model)
    _check(_lib.ants_lrf_write(C.byref(d), os.fsencode(path)))


class LrfSet:
    """Device copy of a detector model (see lrf_desc), or of an LRF-set file
    with LrfSet.load(path)."""

    def __init__(self, model=None, _handle=None):
        self._h = _vp()
        if _handle is not None:
            self._h = _handle
        else:
            d, keep = lrf_desc(model)
            _check(_lib.ants_lrfset_create(C.byref(d), C.byref(self._h)))
        ns, na, kind = C.c_int32(), C.c_int32(), C.c_int32()
        _check(_lib.ants_lrfset_info(self._h, C.byref(ns), C.byref(na), C.byref(kind)))
        self.n_sensors, self.n_active, self.kind = ns.value, na.value, kind.value

    @classmethod
    def load(cls, path):
        h = _vp()
        _check(_lib.ants_lrfset_load(os.fsencode(path), C.byref(h)))
        return cls(_handle=h)

    def save(self, path):
        _check(_lib.ants_lrfset_save(self._h, os.fsencode(path)))

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
    c.seed_steps = int(getattr(g, "seed_steps", 0))
    c.seed_kappa = float(getattr(g, "seed_kappa", 1.0))
    c.seed_kmin = int(getattr(g, "seed_kmin", 1))
    c.seed_kmax = int(getattr(g, "seed_kmax", 1))
    for k, v in enumerate(getattr(g, "seed_scale", (0.0, 0.0, 0.0))):
        c.seed_scale[k] = float(v)
    c.cut_signal = float(getattr(g, "cut_signal", 0.0))
    c.cut_distance = float(getattr(g, "cut_distance", 0.0))
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


def simplex_cfg(g) -> SimplexCfg:
    """SimplexCfg from an object with dims, stat, start, step0, z_start, tol,
    max_iter, l_floor, v_floor (see workloads.SimplexCfg)."""
    c = SimplexCfg()
    c.dims, c.stat, c.start = int(g.dims), int(g.stat), int(g.start)
    for k in range(3):
        c.step0[k] = float(g.step0[k])
    c.z_start, c.tol, c.max_iter = float(g.z_start), float(g.tol), int(g.max_iter)
    c.l_floor, c.v_floor = float(g.l_floor), float(g.v_floor)
    return c


def reconstruct_simplex(lrfset: LrfSet, cfg: SimplexCfg, signals, seeds=None, out=None,
                        stream=None, iters=True, n_eval=False):
    """Simplex search per event (ants_reconstruct_simplex).  Returns the
    dict of output tensors, with "iters" (iterations per event) when
    iters=True and "n_fp64" (statistic evaluations) when n_eval=True
    (asynchronous)."""
    import torch
    assert signals.dtype == torch.float32 and signals.is_cuda and signals.is_contiguous()
    n = signals.shape[0]
    assert signals.dim() == 2 and signals.shape[1] == lrfset.n_sensors, signals.shape
    if out is None:
        out = alloc_out(n, 0, signals.device, n_fp64=n_eval)
    if iters and "iters" not in out:
        out["iters"] = torch.empty(n, dtype=torch.int32, device=signals.device)
    sp = None
    if seeds is not None:
        assert seeds.dtype == torch.float32 and seeds.is_cuda and seeds.is_contiguous()
        assert seeds.shape == (n, 4)
        sp = seeds.data_ptr()
    it = out["iters"].data_ptr() if "iters" in out else None
    _check(_lib.ants_reconstruct_simplex(lrfset.handle, C.byref(cfg), n, signals.data_ptr(), sp,
                                         _out_struct(out), it, _stream_handle(stream)))
    return out


def migrad_cfg(g) -> MigradCfg:
    """MigradCfg from an object with dims, stat, start, step0, z_start, h,
    edm_tol, max_iter, l_floor, v_floor (see workloads.MigradCfg)."""
    c = MigradCfg()
    c.dims, c.stat, c.start = int(g.dims), int(g.stat), int(g.start)
    for k in range(3):
        c.step0[k] = float(g.step0[k])
    c.z_start, c.h, c.edm_tol = float(g.z_start), float(g.h), float(g.edm_tol)
    c.max_iter = int(g.max_iter)
    c.l_floor, c.v_floor = float(g.l_floor), float(g.v_floor)
    return c


def reconstruct_migrad(lrfset: LrfSet, cfg: MigradCfg, signals, seeds=None, out=None,
                       stream=None, iters=True, n_eval=False):
    """Variable-metric search per event (ants_reconstruct_migrad).  Returns
    the dict of output tensors, with "iters" (accepted steps per event) when
    iters=True and "n_fp64" (statistic evaluations) when n_eval=True
    (asynchronous)."""
    import torch
    assert signals.dtype == torch.float32 and signals.is_cuda and signals.is_contiguous()
    n = signals.shape[0]
    assert signals.dim() == 2 and signals.shape[1] == lrfset.n_sensors, signals.shape
    if out is None:
        out = alloc_out(n, 0, signals.device, n_fp64=n_eval)
    if iters and "iters" not in out:
        out["iters"] = torch.empty(n, dtype=torch.int32, device=signals.device)
    sp = None
    if seeds is not None:
        assert seeds.dtype == torch.float32 and seeds.is_cuda and seeds.is_contiguous()
        assert seeds.shape == (n, 4)
        sp = seeds.data_ptr()
    it = out["iters"].data_ptr() if "iters" in out else None
    _check(_lib.ants_reconstruct_migrad(lrfset.handle, C.byref(cfg), n, signals.data_ptr(), sp,
                                        _out_struct(out), it, _stream_handle(stream)))
    return out


class Knn:
    """k-NN calibration set (ants_knn_create): signals [m][n_sensors] and
    positions [m][3], FP32 device tensors of `lrfset`'s detector."""

    def __init__(self, lrfset: LrfSet, signals, positions, stream=None):
        import torch
        assert signals.dtype == torch.float32 and signals.is_cuda and signals.is_contiguous()
        assert signals.shape[1] == lrfset.n_sensors
        pos = positions.to(torch.float32).contiguous()
        assert pos.shape == (signals.shape[0], 3) and pos.is_cuda
        self._h = _vp()
        self.m = signals.shape[0]
        _check(_lib.ants_knn_create(lrfset.handle, self.m, signals.data_ptr(), pos.data_ptr(),
                                    C.byref(self._h), _stream_handle(stream)))
        self._keep = (signals, pos)   # until the stream has copied them

    def reconstruct(self, k, signals, neighbours=False, stream=None):
        """Positions [n][3] and status [n] (and idx, dist [n][k] when
        neighbours=True) as device tensors (asynchronous)."""
        import torch
        assert signals.dtype == torch.float32 and signals.is_cuda and signals.is_contiguous()
        n = signals.shape[0]
        dev = signals.device
        out = {"xyz": torch.empty((n, 3), dtype=torch.float32, device=dev),
               "status": torch.empty(n, dtype=torch.int32, device=dev)}
        if neighbours:
            out["idx"] = torch.empty((n, k), dtype=torch.int32, device=dev)
            out["dist"] = torch.empty((n, k), dtype=torch.float32, device=dev)
        _check(_lib.ants_knn_reconstruct(self._h, int(k), n, signals.data_ptr(),
                                         out["xyz"].data_ptr(), out["status"].data_ptr(),
                                         out["idx"].data_ptr() if neighbours else None,
                                         out["dist"].data_ptr() if neighbours else None,
                                         _stream_handle(stream)))
        return out

    def close(self):
        if self._h:
            _lib.ants_knn_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(lrfset: LrfSet, cfg: GridCfg, signals, seeds=None, stream=None):
    """Time the launch plans of `cfg` on `signals` and store the fastest in
    the set (ants_autotune).  Returns (GridPlan, per-candidate ms)."""
    n = signals.shape[0]
    scratch = alloc_out(n, 0, signals.device)
    best = GridPlan()
    ms = np.zeros(12, np.float64)
    _check(_lib.ants_autotune(lrfset.handle, C.byref(cfg), n, signals.data_ptr(),
                              seeds.data_ptr() if seeds is not None else None,
                              _out_struct(scratch), C.byref(best),
                              ms.ctypes.data_as(C.POINTER(C.c_double)), _stream_handle(stream)))
    return best, ms


def set_plan(lrfset: LrfSet, cfg: GridCfg, plan):
    """Store (or, with plan=None, remove) the set's launch plan for cfg."""
    _check(_lib.ants_set_plan(lrfset.handle, C.byref(cfg),
                              C.byref(plan) if plan is not None else None))


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


def adam_cfg(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8) -> AdamCfg:
    return AdamCfg(lr, beta1, beta2, eps)


class Mlp:
    """Learned-seed network handle (parameters, optimiser state, workspace)."""

    def __init__(self, n_in=37, hidden=256, layers=3, seed=1, pos_scale=(90.0, 90.0, 25.0),
                 pos_offset=(0.0, 0.0, 25.0), _handle=None):
        self._h = _vp()
        if _handle is not None:
            self._h = _handle
        else:
            c = MlpCfg()
            c.n_in, c.hidden, c.n_layers, c.seed = n_in, hidden, layers, seed
            for k in range(3):
                c.pos_scale[k] = pos_scale[k]
                c.pos_offset[k] = pos_offset[k]
            _check(_lib.ants_mlp_create(C.byref(c), C.byref(self._h)))
        self.n_params = int(_lib.ants_mlp_num_params(self._h))

    @property
    def handle(self):
        return self._h

    @classmethod
    def load(cls, path):
        h = _vp()
        _check(_lib.ants_mlp_load(str(path).encode(), C.byref(h)))
        return cls(_handle=h)

    def save(self, path):
        _check(_lib.ants_mlp_save(self._h, str(path).encode()))

    def get_params(self):
        out = np.empty(self.n_params, np.float32)
        _check(_lib.ants_mlp_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float)),
                                        self.n_params))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        _check(_lib.ants_mlp_set_params(self._h, p.ctypes.data_as(C.POINTER(C.c_float)),
                                        self.n_params))

    def forward(self, lrfset, signals, stream=None):
        import torch
        pred = torch.empty((signals.shape[0], 4), dtype=torch.float32, device=signals.device)
        _check(_lib.ants_mlp_forward(self._h, lrfset.handle, signals.shape[0], signals.data_ptr(),
                                     pred.data_ptr(), _stream_handle(stream)))
        return pred

    def grad(self, lrfset, signals, targets, stream=None):
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device=signals.device)
        loss = torch.empty(1, dtype=torch.float32, device=signals.device)
        t = targets.contiguous()
        _check(_lib.ants_mlp_grad(self._h, lrfset.handle, signals.shape[0], signals.data_ptr(),
                                  t.data_ptr(), g.data_ptr(), loss.data_ptr(),
                                  _stream_handle(stream)))
        return g, loss

    def train_step(self, lrfset, signals, targets, adam, stream=None):
        import torch
        loss = torch.empty(1, dtype=torch.float32, device=signals.device)
        t = targets.contiguous()
        _check(_lib.ants_mlp_train_step(self._h, lrfset.handle, signals.shape[0],
                                        signals.data_ptr(), t.data_ptr(), C.byref(adam),
                                        loss.data_ptr(), _stream_handle(stream)))
        return loss

    def train(self, lrfset, recipe, n_train, n_val, batch=4096, epochs=4, lr=1e-3,
              lr_decay=0.7, seed=11, stream=None):
        c = TrainCfg()
        c.n_train, c.n_val, c.batch, c.epochs = n_train, n_val, batch, epochs
        c.adam = adam_cfg(lr)
        c.lr_decay = lr_decay
        c.seed = seed
        c.events = gen_cfg(recipe)
        losses = np.zeros(2 * epochs, np.float64)
        _check(_lib.ants_mlp_train(self._h, lrfset.handle, C.byref(c),
                                   losses.ctypes.data_as(C.POINTER(C.c_double)),
                                   _stream_handle(stream)))
        return losses.reshape(epochs, 2)

    def close(self):
        if self._h:
            _lib.ants_mlp_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reconstruct_seeded(lrfset, mlp, refine: GridCfg, fallback: GridCfg, chi2ndf_max, signals,
                       seeds=None, out=None, stream=None, n_fp64=False, noalloc=False, nfb=None):
    """Seeded reconstruction (network seeds, or explicit seeds [n][4] in mm
    with a log-variance).  Returns (outputs, device tensor with the number of
    fallback events).  noalloc=True calls the allocation-free entry point
    (at most NOALLOC_MAX_EVENTS events; pass `out` and `nfb` to allocate
    nothing here either)."""
    import torch
    n = signals.shape[0]
    if out is None:
        out = alloc_out(n, refine.iterations, signals.device, False, n_fp64)
    if nfb is None:
        nfb = torch.zeros(1, dtype=torch.int32, device=signals.device)
    sp = None
    if seeds is not None:
        assert seeds.shape == (n, 4) and seeds.dtype == torch.float32 and seeds.is_contiguous()
        sp = seeds.data_ptr()
    fn = _lib.ants_reconstruct_seeded_noalloc if noalloc else _lib.ants_reconstruct_seeded
    _check(fn(lrfset.handle, mlp.handle if mlp is not None else None, C.byref(refine),
              C.byref(fallback), float(chi2ndf_max), n, signals.data_ptr(), sp, _out_struct(out),
              nfb.data_ptr(), _stream_handle(stream)))
    return out, nfb


def _multi_args(sets, cfgs, chunks):
    hs = (_vp * len(sets))(*[x.handle.value for x in sets])
    cs = (GridCfg * len(cfgs))(*cfgs)
    ch = (Chunk * len(chunks))()
    for i, (si, sig, off) in enumerate(chunks):
        ch[i].set = si
        ch[i].n_events = sig.shape[0]
        ch[i].d_signals = sig.data_ptr() if sig.shape[0] else None
        ch[i].out_offset = off
    return hs, cs, ch


def reconstruct_multi(sets, cfgs, chunks, n_out, plan=None, out=None, stream=None):
    """One persistent launch over chunks [(set index, signals tensor,
    output offset)] of several detectors."""
    if out is None:
        out = alloc_out(n_out, 0, chunks[0][1].device if chunks else "cuda")
    hs, cs, ch = _multi_args(sets, cfgs, chunks)
    _check(_lib.ants_reconstruct_multi(hs, cs, len(sets), ch, len(chunks),
                                       C.byref(plan) if plan is not None else None,
                                       _out_struct(out), _stream_handle(stream)))
    return out


def autotune_multi(sets, cfgs, chunks, sample_events, stream=None):
    """Time the candidate plans on a sample of sample_events events spread
    over the stream and store each set's part of the best plan in its
    handle (used by reconstruct_multi with plan=None); returns (best Plan
    for the first set, per-candidate milliseconds)."""
    hs, cs, ch = _multi_args(sets, cfgs, chunks)
    scratch = alloc_out(sample_events, 0, chunks[0][1].device)
    best = Plan()
    ms = np.zeros(3 + 6 * len(sets), np.float64)
    _check(_lib.ants_autotune_multi(hs, cs, len(sets), ch, len(chunks), sample_events,
                                    _out_struct(scratch), C.byref(best),
                                    ms.ctypes.data_as(C.POINTER(C.c_double)),
                                    _stream_handle(stream)))
    return best, ms


def fit_cfg(nb, lo, hi, ridge=1e-9, chi2ndf_max=0.0) -> FitCfg:
    c = FitCfg()
    c.nb, c.lo, c.hi, c.ridge, c.chi2ndf_max = int(nb), float(lo), float(hi), float(ridge), \
        float(chi2ndf_max)
    return c


def fit_axial_lrf(lrfset: LrfSet, cfg: FitCfg, signals, rec, stream=None):
    """Shared axial LRF fitted to `signals` ([n][n_sensors] float32, GPU) and
    the reconstruction `rec` (dict of tensors from `reconstruct`) on the
    sensors of `lrfset`.  Returns (coefficients [nb+2] float64, counts [2]
    int64 = events, pairs used), device tensors (asynchronous)."""
    import torch
    assert signals.dtype == torch.float32 and signals.is_cuda and signals.dim() == 2
    assert signals.stride(1) == 1 and signals.shape[1] == lrfset.n_sensors
    n = signals.shape[0]
    coef = torch.empty(cfg.nb + 2, dtype=torch.float64, device=signals.device)
    counts = torch.empty(2, dtype=torch.int64, device=signals.device)
    _check(_lib.ants_fit_axial_lrf(lrfset.handle, C.byref(cfg), n, signals.data_ptr(),
                                   signals.stride(0), _out_struct(rec), coef.data_ptr(),
                                   counts.data_ptr(), _stream_handle(stream)))
    return coef, counts


def _dev_i32(a, device):
    import torch
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=torch.int32).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a, np.int32), device=device)


def _shift_arg(shift, n):
    import torch
    if shift is None:
        return None
    assert shift.dtype == torch.float32 and shift.is_cuda and tuple(shift.shape) == (n, 2)
    return shift.contiguous()


def fit_axial_lrf_grouped(lrfset: LrfSet, cfg: FitCfg, groups, signals, rec, shift=None,
                          stream=None):
    """One axial table per sensor group (Sec. 6.2).  `groups`: the group of
    each sensor ([n_sensors], 0..G-1; -1 leaves a sensor out); `shift`
    ([n][2] float32, GPU, or None) is added to the reconstructed positions
    (Sec. 8).  Returns (coefficients [G][nb+2] float64, counts [G][2] int64
    = events, pairs), device tensors (asynchronous)."""
    import torch
    assert signals.dtype == torch.float32 and signals.is_cuda and signals.dim() == 2
    assert signals.stride(1) == 1 and signals.shape[1] == lrfset.n_sensors
    n = signals.shape[0]
    g = _dev_i32(groups, signals.device)
    assert g.numel() == lrfset.n_sensors
    G = int(g.max().item()) + 1
    assert G >= 1
    sh = _shift_arg(shift, n)
    coef = torch.empty((G, cfg.nb + 2), dtype=torch.float64, device=signals.device)
    counts = torch.empty((G, 2), dtype=torch.int64, device=signals.device)
    _check(_lib.ants_fit_axial_lrf_grouped(
        lrfset.handle, C.byref(cfg), G, g.data_ptr(), n, signals.data_ptr(), signals.stride(0),
        _out_struct(rec), sh.data_ptr() if sh is not None else None, coef.data_ptr(),
        counts.data_ptr(), _stream_handle(stream)))
    return coef, counts


def fit2d_cfg(kind, nb, lo, hi, ridge=1e-9, chi2ndf_max=0.0, base=None,
              z_window=None) -> Fit2dCfg:
    """Fit2dCfg for an r-z (kind 3) or XY (kind 2) LRF fit.  base =
    (coefficients [nb_b + 2] float64 on the GPU, nb_b, lo_b, hi_b): the axial
    part of a composite LRF, subtracted from every estimate (XY residual
    fits); the config keeps a reference to the tensor.  z_window = (a, b):
    only events with a <= z < b (one plane of a sliced LRF)."""
    c = Fit2dCfg()
    c.kind = int(kind)
    for a in range(2):
        c.nb[a], c.lo[a], c.hi[a] = int(nb[a]), float(lo[a]), float(hi[a])
    c.ridge, c.chi2ndf_max = float(ridge), float(chi2ndf_max)
    if base is not None:
        t, bnb, blo, bhi = base
        assert t.is_cuda and t.dtype.is_floating_point and t.numel() == int(bnb) + 2
        t = t.to(dtype=__import__("torch").float64).contiguous()
        c._base = t
        c.d_base, c.base_nb, c.base_lo, c.base_hi = t.data_ptr(), int(bnb), float(blo), float(bhi)
    if z_window is not None:
        c.ev_z_lo, c.ev_z_hi = float(z_window[0]), float(z_window[1])
    return c


def fit_lrf2d_grouped(lrfset: LrfSet, cfg: Fit2dCfg, groups, signals, rec, shift=None,
                      stream=None):
    """One 2-D (r-z or XY) table per sensor group.  Returns (coefficients
    [G][nb1+2][nb0+2] float64, counts [G][2] int64), device tensors
    (asynchronous)."""
    import torch
    assert signals.dtype == torch.float32 and signals.is_cuda and signals.dim() == 2
    assert signals.stride(1) == 1 and signals.shape[1] == lrfset.n_sensors
    n = signals.shape[0]
    g = _dev_i32(groups, signals.device)
    assert g.numel() == lrfset.n_sensors
    G = int(g.max().item()) + 1
    assert G >= 1
    sh = _shift_arg(shift, n)
    coef = torch.empty((G, cfg.nb[1] + 2, cfg.nb[0] + 2), dtype=torch.float64,
                       device=signals.device)
    counts = torch.empty((G, 2), dtype=torch.int64, device=signals.device)
    _check(_lib.ants_fit_lrf2d_grouped(
        lrfset.handle, C.byref(cfg), G, g.data_ptr(), n, signals.data_ptr(), signals.stride(0),
        _out_struct(rec), sh.data_ptr() if sh is not None else None, coef.data_ptr(),
        counts.data_ptr(), _stream_handle(stream)))
    return coef, counts


def fit_composite(lrfset: LrfSet, nb, lo, hi, xy_nb, xy_lo, xy_hi, xy_groups, signals, rec,
                  shift=None, ridge=1e-9, chi2ndf_max=0.0, stream=None):
    """Composite LRF fit (Sec. 6.1.1) in two stages: the shared axial table
    (nb, lo, hi), then one XY residual table per group of xy_groups fitted to
    the estimates minus that axial spline.  Returns (axial [nb + 2], residuals
    [G][xy_nb1 + 2][xy_nb0 + 2], residual counts [G][2]), device tensors
    (asynchronous).  A shift, when given, applies to both stages."""
    ax, _ = fit_axial_lrf_grouped(lrfset, fit_cfg(nb, lo, hi, ridge, chi2ndf_max),
                                  groups_all(lrfset.n_sensors), signals, rec, shift, stream)
    ax = ax[0]
    cfg = fit2d_cfg(LRF_XY, xy_nb, xy_lo, xy_hi, ridge, chi2ndf_max, base=(ax, nb, lo, hi))
    res, counts = fit_lrf2d_grouped(lrfset, cfg, xy_groups, signals, rec, shift, stream)
    return ax, res, counts


def slice_windows(n_planes, z_lo, z_hi):
    """Depth window [a, b) of each plane of a sliced LRF: the events nearest
    that plane (cuts halfway between planes; the outer windows open)."""
    d = (z_hi - z_lo) / (n_planes - 1)
    cuts = [z_lo + (p + 0.5) * d for p in range(n_planes - 1)]
    return list(zip([-math.inf] + cuts, cuts + [math.inf]))


def fit_sliced(lrfset: LrfSet, nb, lo, hi, n_planes, z_lo, z_hi, groups, signals, rec,
               shift=None, ridge=1e-9, chi2ndf_max=0.0, stream=None):
    """Sliced LRF fit (Sec. 6.1.2): each plane's XY tables, one per group,
    fitted to the events nearest that plane.  Returns (tables [G][n_planes]
    [nb1 + 2][nb0 + 2], counts [n_planes][G][2]), device tensors
    (asynchronous)."""
    import torch
    tabs, counts = [], []
    for w in slice_windows(n_planes, z_lo, z_hi):
        cfg = fit2d_cfg(LRF_XY, nb, lo, hi, ridge, chi2ndf_max, z_window=w)
        c, k = fit_lrf2d_grouped(lrfset, cfg, groups, signals, rec, shift, stream)
        tabs.append(c)
        counts.append(k)
    return torch.stack(tabs, 1), torch.stack(counts)


def fit_axial_gains(lrfset: LrfSet, cfg: FitCfg, tables, table_of, signals, rec, shift=None,
                    stream=None):
    """Relative gains re-calculated within fixed groups (Sec. 6.3): `tables`
    [T][nb+2] float64 (the groups' LRFs), `table_of` [n_sensors] (the table
    of each sensor, -1: none).  Returns (gains [n_sensors] float64, NaN
    where not fitted; pairs [n_sensors] int64, 0 where not fitted)."""
    import torch
    assert signals.dtype == torch.float32 and signals.is_cuda and signals.dim() == 2
    assert signals.stride(1) == 1 and signals.shape[1] == lrfset.n_sensors
    n = signals.shape[0]
    t = torch.as_tensor(np.ascontiguousarray(tables, np.float64), device=signals.device) \
        if not isinstance(tables, torch.Tensor) else tables.to(signals.device, torch.float64)
    t = t.reshape(-1, cfg.nb + 2).contiguous()
    tof = _dev_i32(table_of, signals.device)
    assert tof.numel() == lrfset.n_sensors
    sh = _shift_arg(shift, n)
    gains = torch.full((lrfset.n_sensors,), float("nan"), dtype=torch.float64,
                       device=signals.device)
    pairs = torch.zeros(lrfset.n_sensors, dtype=torch.int64, device=signals.device)
    _check(_lib.ants_fit_axial_gains(
        lrfset.handle, C.byref(cfg), t.shape[0], t.data_ptr(), tof.data_ptr(), n,
        signals.data_ptr(), signals.stride(0), _out_struct(rec),
        sh.data_ptr() if sh is not None else None, gains.data_ptr(), pairs.data_ptr(),
        _stream_handle(stream)))
    return gains, pairs


# ---- sensor grouping options (Sec. 6.2), host side
def groups_all(n_sensors):
    """One group for all sensors."""
    return np.zeros(n_sensors, np.int32)


def groups_individual(n_sensors):
    """Every sensor its own group (grouping disabled)."""
    return np.arange(n_sensors, dtype=np.int32)


def groups_by_distance(sxy, tol=1e-3):
    """Groups of sensors at the same distance (within tol mm) from the
    array centre (the mean sensor position), numbered outwards."""
    sxy = np.asarray(sxy, np.float64)
    d = np.hypot(*(sxy - sxy.mean(0)).T)
    order = np.argsort(d, kind="stable")
    g = np.empty(len(d), np.int32)
    k, last = -1, None
    for i in order:
        if last is None or d[i] - last > tol:
            k += 1
            last = d[i]
        g[i] = k
    return g


def groups_by_symmetry(sxy, order, reflect=True, tol=1e-3):
    """Orbits of the sensors under rotations by 2 pi / order about the array
    centre (and the reflection x -> -x when `reflect`): order 6 for
    hexagonal, 4 for square, 2 for rectangular arrays.  Groups are numbered
    by the orbit's smallest sensor index."""
    sxy = np.asarray(sxy, np.float64)
    c = sxy - sxy.mean(0)
    n = len(c)
    maps = []
    for k in range(order):
        a = 2.0 * np.pi * k / order
        R = np.array([[np.cos(a), -np.sin(a)], [np.sin(a), np.cos(a)]])
        maps.append(R)
        if reflect:
            maps.append(R @ np.diag([-1.0, 1.0]))
    g = np.full(n, -1, np.int32)
    k = 0
    for i in range(n):
        if g[i] >= 0:
            continue
        for M in maps:
            p = M @ c[i]
            j = np.where(np.hypot(*(c - p).T) <= tol)[0]
            for jj in j:
                if g[jj] < 0:
                    g[jj] = k
        g[i] = k
        k += 1
    return g


class AxialModel:
    """Detector model with axial LRFs: `tables` [T][nb+2] and the table of
    each sensor (`table_of`, default: one shared table); the fields LrfSet
    reads (per-sensor rows when there are several tables)."""

    def __init__(self, sxy, gain, active, nb, lo, hi, coef, table_of=None):
        self.kind = 1
        self.sxy = np.ascontiguousarray(sxy, np.float64)
        self.gain = np.ascontiguousarray(gain, np.float64)
        self.active = np.ascontiguousarray(active, np.uint8)
        self.nb, self.lo, self.hi = (int(nb), 1), (float(lo), 0.0), (float(hi), 0.0)
        self.tables = np.ascontiguousarray(coef, np.float64).reshape(-1, int(nb) + 2)
        n = len(self.sxy)
        self.table_of = (np.zeros(n, np.int32) if table_of is None
                         else np.ascontiguousarray(table_of, np.int32))
        if len(self.tables) == 1 and (self.table_of == 0).all():
            self.shared = 1
            self.coef = self.tables.reshape(1, 1, -1)
        else:
            self.shared = 0
            self.coef = self.tables[np.maximum(self.table_of, 0)].reshape(n, 1, -1)

    def with_active(self, active):
        return AxialModel(self.sxy, self.gain, active, self.nb[0], self.lo[0], self.hi[0],
                          self.tables, self.table_of)


class Lrf2dModel:
    """Detector model with 2-D LRFs (kind 3 r-z or 2 XY): `tables`
    [T][nb1+2][nb0+2] and the table of each sensor (`table_of`, default one
    shared table); the fields LrfSet reads."""

    def __init__(self, kind, sxy, gain, active, nb, lo, hi, tables, table_of=None):
        self.kind = int(kind)
        self.sxy = np.ascontiguousarray(sxy, np.float64)
        self.gain = np.ascontiguousarray(gain, np.float64)
        self.active = np.ascontiguousarray(active, np.uint8)
        self.nb = (int(nb[0]), int(nb[1]))
        self.lo, self.hi = (float(lo[0]), float(lo[1])), (float(hi[0]), float(hi[1]))
        self.tables = np.ascontiguousarray(tables, np.float64).reshape(
            -1, self.nb[1] + 2, self.nb[0] + 2)
        n = len(self.sxy)
        self.table_of = (np.zeros(n, np.int32) if table_of is None
                         else np.ascontiguousarray(table_of, np.int32))
        if len(self.tables) == 1 and (self.table_of == 0).all():
            self.shared = 1
            self.coef = self.tables
        else:
            self.shared = 0
            self.coef = self.tables[np.maximum(self.table_of, 0)]

    def with_active(self, active):
        return Lrf2dModel(self.kind, self.sxy, self.gain, active, self.nb, self.lo, self.hi,
                          self.tables, self.table_of)


class CompositeModel:
    """Detector model with a composite LRF (Sec. 6.1.1): the shared axial
    table `axial` [nb + 2] on [lo, hi] plus XY residual tables `xy_tables`
    [T][xy_nb1 + 2][xy_nb0 + 2] (`xy_table_of`: the table of each sensor,
    default one shared table); the fields LrfSet reads."""

    def __init__(self, sxy, gain, active, nb, lo, hi, axial, xy_nb, xy_lo, xy_hi, xy_tables,
                 xy_table_of=None):
        self.kind = LRF_COMPOSITE
        self.shared = 1
        self.sxy = np.ascontiguousarray(sxy, np.float64)
        self.gain = np.ascontiguousarray(gain, np.float64)
        self.active = np.ascontiguousarray(active, np.uint8)
        self.nb, self.lo, self.hi = (int(nb), 1), (float(lo), 0.0), (float(hi), 0.0)
        self.axial = np.ascontiguousarray(axial, np.float64).reshape(-1)
        self.coef = self.axial.reshape(1, 1, -1)
        self.xy_nb = (int(xy_nb[0]), int(xy_nb[1]))
        self.xy_lo = (float(xy_lo[0]), float(xy_lo[1]))
        self.xy_hi = (float(xy_hi[0]), float(xy_hi[1]))
        self.xy_tables = np.ascontiguousarray(xy_tables, np.float64).reshape(
            -1, self.xy_nb[1] + 2, self.xy_nb[0] + 2)
        n = len(self.sxy)
        self.xy_table_of = (np.zeros(n, np.int32) if xy_table_of is None
                            else np.ascontiguousarray(xy_table_of, np.int32))
        if len(self.xy_tables) == 1 and (self.xy_table_of == 0).all():
            self.xy_shared = 1
            self.xy_coef = self.xy_tables
        else:
            self.xy_shared = 0
            self.xy_coef = self.xy_tables[np.maximum(self.xy_table_of, 0)]

    def with_active(self, active):
        return CompositeModel(self.sxy, self.gain, active, self.nb[0], self.lo[0], self.hi[0],
                              self.axial, self.xy_nb, self.xy_lo, self.xy_hi, self.xy_tables,
                              self.xy_table_of)


def iterate_composite(model, grid: GridCfg, signals, iterations, xy_groups=None, ridge=1e-9,
                      chi2ndf_max=0.0, stream=None, shift_sigma=0.0, shift_iterations=0,
                      shift_seed=0, disable=None):
    """Iterative LRF reconstruction (Sec. 8) for composite models: each fit
    is the two-stage composite fit (the shared axial table, then the XY
    residuals per group of xy_groups: None for one residual per sensor, an
    array, or a function of the fit index).  Shifts and disabled sensors as
    in iterate_axial_lrf; a residual group whose fit fails keeps its
    previous tables, and a failed axial fit keeps the model.  Returns the
    models and the last reconstruction."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    models = [model]
    n = signals.shape[0]
    for k in range(iterations + 1):
        cur = models[-1]
        act = np.asarray(cur.active, np.uint8).copy()
        if disable and k in disable:
            act[np.asarray(disable[k], np.int64)] = 0
        ls = LrfSet(cur.with_active(act))
        rec = reconstruct(ls, grid, signals, stream=st)
        if k == iterations:
            st.synchronize()
            ls.close()
            break
        fs = LrfSet(cur) if disable and k in disable else ls
        ns = len(cur.sxy)
        g = xy_groups(k) if callable(xy_groups) else xy_groups
        g = groups_individual(ns) if g is None else np.asarray(g, np.int32)
        shift = None
        if shift_sigma > 0.0 and k < shift_iterations:
            gen = torch.Generator(device=signals.device).manual_seed(int(shift_seed) + k)
            shift = torch.randn((n, 2), generator=gen, device=signals.device,
                                dtype=torch.float32) * float(shift_sigma)
        ax, res, _ = fit_composite(fs, cur.nb[0], cur.lo[0], cur.hi[0], cur.xy_nb, cur.xy_lo,
                                   cur.xy_hi, g, signals, rec, shift, ridge, chi2ndf_max, st)
        st.synchronize()
        ax, res = ax.cpu().numpy(), res.cpu().numpy()
        if fs is not ls:
            fs.close()
        ls.close()
        if not np.isfinite(ax).all():
            models.append(cur)
            continue
        new = cur.xy_tables[np.maximum(cur.xy_table_of, 0)].copy()
        for i in range(ns):
            if 0 <= g[i] < len(res) and np.isfinite(res[g[i]]).all():
                new[i] = res[g[i]]
        if (g == 0).all() and np.isfinite(res[0]).all():
            nxt = CompositeModel(cur.sxy, cur.gain, cur.active, cur.nb[0], cur.lo[0], cur.hi[0],
                                 ax, cur.xy_nb, cur.xy_lo, cur.xy_hi, res[0])
        else:
            nxt = CompositeModel(cur.sxy, cur.gain, cur.active, cur.nb[0], cur.lo[0], cur.hi[0],
                                 ax, cur.xy_nb, cur.xy_lo, cur.xy_hi, new, np.arange(ns))
        models.append(nxt)
    return models, rec


class SlicedModel:
    """Detector model with a sliced LRF (Sec. 6.1.2): XY tables on n_planes
    z planes between z_lo and z_hi, `tables` [T][n_planes][nb1 + 2][nb0 + 2]
    (`table_of`: the table of each sensor, default one per sensor); the
    fields LrfSet reads."""

    def __init__(self, sxy, gain, active, nb, lo, hi, n_planes, z_lo, z_hi, tables,
                 table_of=None):
        self.kind = LRF_SLICED
        self.sxy = np.ascontiguousarray(sxy, np.float64)
        self.gain = np.ascontiguousarray(gain, np.float64)
        self.active = np.ascontiguousarray(active, np.uint8)
        self.nb = (int(nb[0]), int(nb[1]))
        self.lo, self.hi = (float(lo[0]), float(lo[1])), (float(hi[0]), float(hi[1]))
        self.n_planes, self.z_lo, self.z_hi = int(n_planes), float(z_lo), float(z_hi)
        self.tables = np.ascontiguousarray(tables, np.float64).reshape(
            -1, self.n_planes, self.nb[1] + 2, self.nb[0] + 2)
        n = len(self.sxy)
        self.table_of = (np.arange(n, dtype=np.int32) if table_of is None
                         else np.ascontiguousarray(table_of, np.int32))
        if len(self.tables) == 1 and (self.table_of == 0).all():
            self.shared = 1
            self.coef = self.tables
        else:
            self.shared = 0
            self.coef = self.tables[np.maximum(self.table_of, 0)]

    def with_active(self, active):
        return SlicedModel(self.sxy, self.gain, active, self.nb, self.lo, self.hi, self.n_planes,
                           self.z_lo, self.z_hi, self.tables, self.table_of)


def iterate_sliced(model, grid: GridCfg, signals, iterations, groups=None, ridge=1e-9,
                   chi2ndf_max=0.0, stream=None, shift_sigma=0.0, shift_iterations=0,
                   shift_seed=0, disable=None):
    """Iterative LRF reconstruction (Sec. 8) for sliced models: each fit
    refits every plane's XY tables per group (groups: None for one table per
    sensor, an array, or a function of the fit index) from the events
    nearest the plane.  Shifts and disabled sensors as in iterate_axial_lrf;
    a group or plane whose fit fails keeps its previous tables.  Returns the
    models and the last reconstruction."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    models = [model]
    n = signals.shape[0]
    for k in range(iterations + 1):
        cur = models[-1]
        act = np.asarray(cur.active, np.uint8).copy()
        if disable and k in disable:
            act[np.asarray(disable[k], np.int64)] = 0
        ls = LrfSet(cur.with_active(act))
        rec = reconstruct(ls, grid, signals, stream=st)
        if k == iterations:
            st.synchronize()
            ls.close()
            break
        fs = LrfSet(cur) if disable and k in disable else ls
        ns = len(cur.sxy)
        g = groups(k) if callable(groups) else groups
        g = groups_individual(ns) if g is None else np.asarray(g, np.int32)
        shift = None
        if shift_sigma > 0.0 and k < shift_iterations:
            gen = torch.Generator(device=signals.device).manual_seed(int(shift_seed) + k)
            shift = torch.randn((n, 2), generator=gen, device=signals.device,
                                dtype=torch.float32) * float(shift_sigma)
        tabs, _ = fit_sliced(fs, cur.nb, cur.lo, cur.hi, cur.n_planes, cur.z_lo, cur.z_hi, g,
                             signals, rec, shift, ridge, chi2ndf_max, st)
        st.synchronize()
        tabs = tabs.cpu().numpy()
        if fs is not ls:
            fs.close()
        ls.close()
        new = cur.tables[np.maximum(cur.table_of, 0)].copy()
        for i in range(ns):
            if 0 <= g[i] < len(tabs):
                for p in range(cur.n_planes):
                    if np.isfinite(tabs[g[i], p]).all():
                        new[i, p] = tabs[g[i], p]
        models.append(SlicedModel(cur.sxy, cur.gain, cur.active, cur.nb, cur.lo, cur.hi,
                                  cur.n_planes, cur.z_lo, cur.z_hi, new, np.arange(ns)))
    return models, rec


def _check_rz_groups(kind, g):
    if kind == LRF_RZ and g is not None and not (np.asarray(g) == 0).all():
        raise ValueError("r-z LRF sets share one table: fit them with one group")


def iterate_lrf2d(model, grid: GridCfg, signals, iterations, ridge=1e-9, chi2ndf_max=0.0,
                  stream=None, groups=None, shift_sigma=0.0, shift_iterations=0, shift_seed=0,
                  disable=None):
    """Iterative LRF reconstruction (Sec. 8) for r-z or XY models: as
    iterate_axial_lrf, with the 2-D fits (groups: None for one shared table,
    an array, or a function of the fit index).  r-z sets hold one table
    shared by every sensor, so r-z models take only the shared fit.  A group
    whose fit fails (no pairs) keeps its previous tables.  Returns the models
    and the last reconstruction."""
    import torch
    if not callable(groups):
        _check_rz_groups(model.kind, groups)
    st = stream if stream is not None else torch.cuda.current_stream()
    models = [model]
    n = signals.shape[0]
    for k in range(iterations + 1):
        cur = models[-1]
        act = np.asarray(cur.active, np.uint8).copy()
        if disable and k in disable:
            act[np.asarray(disable[k], np.int64)] = 0
        ls = LrfSet(cur.with_active(act))
        rec = reconstruct(ls, grid, signals, stream=st)
        if k == iterations:
            st.synchronize()
            ls.close()
            break
        fs = LrfSet(cur) if disable and k in disable else ls
        g = groups(k) if callable(groups) else groups
        ns = len(cur.sxy)
        g = groups_all(ns) if g is None else np.asarray(g, np.int32)
        _check_rz_groups(cur.kind, g)
        shift = None
        if shift_sigma > 0.0 and k < shift_iterations:
            gen = torch.Generator(device=signals.device).manual_seed(int(shift_seed) + k)
            shift = torch.randn((n, 2), generator=gen, device=signals.device,
                                dtype=torch.float32) * float(shift_sigma)
        cfg = fit2d_cfg(cur.kind, cur.nb, cur.lo, cur.hi, ridge, chi2ndf_max)
        coef, _ = fit_lrf2d_grouped(fs, cfg, g, signals, rec, shift, st)
        st.synchronize()
        coef = coef.cpu().numpy()
        new = cur.tables[np.maximum(cur.table_of, 0)].copy()
        for i in range(ns):
            if 0 <= g[i] < len(coef) and np.isfinite(coef[g[i]]).all():
                new[i] = coef[g[i]]
        if fs is not ls:
            fs.close()
        ls.close()
        if (g == 0).all():
            nxt = (Lrf2dModel(cur.kind, cur.sxy, cur.gain, cur.active, cur.nb, cur.lo, cur.hi,
                              coef[0]) if np.isfinite(coef[0]).all() else cur)
        else:
            nxt = Lrf2dModel(cur.kind, cur.sxy, cur.gain, cur.active, cur.nb, cur.lo, cur.hi,
                             new, np.arange(ns))
        models.append(nxt)
    return models, rec


def iterate_axial_lrf(model, grid: GridCfg, signals, iterations, ridge=1e-9, chi2ndf_max=0.0,
                      stream=None, groups=None, shift_sigma=0.0, shift_iterations=0,
                      shift_seed=0, disable=None, refit_gains=False):
    """Iterative LRF reconstruction (Sec. 8): reconstruct every event with the
    current LRFs, keep the events that pass the filter, fit the LRFs to their
    signals, reconstructed positions and energies, repeat.  `model` is the
    initial guess (an AxialModel).

    groups: None (one shared table), a per-sensor group array, or a function
      k -> group array for fit k (e.g. one common LRF for the first fits,
      then individual ones: Sec. 8);
    shift_sigma, shift_iterations, shift_seed: the first shift_iterations
      fits read the positions shifted by N(0, shift_sigma^2) per axis (drawn
      with torch's generator from shift_seed + k);
    disable: {k: [sensor indices]} sensors left out of the reconstruction of
      iteration k (their LRFs are still fitted; Sec. 8);
    refit_gains: after each fit, re-calculate the relative gains within the
      new groups (Sec. 6.3).
    Sensors of a group without pairs keep their previous LRF.  Returns the
    list of models, the initial one first, and the last reconstruction."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    models = [model]
    n = signals.shape[0]
    for k in range(iterations + 1):
        cur = models[-1]
        act = np.asarray(cur.active, np.uint8).copy()
        if disable and k in disable:
            act[np.asarray(disable[k], np.int64)] = 0
        ls = LrfSet(cur.with_active(act))
        rec = reconstruct(ls, grid, signals, stream=st)
        if k == iterations:
            st.synchronize()
            ls.close()
            break
        fs = LrfSet(cur) if disable and k in disable else ls
        g = groups(k) if callable(groups) else groups
        g = groups_all(len(cur.sxy)) if g is None else np.asarray(g, np.int32)
        shift = None
        if shift_sigma > 0.0 and k < shift_iterations:
            gen = torch.Generator(device=signals.device).manual_seed(int(shift_seed) + k)
            shift = torch.randn((n, 2), generator=gen, device=signals.device,
                                dtype=torch.float32) * float(shift_sigma)
        cfg = fit_cfg(cur.nb[0], cur.lo[0], cur.hi[0], ridge, chi2ndf_max)
        coef, counts = fit_axial_lrf_grouped(fs, cfg, g, signals, rec, shift, st)
        gains = None
        if refit_gains:
            gains, _ = fit_axial_gains(fs, cfg, coef, g, signals, rec, shift, st)
        st.synchronize()
        coef = coef.cpu().numpy()
        # groups without a solution keep the previous tables of their sensors
        ns = len(cur.sxy)
        new = cur.tables[np.maximum(cur.table_of, 0)].copy()
        for i in range(ns):
            if 0 <= g[i] < len(coef) and np.isfinite(coef[g[i]]).all():
                new[i] = coef[g[i]]
        gain = cur.gain.copy()
        if gains is not None:
            gh = gains.cpu().numpy()
            ok = np.isfinite(gh)
            gain[ok] = gh[ok]
        if fs is not ls:
            fs.close()
        ls.close()
        if (g == 0).all() and np.isfinite(coef[0]).all():
            nxt = AxialModel(cur.sxy, gain, cur.active, cur.nb[0], cur.lo[0], cur.hi[0], coef[0])
        else:
            nxt = AxialModel(cur.sxy, gain, cur.active, cur.nb[0], cur.lo[0], cur.hi[0], new,
                             np.arange(ns))
        models.append(nxt)
    return models, rec


