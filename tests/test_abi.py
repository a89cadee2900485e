"""C ABI checks that need no GPU: every function declared in include/ants.h
is exported by the library, and argument errors are reported with the
documented codes before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(ants_[a-z0-9_]+)\s*\(", txt))
    return names


@pytest.fixture(scope="module")
def ants():
    from paper_1602_07247_amd import ants as A
    return A


def test_every_declared_symbol_is_exported(ants):
    lib = C.CDLL(ants.LIB_PATH)
    declared = _declared()
    assert declared, "no declarations found"
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(ants.EXPORTED) <= declared


def test_version_string(ants):
    assert "gfx950" in ants.version()


def _desc(ants, model, **over):
    d = ants.LrfDesc()
    keep = []
    sxy = np.ascontiguousarray(model.sxy, np.float64)
    coef = np.ascontiguousarray(model.coef, np.float64)
    keep += [sxy, coef]
    d.n_sensors = sxy.shape[0]
    d.sensor_xy = sxy.ctypes.data_as(C.POINTER(C.c_double))
    d.gain = None
    d.active = None
    d.kind = model.kind
    d.shared = model.shared
    d.n_knots[0], d.n_knots[1] = model.nb
    d.lo[0], d.lo[1] = model.lo
    d.hi[0], d.hi[1] = model.hi
    d.coef = coef.ctypes.data_as(C.POINTER(C.c_double))
    for k, v in over.items():
        if k in ("lo", "hi", "n_knots"):
            getattr(d, k)[0] = v
        else:
            setattr(d, k, v)
    return d, keep


@pytest.mark.parametrize("over,code", [
    ({"n_sensors": 0}, -1), ({"n_sensors": 1000}, -1), ({"kind": 9}, -1),
    ({"n_knots": 1}, -1), ({"lo": 5.0}, -5), ({"hi": -1.0}, -2)])
def test_descriptor_errors(ants, over, code):
    d, keep = _desc(ants, W.axial_lrf(W.hex_array(2, 30.0)), **over)
    h = C.c_void_p()
    assert ants._lib.ants_lrfset_create(C.byref(d), C.byref(h)) == code
    assert not h.value
    assert ants._lib.ants_last_error()


def test_non_finite_coefficient_and_rz_per_sensor(ants):
    m = W.rz_lrf(W.hex_array(1, 30.0))
    m.coef = m.coef.copy()
    m.coef[0, 3, 3] = np.nan
    d, keep = _desc(ants, m)
    h = C.c_void_p()
    assert ants._lib.ants_lrfset_create(C.byref(d), C.byref(h)) == ants.E_FORMAT
    m = W.rz_lrf(W.hex_array(1, 30.0))
    d, keep = _desc(ants, m, shared=0)
    assert ants._lib.ants_lrfset_create(C.byref(d), C.byref(h)) == ants.E_UNSUPPORTED


def test_reconstruct_argument_errors(ants):
    cfg = ants.grid_cfg(W.workload(0).grid)
    out = ants.Out()
    assert ants._lib.ants_reconstruct(None, C.byref(cfg), 10, None, None, out, None) == ants.E_ARG
    assert ants._lib.ants_lrfset_create(None, C.byref(C.c_void_p())) == ants.E_ARG
    assert ants._lib.ants_lrfset_destroy(None) == ants.OK


def test_fit_argument_errors(ants):
    cfg = ants.fit_cfg(20, 0.0, 150.0)
    out = ants.Out()
    coef = C.c_void_p(1)
    assert ants._lib.ants_fit_axial_lrf(None, C.byref(cfg), 0, None, 0, out, coef, None,
                                        None) == ants.E_ARG
    assert ants._lib.ants_fit_axial_lrf(None, None, 0, None, 0, out, coef, None,
                                        None) == ants.E_ARG


# ------------------------------------------------------------ LRF-set files


def _parse_lrf_file(raw):
    # the layout documented in include/ants.h, read independently here
    import struct
    assert raw[:8] == b"ANTSLRF1"
    ns, kind, shared, nb0, nb1, _ = struct.unpack_from("<6i", raw, 8)
    lo0, lo1, hi0, hi1 = struct.unpack_from("<4d", raw, 32)
    (ncoef,) = struct.unpack_from("<q", raw, 64)
    o = 72
    xy = np.frombuffer(raw, "<f8", 2 * ns, o).reshape(ns, 2)
    o += 16 * ns
    gain = np.frombuffer(raw, "<f8", ns, o)
    o += 8 * ns
    active = np.frombuffer(raw, np.uint8, ns, o)
    o += (ns + 7) // 8 * 8
    coef = np.frombuffer(raw, "<f8", ncoef, o)
    o += 8 * ncoef
    (h,) = struct.unpack_from("<Q", raw, o)
    fnv = 1469598103934665603
    for b in raw[:o]:
        fnv = ((fnv ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    assert h == fnv and o + 8 == len(raw)
    return dict(ns=ns, kind=kind, shared=shared, nb=(nb0, nb1), lo=(lo0, lo1), hi=(hi0, hi1),
                xy=xy, gain=gain, active=active, coef=coef)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_lrf_file_layout(ants, k, tmp_path):
    m = W.workload(k).lrf
    m.active = np.ones(m.sxy.shape[0], np.uint8)
    m.active[1] = 0
    f = tmp_path / "set.lrf"
    ants.write_lrf(m, str(f))
    got = _parse_lrf_file(f.read_bytes())
    assert got["ns"] == m.sxy.shape[0] and got["kind"] == m.kind and got["shared"] == m.shared
    assert got["nb"][0] == m.nb[0] and got["nb"][1] == (0 if m.kind == 1 else m.nb[1])
    np.testing.assert_array_equal(got["xy"], m.sxy)
    np.testing.assert_array_equal(got["gain"], m.gain)
    np.testing.assert_array_equal(got["active"], m.active)
    np.testing.assert_array_equal(got["coef"], np.asarray(m.coef).reshape(-1))


def _load_code(ants, path):
    h = C.c_void_p()
    code = ants._lib.ants_lrfset_load(os.fsencode(str(path)), C.byref(h))
    assert not h.value or code == ants.OK
    return code


def test_lrf_file_errors(ants, tmp_path):
    m = W.workload(0).lrf
    f = tmp_path / "set.lrf"
    ants.write_lrf(m, str(f))
    raw = f.read_bytes()
    bad = tmp_path / "bad.lrf"
    cases = {
        "truncated": raw[:-1],
        "extended": raw + b"\0",
        "header only": raw[:72],
        "empty": b"",
        "foreign": b"ANTSMLP1" + raw[8:],
        "flipped coefficient": raw[:-20] + bytes([raw[-20] ^ 1]) + raw[-19:],
    }
    for name, data in cases.items():
        bad.write_bytes(data)
        assert _load_code(ants, bad) == ants.E_FORMAT, name
        assert ants._lib.ants_last_error(), name
    # a header out of range, with a valid checksum
    import struct
    b = bytearray(raw)
    struct.pack_into("<i", b, 12, 7)          # kind 7
    fnv = 1469598103934665603
    for x in b[:-8]:
        fnv = ((fnv ^ x) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    struct.pack_into("<Q", b, len(b) - 8, fnv)
    bad.write_bytes(bytes(b))
    assert _load_code(ants, bad) == ants.E_FORMAT
    assert _load_code(ants, tmp_path / "missing.lrf") == ants.E_ARG
    assert ants._lib.ants_lrf_write(None, b"x") == ants.E_ARG


def test_grouping_helpers():
    # Sec. 6.2 grouping options on the host: one group, individual, by
    # distance from the array centre, by rotation/reflection symmetry
    import workloads as W
    from paper_1602_07247_amd import ants as A
    hex61, _ = W.mixed_geometries()[1]
    sxy = hex61.sxy
    assert (A.groups_all(61) == 0).all()
    assert (A.groups_individual(61) == np.arange(61)).all()
    ring = A.groups_by_distance(sxy)
    d = np.hypot(*(sxy - sxy.mean(0)).T)
    for k in range(ring.max() + 1):
        assert np.ptp(d[ring == k]) < 1e-6
    assert np.all(np.diff([d[ring == k].mean() for k in range(ring.max() + 1)]) > 0)
    sym = A.groups_by_symmetry(sxy, 6)
    # orbits of the hexagonal group: sizes 1, 6 or 12; each within one ring
    sizes = np.bincount(sym)
    assert set(sizes.tolist()) <= {1, 6, 12} and sizes.sum() == 61
    for k in range(sym.max() + 1):
        assert len(set(ring[sym == k].tolist())) == 1
    sq = W.square_array(8, 6.0)
    s4 = A.groups_by_symmetry(sq, 4)
    assert s4.max() + 1 == 10 and sorted(np.bincount(s4).tolist()) == [4] * 4 + [8] * 6


def test_rz_loop_takes_one_group():
    # r-z sets share one table, so the r-z reconstruct-refit loop refuses a
    # grouping before any GPU work
    import workloads as W
    from paper_1602_07247_amd import ants as A
    lrf = W.workload(2).lrf
    m = A.Lrf2dModel(lrf.kind, lrf.sxy, lrf.gain, lrf.active, lrf.nb, lrf.lo, lrf.hi,
                     np.asarray(lrf.coef)[0])
    with pytest.raises(ValueError):
        A.iterate_lrf2d(m, None, None, 1, groups=np.arange(len(lrf.sxy), dtype=np.int32))
    assert m.shared == 1 and m.coef.shape == (1, lrf.nb[1] + 2, lrf.nb[0] + 2)
