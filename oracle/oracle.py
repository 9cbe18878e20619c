"""ctypes binding of the CPU oracle (test infrastructure only).

Same entry points as the GPU library, on host numpy arrays. Builds the shared
library on first use when it is missing.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

OK, ERR_ARG, ERR_NONFINITE, ERR_BUFFER, ERR_CORRUPT = 0, -1, -2, -3, -4
EB_ABS, EB_REL = 0, 1
CODING_DEFAULT, CODING_HUFFMAN, CODING_ZERO_CHUNKS = 0, 1, 2


class Config(C.Structure):
    _fields_ = [("block", C.c_uint32), ("levels", C.c_uint32), ("radius", C.c_uint32),
                ("coding", C.c_uint32), ("eb_ratio", C.c_double)]


class Info(C.Structure):
    _fields_ = [("dims", C.c_uint64 * 3), ("block", C.c_uint32), ("levels", C.c_uint32),
                ("radius", C.c_uint32), ("lmax", C.c_uint32), ("eb_mode", C.c_uint32),
                ("dtype", C.c_uint32), ("eb", C.c_double), ("eb_abs", C.c_double),
                ("eb_ratio", C.c_double), ("total_bytes", C.c_uint64),
                ("coding", C.c_uint32), ("reserved", C.c_uint32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        override = os.environ.get("STZ_ORACLE_LIB")  # a mutated copy, for pin checks
        if override:
            _build.LIB = override
        elif not os.path.exists(_build.LIB) or (
                os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build()
        L = C.CDLL(_build.LIB)
        u64p = C.POINTER(C.c_uint64)
        for sfx in ("", "_f64"):
            f = getattr(L, "stz_ref_compress_bound" + sfx)
            f.restype = C.c_uint64
            f.argtypes = [u64p, C.POINTER(Config)]
            f = getattr(L, "stz_ref_compress" + sfx)
            f.restype = C.c_int
            f.argtypes = [C.c_void_p, u64p, C.c_int, C.c_double, C.POINTER(Config), C.c_void_p,
                          C.c_uint64, u64p]
            f = getattr(L, "stz_ref_decompress" + sfx)
            f.restype = C.c_int
            f.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64]
            f = getattr(L, "stz_ref_decompress_level" + sfx)
            f.restype = C.c_int
            f.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_void_p, C.c_uint64, u64p]
            f = getattr(L, "stz_ref_decompress_region" + sfx)
            f.restype = C.c_int
            f.argtypes = [C.c_void_p, C.c_uint64, u64p, u64p, C.c_uint32, C.c_void_p,
                          C.c_uint64, u64p]
        L.stz_ref_info.restype = C.c_int
        L.stz_ref_info.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(Info)]
        for f in (L.stz_ref_symbols, L.stz_ref_symbols_f64):
            f.restype = C.c_int
            f.argtypes = [C.c_void_p, u64p, C.c_int, C.c_double, C.POINTER(Config),
                          C.c_void_p, C.c_void_p, C.c_void_p]
        L.stz_ref_predict.restype = C.c_float
        L.stz_ref_predict.argtypes = [C.c_void_p, u64p, u64p, C.c_uint64]
        L.stz_ref_predict_f64.restype = C.c_double
        L.stz_ref_predict_f64.argtypes = [C.c_void_p, u64p, u64p, C.c_uint64]
        L.stz_ref_units_decoded.restype = None
        L.stz_ref_units_decoded.argtypes = [C.c_void_p]
        L.stz_ref_huffman_lengths.restype = None
        L.stz_ref_huffman_lengths.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p]
        L.stz_ref_canonical_codes.restype = None
        L.stz_ref_canonical_codes.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
        L.stz_ref_level_bounds.restype = None
        L.stz_ref_roi_select.restype = C.c_int
        L.stz_ref_roi_select.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint32,
                                         C.c_uint32, C.c_uint32, C.c_double, C.c_void_p,
                                         C.c_uint64, C.POINTER(C.c_uint64), C.c_void_p]
        L.stz_ref_level_bounds.argtypes = [C.c_double, C.c_double, C.c_int, C.c_void_p,
                                           C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def _dims(shape):
    return (C.c_uint64 * 3)(*[int(v) for v in shape])


def config(block=32, levels=0, radius=0, eb_ratio=0.0, coding=CODING_DEFAULT):
    return Config(block, levels, radius, coding, eb_ratio)


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: status {status}")
        self.status = status


def _sfx(dtype):
    dt = np.dtype(dtype)
    if dt == np.float32:
        return ""
    if dt == np.float64:
        return "_f64"
    raise TypeError(f"unsupported value type {dt}")


def compress_bound(shape, cfg, dtype=np.float32):
    return int(getattr(lib(), "stz_ref_compress_bound" + _sfx(dtype))(_dims(shape),
                                                                       C.byref(cfg)))


def compress(x, eb_mode, eb, cfg, dtype=np.float32):
    """Compress a C-contiguous array of shape (nz, ny, nx), converted to `dtype`
    (float32 or float64); returns bytes."""
    x = np.ascontiguousarray(x, dtype=dtype)
    assert x.ndim == 3
    cap = compress_bound(x.shape, cfg, dtype)
    out = np.zeros(cap, dtype=np.uint8)
    size = C.c_uint64(0)
    st = getattr(lib(), "stz_ref_compress" + _sfx(dtype))(
        x.ctypes.data, _dims(x.shape), eb_mode, eb, C.byref(cfg), out.ctypes.data, cap,
        C.byref(size))
    if st != OK:
        raise OracleError(st, "compress")
    return out[: size.value].tobytes()


def compress_status(x, eb_mode, eb, cfg, cap=None, dtype=np.float32):
    x = np.ascontiguousarray(x, dtype=dtype)
    if cap is None:
        cap = max(compress_bound(x.shape, cfg, dtype), 1)
    out = np.zeros(max(cap, 1), dtype=np.uint8)
    size = C.c_uint64(0)
    return getattr(lib(), "stz_ref_compress" + _sfx(dtype))(
        x.ctypes.data, _dims(x.shape), eb_mode, eb, C.byref(cfg), out.ctypes.data, cap,
        C.byref(size))


def value_type(inf):
    """numpy value type of a stream from its info record."""
    return np.float64 if inf.dtype == 1 else np.float32


def info(comp):
    buf = np.frombuffer(comp, dtype=np.uint8)
    inf = Info()
    st = lib().stz_ref_info(buf.ctypes.data, buf.size, C.byref(inf))
    if st != OK:
        raise OracleError(st, "info")
    return inf


def decompress(comp):
    inf = info(comp)
    shape = tuple(int(v) for v in inf.dims)
    vt = value_type(inf)
    out = np.empty(shape, dtype=vt)
    buf = np.frombuffer(comp, dtype=np.uint8)
    st = getattr(lib(), "stz_ref_decompress" + _sfx(vt))(buf.ctypes.data, buf.size,
                                                         out.ctypes.data, out.size)
    if st != OK:
        raise OracleError(st, "decompress")
    return out


def decompress_level(comp, level):
    inf = info(comp)
    s = 1 << (inf.levels - level)
    shape = tuple((int(n) - 1) // s + 1 for n in inf.dims)
    vt = value_type(inf)
    out = np.empty(shape, dtype=vt)
    od = (C.c_uint64 * 3)()
    buf = np.frombuffer(comp, dtype=np.uint8)
    st = getattr(lib(), "stz_ref_decompress_level" + _sfx(vt))(
        buf.ctypes.data, buf.size, level, out.ctypes.data, out.size, od)
    if st != OK:
        raise OracleError(st, "decompress_level")
    assert tuple(od) == shape
    return out


def decompress_region(comp, lo, hi, level):
    inf = info(comp)
    s = 1 << (inf.levels - level)
    shape = []
    for d in range(3):
        first = -(-int(lo[d]) // s) * s
        shape.append((int(hi[d]) - 1 - first) // s + 1 if first < int(hi[d]) else 0)
    shape = tuple(shape)
    vt = value_type(inf)
    out = np.empty(shape, dtype=vt)
    od = (C.c_uint64 * 3)()
    buf = np.frombuffer(comp, dtype=np.uint8)
    st = getattr(lib(), "stz_ref_decompress_region" + _sfx(vt))(
        buf.ctypes.data, buf.size, _dims(lo), _dims(hi), level, out.ctypes.data,
        max(out.size, 0), od)
    if st != OK:
        raise OracleError(st, "decompress_region")
    assert tuple(od) == shape, (tuple(od), shape)
    return out


def decode_status(comp, fn="decompress", level=0, lo=None, hi=None, dtype=np.float32):
    """Status of a decode call (the `dtype` variant) on possibly corrupt bytes
    (never raises)."""
    buf = np.frombuffer(comp, dtype=np.uint8)
    out = np.empty(1 << 22, dtype=dtype)
    od = (C.c_uint64 * 3)()
    L = lib()
    x = _sfx(dtype)
    if fn == "decompress":
        return getattr(L, "stz_ref_decompress" + x)(buf.ctypes.data, buf.size, out.ctypes.data,
                                                    out.size)
    if fn == "level":
        return getattr(L, "stz_ref_decompress_level" + x)(buf.ctypes.data, buf.size, level,
                                                          out.ctypes.data, out.size, od)
    return getattr(L, "stz_ref_decompress_region" + x)(buf.ctypes.data, buf.size, _dims(lo),
                                                       _dims(hi), level, out.ctypes.data,
                                                       out.size, od)


def symbols(x, eb_mode, eb, cfg, dtype=np.float32):
    """Per-point symbol (-1 for anchors), reconstruction and level."""
    x = np.ascontiguousarray(x, dtype=dtype)
    sym = np.empty(x.shape, dtype=np.int32)
    rec = np.empty(x.shape, dtype=dtype)
    lvl = np.empty(x.shape, dtype=np.int32)
    st = getattr(lib(), "stz_ref_symbols" + _sfx(dtype))(
        x.ctypes.data, _dims(x.shape), eb_mode, eb, C.byref(cfg), sym.ctypes.data,
        rec.ctypes.data, lvl.ctypes.data)
    if st != OK:
        raise OracleError(st, "symbols")
    return sym, rec, lvl


def predict(rec, p, s, dtype=np.float32):
    rec = np.ascontiguousarray(rec, dtype=dtype)
    f = getattr(lib(), "stz_ref_predict" + _sfx(dtype))
    return float(f(rec.ctypes.data, _dims(rec.shape), _dims(p), s))


def huffman_lengths(counts, lmax=12):
    counts = np.ascontiguousarray(counts, dtype=np.uint64)
    lens = np.zeros(counts.size, dtype=np.uint8)
    lib().stz_ref_huffman_lengths(counts.ctypes.data, counts.size, lmax, lens.ctypes.data)
    return lens


def canonical_codes(lens):
    lens = np.ascontiguousarray(lens, dtype=np.uint8)
    codes = np.zeros(lens.size, dtype=np.uint32)
    lib().stz_ref_canonical_codes(lens.ctypes.data, lens.size, codes.ctypes.data)
    return codes


def level_bounds(eb_abs, ratio, L):
    e = np.zeros(L + 1, dtype=np.float64)
    E2 = np.zeros(L + 1, dtype=np.float32)
    INV = np.zeros(L + 1, dtype=np.float32)
    lib().stz_ref_level_bounds(eb_abs, ratio, L, e.ctypes.data, E2.ctypes.data, INV.ctypes.data)
    return e, E2, INV


def units_decoded():
    """Units decoded by the last decode call, as an array [level, class]."""
    out = np.zeros(9 * 8, dtype=np.uint64)
    lib().stz_ref_units_decoded(out.ctypes.data)
    return out.reshape(9, 8)


def roi_units(comp, level, unit):
    """Number of ROI units: blocks (unit 0) or level-grid planes across an axis."""
    inf = info(comp)
    if unit == 0:
        n = 1
        for d in inf.dims:
            n *= (int(d) + inf.block - 1) // inf.block
        return n
    s = 1 << (inf.levels - level)
    return (int(inf.dims[unit - 1]) - 1) // s + 1


def roi_select(comp, level, unit, stat, rule, value):
    """ROI selection (Sec. 3.3): (selected unit indices, per-unit statistic)."""
    n = roi_units(comp, level, unit)
    sel = np.empty(max(n, 1), dtype=np.uint32)
    stats = np.empty(max(n, 1), dtype=np.float64)
    cnt = C.c_uint64(0)
    buf = np.frombuffer(comp, dtype=np.uint8)
    st = lib().stz_ref_roi_select(buf.ctypes.data, buf.size, level, unit, stat, rule, value,
                                  sel.ctypes.data, sel.size, C.byref(cnt), stats.ctypes.data)
    if st != OK:
        raise OracleError(st, "roi_select")
    return sel[:cnt.value].copy(), stats[:n].copy()

