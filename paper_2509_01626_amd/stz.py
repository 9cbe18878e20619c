"""ctypes binding of the C ABI in include/stz.h (argument marshalling only).

Every step of the compressor runs in the HIP library ``libstz.so``; this
module passes device pointers taken from torch tensors and the current HIP
stream. Importing it never falls back to a CPU path: if the library is missing
or fails to load, every call raises.
"""
import ctypes as C
import os

import torch

from . import build as _build

OK, ERR_ARG, ERR_NONFINITE, ERR_BUFFER, ERR_CORRUPT, ERR_DEVICE, ERR_NOMEM = 0, -1, -2, -3, -4, -5, -6
EB_ABS, EB_REL = 0, 1


class Config(C.Structure):
    _fields_ = [("block", C.c_uint32), ("levels", C.c_uint32), ("radius", C.c_uint32),
                ("coding", C.c_uint32), ("eb_ratio", C.c_double)]


class Info(C.Structure):
    _fields_ = [("dims", C.c_uint64 * 3), ("block", C.c_uint32), ("levels", C.c_uint32),
                ("radius", C.c_uint32), ("lmax", C.c_uint32), ("eb_mode", C.c_uint32),
                ("dtype", C.c_uint32), ("eb", C.c_double), ("eb_abs", C.c_double),
                ("eb_ratio", C.c_double), ("total_bytes", C.c_uint64),
                ("coding", C.c_uint32), ("reserved", C.c_uint32)]


class Job(C.Structure):
    _fields_ = [("x", C.c_void_p), ("dims", C.c_uint64 * 3), ("eb_mode", C.c_int32),
                ("reserved", C.c_uint32), ("eb", C.c_double), ("cfg", Config),
                ("out", C.c_void_p), ("out_cap", C.c_uint64), ("out_size", C.c_uint64),
                ("status", C.c_int32), ("reserved2", C.c_uint32)]


class Request(C.Structure):
    _fields_ = [("field", C.c_void_p), ("lo", C.c_uint64 * 3), ("hi", C.c_uint64 * 3),
                ("level", C.c_uint32), ("reserved", C.c_uint32), ("out", C.c_void_p),
                ("out_cap_elems", C.c_uint64), ("out_dims", C.c_uint64 * 3),
                ("status", C.c_int32), ("reserved2", C.c_uint32)]


class StzError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {_status_string(status)} ({status})")
        self.status = status


_lib = None


def lib():
    """Load libstz.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            raise RuntimeError(f"HIP library not built: {_build.LIB} is missing "
                               "(run __graft_entry__.build())")
        L = C.CDLL(_build.LIB)
        u64p = C.POINTER(C.c_uint64)
        for sfx in ("", "_f64"):  # float32 and float64 variants, same signatures
            f = getattr(L, "stz_compress_bound" + sfx)
            f.restype = C.c_uint64
            f.argtypes = [u64p, C.POINTER(Config)]
            f = getattr(L, "stz_compress" + sfx)
            f.restype = C.c_int
            f.argtypes = [C.c_void_p, u64p, C.c_int, C.c_double, C.POINTER(Config), C.c_void_p,
                          C.c_uint64, u64p, C.c_void_p]
            f = getattr(L, "stz_decompress" + sfx)
            f.restype = C.c_int
            f.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.c_void_p]
            f = getattr(L, "stz_decompress_level" + sfx)
            f.restype = C.c_int
            f.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_void_p, C.c_uint64, u64p,
                          C.c_void_p]
            f = getattr(L, "stz_decompress_region" + sfx)
            f.restype = C.c_int
            f.argtypes = [C.c_void_p, C.c_uint64, u64p, u64p, C.c_uint32, C.c_void_p,
                          C.c_uint64, u64p, C.c_void_p]
        L.stz_decompress_region_noalloc.restype = C.c_int
        L.stz_decompress_region_noalloc.argtypes = [C.c_void_p, C.c_uint64, u64p, u64p,
                                                    C.c_uint32, C.c_void_p, C.c_uint64, u64p,
                                                    C.c_void_p]
        L.stz_info.restype = C.c_int
        L.stz_info.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(Info), C.c_void_p]
        L.stz_compress_batch.restype = C.c_int
        L.stz_compress_batch.argtypes = [C.POINTER(Job), C.c_uint64, C.c_void_p]
        L.stz_open.restype = C.c_int
        L.stz_open.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_void_p), C.c_void_p]
        L.stz_field_info.restype = C.c_int
        L.stz_field_info.argtypes = [C.c_void_p, C.POINTER(Info)]
        L.stz_close.restype = None
        L.stz_close.argtypes = [C.c_void_p]
        L.stz_decompress_batch.restype = C.c_int
        L.stz_decompress_batch.argtypes = [C.POINTER(Request), C.c_uint64, C.c_void_p,
                                           C.c_void_p]
        L.stz_compress_batch_plan.restype = C.c_int
        L.stz_compress_batch_plan.argtypes = [C.POINTER(Job), C.c_uint64, C.POINTER(C.c_void_p),
                                              C.c_void_p]
        L.stz_decompress_batch_plan.restype = C.c_int
        L.stz_decompress_batch_plan.argtypes = [C.POINTER(Request), C.c_uint64,
                                                C.POINTER(C.c_void_p), C.c_void_p]
        L.stz_batch_run.restype = C.c_int
        L.stz_batch_run.argtypes = [C.c_void_p, C.c_void_p]
        L.stz_batch_status.restype = C.c_int
        L.stz_batch_status.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64,
                                       C.c_void_p]
        L.stz_batch_destroy.restype = None
        L.stz_batch_destroy.argtypes = [C.c_void_p]
        L.stz_autotune_batch.restype = C.c_int
        L.stz_autotune_batch.argtypes = [C.POINTER(Job), C.c_uint64, C.c_char_p, C.c_uint64,
                                         C.c_void_p]
        L.stz_roi_select.restype = C.c_int
        L.stz_roi_select.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                     C.c_double, C.c_void_p, C.c_uint64,
                                     C.POINTER(C.c_uint64), C.c_void_p, C.c_void_p]
        L.stz_trim.restype = C.c_int
        L.stz_trim.argtypes = []
        L.stz_status_string.restype = C.c_char_p
        L.stz_status_string.argtypes = [C.c_int]
        _lib = L
    return _lib


def _status_string(st):
    try:
        return lib().stz_status_string(st).decode()
    except Exception:  # pragma: no cover
        return "status"


def _dims(shape):
    return (C.c_uint64 * 3)(*[int(v) for v in shape])


# The current stream's raw handle without building a torch Stream object
# (the per-call cost of torch.cuda.current_stream() is ~2.5 us).
_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)
_cur_device = getattr(torch._C, "_cuda_getDevice", None)


def _stream(stream=None):
    if stream is not None:
        return C.c_void_p(stream.cuda_stream)
    if _raw_stream is not None and _cur_device is not None:
        return C.c_void_p(_raw_stream(_cur_device()))
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


_FN = {}


def _fn(name):
    """Entry point `name` of the library (looked up once)."""
    f = _FN.get(name)
    if f is None:
        f = _FN[name] = getattr(lib(), name)
    return f


def _as_shape(t, shape, n):
    """The first n elements of t viewed as `shape` (t itself when it already
    has that shape)."""
    if t.shape == shape:
        return t
    return t.reshape(-1)[:n].view(shape)


def stz_trim():
    """Release the library's cached device scratch on the current device."""
    st = lib().stz_trim()
    if st != OK:
        raise StzError(st, "stz_trim")


CODING_DEFAULT, CODING_HUFFMAN, CODING_ZERO_CHUNKS = 0, 1, 2


def config(block=32, levels=0, radius=0, eb_ratio=0.0, coding=CODING_DEFAULT):
    return Config(block, levels, radius, coding, eb_ratio)


def _check_dev(t, dtype):
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} tensor on a GPU")


def _sfx(dtype):
    """Entry-point suffix of a value type: float32 -> "", float64 -> "_f64"."""
    if dtype == torch.float32:
        return ""
    if dtype == torch.float64:
        return "_f64"
    raise ValueError(f"unsupported value type {dtype} (float32 or float64)")


def value_type(inf):
    """torch value type of a stream, from its info record."""
    return torch.float64 if inf.dtype == 1 else torch.float32


def stz_compress_bound(shape, cfg, dtype=torch.float32):
    return int(getattr(lib(), "stz_compress_bound" + _sfx(dtype))(_dims(shape), C.byref(cfg)))


def stz_compress(x, eb_mode, eb, cfg, out=None, stream=None):
    """Compress device tensor x (float32 or float64, shape (nz, ny, nx)).
    Returns a uint8 device tensor holding the stream (a view of `out` when
    given)."""
    sfx = _sfx(x.dtype)
    _check_dev(x, x.dtype)
    assert x.dim() == 3
    if out is None:
        out = torch.empty(stz_compress_bound(x.shape, cfg, x.dtype), dtype=torch.uint8,
                          device=x.device)
    _check_dev(out, torch.uint8)
    size = C.c_uint64(0)
    st = _fn("stz_compress" + sfx)(
        x.data_ptr(), _dims(x.shape), eb_mode, eb, C.byref(cfg),
        out.data_ptr(), out.numel(), C.byref(size), _stream(stream))
    if st != OK:
        raise StzError(st, "stz_compress" + sfx)
    return out[: size.value]


def stz_compress_status(x, eb_mode, eb, cfg, out_cap=None, stream=None):
    """Status code and reported size of a compress call (never raises)."""
    sfx = _sfx(x.dtype)
    cap = stz_compress_bound(x.shape, cfg, x.dtype) if out_cap is None else out_cap
    out = torch.empty(max(cap, 1), dtype=torch.uint8, device=x.device)
    size = C.c_uint64(0)
    st = getattr(lib(), "stz_compress" + sfx)(
        C.c_void_p(x.data_ptr()), _dims(x.shape), eb_mode, eb, C.byref(cfg),
        C.c_void_p(out.data_ptr()), cap, C.byref(size), _stream(stream))
    return st, size.value


def stz_info(comp, stream=None):
    _check_dev(comp, torch.uint8)
    inf = Info()
    st = lib().stz_info(C.c_void_p(comp.data_ptr()), comp.numel(), C.byref(inf), _stream(stream))
    if st != OK:
        raise StzError(st, "stz_info")
    return inf


# The decoders take the variant of the output's value type: by default the
# stream's own; a given `out` of the other type gets STZ_ERR_ARG back.
def stz_decompress(comp, out=None, stream=None, info=None):
    inf = info if info is not None else stz_info(comp, stream)
    shape = tuple(int(v) for v in inf.dims)
    if out is None:
        out = torch.empty(shape, dtype=value_type(inf), device=comp.device)
    sfx = _sfx(out.dtype)
    _check_dev(out, out.dtype)
    st = _fn("stz_decompress" + sfx)(comp.data_ptr(), comp.numel(), out.data_ptr(), out.numel(),
                                     _stream(stream))
    if st != OK:
        raise StzError(st, "stz_decompress" + sfx)
    return out if out.shape == shape else out.view(shape)


def level_shape(inf, level):
    s = 1 << (inf.levels - level)
    return tuple((int(n) - 1) // s + 1 for n in inf.dims)


def region_shape(inf, lo, hi, level):
    s = 1 << (inf.levels - level)
    out = []
    for d in range(3):
        first = -(-int(lo[d]) // s) * s
        out.append((int(hi[d]) - 1 - first) // s + 1 if first < int(hi[d]) else 0)
    return tuple(out)


def stz_decompress_level(comp, level, out=None, stream=None, info=None):
    inf = info if info is not None else stz_info(comp, stream)
    shape = level_shape(inf, level)
    n = shape[0] * shape[1] * shape[2]
    if out is None:
        out = torch.empty(shape, dtype=value_type(inf), device=comp.device)
    sfx = _sfx(out.dtype)
    _check_dev(out, out.dtype)
    od = (C.c_uint64 * 3)()
    st = _fn("stz_decompress_level" + sfx)(
        comp.data_ptr(), comp.numel(), level, out.data_ptr(), out.numel(), od, _stream(stream))
    if st != OK:
        raise StzError(st, "stz_decompress_level" + sfx)
    assert tuple(od) == shape
    return _as_shape(out, shape, n)


def stz_decompress_region(comp, lo, hi, level, out=None, stream=None, info=None):
    inf = info if info is not None else stz_info(comp, stream)
    shape = region_shape(inf, lo, hi, level)
    n = shape[0] * shape[1] * shape[2]
    if out is None:
        out = torch.empty(max(n, 1), dtype=value_type(inf), device=comp.device)
    sfx = _sfx(out.dtype)
    _check_dev(out, out.dtype)
    od = (C.c_uint64 * 3)()
    st = _fn("stz_decompress_region" + sfx)(
        comp.data_ptr(), comp.numel(), _dims(lo), _dims(hi), level, out.data_ptr(), out.numel(),
        od, _stream(stream))
    if st != OK:
        raise StzError(st, "stz_decompress_region" + sfx)
    assert tuple(od) == shape, (tuple(od), shape)
    return _as_shape(out, shape, n)


NOALLOC_SCRATCH_BYTES = 64 << 20  # STZ_NOALLOC_SCRATCH_BYTES


def stz_decompress_region_noalloc(comp, lo, hi, level, out, stream=None):
    """The allocation-free region decode (float32 streams) into the caller's
    `out` (device float32); returns (status, out_dims) and never raises."""
    _check_dev(out, torch.float32)
    od = (C.c_uint64 * 3)()
    st = lib().stz_decompress_region_noalloc(
        C.c_void_p(comp.data_ptr()), comp.numel(), _dims(lo), _dims(hi), level,
        C.c_void_p(out.data_ptr()), out.numel(), od, _stream(stream))
    return st, tuple(int(v) for v in od)


def decode_status(comp, fn="decompress", level=0, lo=None, hi=None, stream=None,
                  dtype=torch.float32):
    """Status of a decode call (the `dtype` variant) on possibly corrupt bytes
    (never raises)."""
    out = torch.empty(1 << 22, dtype=dtype, device=comp.device)
    od = (C.c_uint64 * 3)()
    L = lib()
    x = _sfx(dtype)
    p, n = C.c_void_p(comp.data_ptr()), comp.numel()
    if fn == "decompress":
        return getattr(L, "stz_decompress" + x)(p, n, C.c_void_p(out.data_ptr()), out.numel(),
                                                _stream(stream))
    if fn == "level":
        return getattr(L, "stz_decompress_level" + x)(p, n, level, C.c_void_p(out.data_ptr()),
                                                      out.numel(), od, _stream(stream))
    return getattr(L, "stz_decompress_region" + x)(p, n, _dims(lo), _dims(hi), level,
                                                   C.c_void_p(out.data_ptr()), out.numel(), od,
                                                   _stream(stream))


# ---- batched compression -------------------------------------------------------
def make_jobs(xs, modes, ebs, cfgs, outs):
    """ctypes job array for device tensors xs (float32) and byte buffers outs."""
    n = len(xs)
    jobs = (Job * n)()
    for i in range(n):
        x, out = xs[i], outs[i]
        _check_dev(x, torch.float32)
        _check_dev(out, torch.uint8)
        j = jobs[i]
        j.x = x.data_ptr()
        for d in range(3):
            j.dims[d] = int(x.shape[d])
        j.eb_mode = int(modes[i])
        j.eb = float(ebs[i])
        j.cfg = cfgs[i]
        j.out = out.data_ptr()
        j.out_cap = out.numel()
    return jobs


def stz_compress_batch(xs, modes, ebs, cfgs, outs, stream=None, check=True):
    """Compress many fields with one launch sequence; returns the compressed
    views (outs[i][:size]) and the ctypes job array (per-job status/size)."""
    jobs = make_jobs(xs, modes, ebs, cfgs, outs)
    st = lib().stz_compress_batch(jobs, len(xs), _stream(stream))
    if check and st != OK:
        raise StzError(st, "stz_compress_batch")
    return [outs[i][:jobs[i].out_size] for i in range(len(xs))], jobs


def stz_autotune_batch(jobs, stream=None):
    """Tune the batched launch shapes on `jobs` (a job array); returns the report."""
    buf = C.create_string_buffer(8192)
    st = lib().stz_autotune_batch(jobs, len(jobs), buf, 8192, _stream(stream))
    if st != OK:
        raise StzError(st, "stz_autotune_batch")
    return buf.value.decode()


# ---- resident fields and batched decoding ----------------------------------------
class Field:
    """A compressed stream kept in device memory with its decoder table
    (stz_open); `comp` must stay alive and unchanged while the field is open."""

    def __init__(self, comp, stream=None):
        _check_dev(comp, torch.uint8)
        self.comp = comp
        h = C.c_void_p()
        st = lib().stz_open(C.c_void_p(comp.data_ptr()), comp.numel(), C.byref(h),
                            _stream(stream))
        if st != OK:
            raise StzError(st, "stz_open")
        self.handle = h
        self.info = Info()
        lib().stz_field_info(h, C.byref(self.info))

    def close(self):
        if self.handle:
            lib().stz_close(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # pragma: no cover
            pass


def make_requests(items):
    """items: (field, lo, hi, level, out tensor) tuples -> ctypes request array."""
    n = len(items)
    reqs = (Request * n)()
    for i, (f, lo, hi, level, out) in enumerate(items):
        _check_dev(out, torch.float32)
        r = reqs[i]
        r.field = f.handle
        for d in range(3):
            r.lo[d] = int(lo[d])
            r.hi[d] = int(hi[d])
        r.level = int(level)
        r.out = out.data_ptr()
        r.out_cap_elems = out.numel()
    return reqs


def stz_decompress_batch(reqs, flags=None, stream=None, check=True):
    """Run a request array. With `flags` (device uint32 tensor, one word per
    request) the call is asynchronous and corruption lands in the flags."""
    fp = None
    if flags is not None:
        if not flags.is_cuda or flags.dtype != torch.int32 or flags.numel() < len(reqs):
            raise ValueError("flags must be a device int32 tensor with one word per request")
        fp = C.c_void_p(flags.data_ptr())
    st = lib().stz_decompress_batch(reqs, len(reqs), fp, _stream(stream))
    if check and st != OK:
        raise StzError(st, "stz_decompress_batch")
    return st


# ---- captured batches (HIP graphs) ------------------------------------------
class BatchPlan:
    """A compression plan over a job array (stz_compress_batch_plan) or a
    decode plan over a request array (stz_decompress_batch_plan): run()
    replays the captured graph asynchronously, status() reads the last run."""

    def __init__(self, jobs=None, reqs=None, stream=None):
        h = C.c_void_p()
        if (jobs is None) == (reqs is None):
            raise ValueError("give exactly one of jobs, reqs")
        self.jobs, self.reqs = jobs, reqs
        if jobs is not None:
            st = lib().stz_compress_batch_plan(jobs, len(jobs), C.byref(h), _stream(stream))
            what = "stz_compress_batch_plan"
        else:
            st = lib().stz_decompress_batch_plan(reqs, len(reqs), C.byref(h), _stream(stream))
            what = "stz_decompress_batch_plan"
        if st != OK:
            raise StzError(st, what)
        self.handle = h

    def run(self, stream=None):
        st = lib().stz_batch_run(self.handle, _stream(stream))
        if st != OK:
            raise StzError(st, "stz_batch_run")

    def status(self, stream=None):
        """Synchronize and write the last run's statuses (and sizes) into the
        planned array; returns the first failing status."""
        n = len(self.jobs) if self.jobs is not None else len(self.reqs)
        return lib().stz_batch_status(self.handle, self.jobs, self.reqs, n, _stream(stream))

    def close(self):
        if self.handle:
            lib().stz_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # pragma: no cover
            pass


# ---- ROI selection ------------------------------------------------------------
ROI_BLOCKS, ROI_SLICES_Z, ROI_SLICES_Y, ROI_SLICES_X = 0, 1, 2, 3
ROI_MAX, ROI_RANGE = 0, 1
ROI_THRESHOLD, ROI_TOP_FRACTION = 0, 1


def roi_units(info, level, unit):
    if unit == ROI_BLOCKS:
        n = 1
        for d in info.dims:
            n *= (int(d) + info.block - 1) // info.block
        return n
    s = 1 << (info.levels - level)
    return (int(info.dims[unit - 1]) - 1) // s + 1


def stz_roi_select(field, level, unit=ROI_BLOCKS, stat=ROI_MAX, rule=ROI_THRESHOLD, value=0.0,
                   stream=None):
    """Select ROI units of a resident field from its level-`level` decode:
    returns (selected unit indices, per-unit statistic) as numpy arrays."""
    import numpy as np
    n = roi_units(field.info, level, unit)
    sel = np.empty(max(n, 1), dtype=np.uint32)
    stats = np.empty(max(n, 1), dtype=np.float64)
    cnt = C.c_uint64(0)
    st = lib().stz_roi_select(field.handle, level, unit, stat, rule, float(value),
                              sel.ctypes.data, sel.size, C.byref(cnt), stats.ctypes.data,
                              _stream(stream))
    if st != OK:
        raise StzError(st, "stz_roi_select")
    return sel[:cnt.value].copy(), stats[:n].copy()


def roi_block_boxes(info, blocks):
    """Full-resolution boxes [lo, hi) of ROI block indices (raster order)."""
    B = info.block
    nb = [(int(d) + B - 1) // B for d in info.dims]
    out = []
    for b in blocks:
        b = int(b)
        idx = (b // (nb[1] * nb[2]), (b // nb[2]) % nb[1], b % nb[2])
        lo = [i * B for i in idx]
        hi = [min(int(d), l + B) for d, l in zip(info.dims, lo)]
        out.append((lo, hi))
    return out

