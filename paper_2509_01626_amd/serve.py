"""Continuous-batching decode server over resident compressed fields.

Compressed streams stay in device memory (``stz.Field``: header parsed and
decoder table uploaded once). Requests for a box of a field at a progressive
level (Sec. 3.3: progressive and random-access decompression) arrive at any
time. The loop

1. admits waiting requests in arrival order while their outputs fit in the
   output arena (admission by memory; a request larger than the whole arena is
   rejected);
2. whenever one of its ``slots`` (HIP streams) is idle, launches every
   admitted request (up to ``max_batch``) as one batched decode on that stream,
   asynchronously, with one device status word per request;
3. polls the in-flight batches' events; a finished batch hands each result to
   ``on_done`` and frees its arena space, which lets more requests in.

Nothing allocates or frees device or pinned memory inside the loop: each
slot's flag words (device and pinned host) are allocated once, the status
words come back by an asynchronous copy on the slot's own stream (no call on
the default stream, which would wait for every slot), and ``prewarm`` sizes
the library's per-stream scratch and staging for the largest batch up front.
A result view handed to ``on_done`` is valid only until the callback returns;
work the callback enqueues on the current stream (a copy of the view, say) is
ordered before the region is reused: the region goes back to the arena only
once an event recorded on that stream after the callbacks has completed.

So requests arriving while others are on the GPU join the next batch as soon
as a slot and memory free up, and batches on different slots overlap on the
device. Latency = time the host sees the batch finished - arrival time.

All decoding runs in the HIP library; this module only schedules.
"""
import collections
import gc
import time

import torch

from . import stz


class Arena:
    """First-fit allocator over one device float32 buffer (offsets in floats,
    rounded up to 64-float granules)."""

    G = 64

    def __init__(self, n_floats, device):
        self.n = (int(n_floats) // self.G) * self.G
        self.buf = torch.empty(self.n, dtype=torch.float32, device=device)
        self.free = [(0, self.n)]  # sorted (offset, length)

    def alloc(self, n):
        n = max(self.G, -(-int(n) // self.G) * self.G)
        for i, (o, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (o + n, ln - n)
                return o, n
        return None

    def release(self, o, n):
        self.free.append((o, n))
        self.free.sort()
        merged = []
        for a, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == a:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((a, ln))
        self.free = merged

    def view(self, o, n):
        return self.buf[o:o + n]


class Request:
    __slots__ = ("rid", "field", "lo", "hi", "level", "t_arrive", "t_done", "shape", "n",
                 "off", "cap", "status")

    def __init__(self, rid, field, lo, hi, level, t_arrive):
        self.rid = rid
        self.field = field
        self.lo = list(lo)
        self.hi = list(hi)
        self.level = int(level)
        self.t_arrive = t_arrive
        self.t_done = None
        self.shape = None
        self.n = 0
        self.off = None
        self.cap = 0
        self.status = None


class Server:
    def __init__(self, fields, arena_bytes, slots=2, max_batch=64, device="cuda:0",
                 on_done=None):
        self.fields = fields
        self.arena = Arena(arena_bytes // 4, device)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
        self.busy = [None] * slots        # per slot: batch in flight, or None
        self.t_launch = [0.0] * slots
        self.events = [torch.cuda.Event() for _ in range(slots)]
        self.dflags = [torch.empty(max_batch, dtype=torch.int32, device=device)
                       for _ in range(slots)]
        self.hflags = [torch.empty(max_batch, dtype=torch.int32, pin_memory=True)
                       for _ in range(slots)]
        self.max_batch = max_batch
        self.device = device
        self.on_done = on_done
        self.waiting = collections.deque()
        self.admitted = []
        self.done = []
        self.releasing = collections.deque()  # (event, [(off, cap)]) after on_done
        self.batches = 0
        self.batch_sizes = []
        self.trace = []  # per batch: (launch time, time seen done, size)

    def prewarm(self, field, edge, level):
        """Decode a full batch of the largest expected request (a box of
        `edge` points per axis in the middle of the field, whose dependency
        cone no face clips) on every slot into a temporary buffer, so the
        library's per-stream scratch and pinned staging reach their final
        size before serving starts."""
        f = self.fields[field]
        dims = [int(v) for v in f.info.dims]
        lo = [max(0, (d - edge) // 2) for d in dims]
        hi = [min(d, a + edge) for a, d in zip(lo, dims)]
        shp = stz.region_shape(f.info, lo, hi, level)
        n = max(1, shp[0] * shp[1] * shp[2])
        tmp = torch.empty(n * self.max_batch, dtype=torch.float32, device=self.device)
        for s, st in enumerate(self.streams):
            items = [(f, lo, hi, level, tmp[i * n:(i + 1) * n]) for i in range(self.max_batch)]
            arr = stz.make_requests(items)
            with torch.cuda.stream(st):
                stz.stz_decompress_batch(arr, flags=self.dflags[s], stream=st, check=False)
            st.synchronize()
        del tmp

    # -- request intake ---------------------------------------------------------------
    def submit(self, req):
        f = self.fields[req.field]
        req.shape = stz.region_shape(f.info, req.lo, req.hi, req.level)
        req.n = req.shape[0] * req.shape[1] * req.shape[2]
        if req.n > self.arena.n:
            req.status = stz.ERR_NOMEM
            req.t_done = time.perf_counter()
            self.done.append(req)
            return
        self.waiting.append(req)

    def _admit(self):
        while self.releasing and self.releasing[0][0].query():
            for o, n in self.releasing.popleft()[1]:
                self.arena.release(o, n)
        while self.waiting:
            r = self.waiting[0]
            got = self.arena.alloc(max(r.n, 1))
            if got is None:
                return
            r.off, r.cap = got
            self.admitted.append(self.waiting.popleft())

    def _launch(self):
        for s in range(len(self.streams)):
            if not self.admitted:
                return
            if self.busy[s] is not None:
                continue
            batch = self.admitted[:self.max_batch]
            del self.admitted[:len(batch)]
            items = [(self.fields[r.field], r.lo, r.hi, r.level,
                      self.arena.view(r.off, r.cap)) for r in batch]
            arr = stz.make_requests(items)
            st = self.streams[s]
            nb = len(batch)
            with torch.cuda.stream(st):
                stz.stz_decompress_batch(arr, flags=self.dflags[s], stream=st, check=False)
                self.hflags[s][:nb].copy_(self.dflags[s][:nb], non_blocking=True)
                self.events[s].record(st)
            for i, r in enumerate(batch):
                r.status = arr[i].status
            self.busy[s] = batch
            self.t_launch[s] = time.perf_counter()
            self.batches += 1
            self.batch_sizes.append(nb)

    def _reap(self):
        for s in range(len(self.streams)):
            batch = self.busy[s]
            if batch is None or not self.events[s].query():
                continue
            t = time.perf_counter()
            self.trace.append((self.t_launch[s], t, len(batch)))
            fl = self.hflags[s][:len(batch)].tolist()
            regions = []
            for r, f in zip(batch, fl):
                if r.status == stz.OK and f:
                    r.status = stz.ERR_CORRUPT
                r.t_done = t
                if self.on_done is not None:
                    self.on_done(r, self.arena.view(r.off, max(r.n, 1))[:r.n].view(r.shape))
                regions.append((r.off, r.cap))
                self.done.append(r)
            if self.on_done is not None:
                ev = torch.cuda.Event()
                ev.record(torch.cuda.current_stream(self.device))
                self.releasing.append((ev, regions))
            else:
                for o, n in regions:
                    self.arena.release(o, n)
            self.busy[s] = None

    def step(self):
        self._reap()
        self._admit()
        self._launch()

    def idle(self):
        return (not self.waiting and not self.admitted and not self.releasing and
                all(b is None for b in self.busy))

    # -- driver ---------------------------------------------------------------------
    def run(self, arrivals):
        """arrivals: list of (t_offset_seconds, field, lo, hi, level), sorted by time.
        Submits each at its arrival time (relative to the start) and runs the loop
        until every request is done. Returns the finished requests."""
        # Python's cyclic garbage collector is paused while serving: a full
        # collection over a long run's objects stalls the loop for tens of ms
        gc_was_on = gc.isenabled()
        gc.disable()
        try:
            t0 = time.perf_counter()
            i = 0
            n = len(arrivals)
            while i < n or not self.idle():
                now = time.perf_counter()
                while i < n and arrivals[i][0] <= now - t0:
                    ta, f, lo, hi, lv = arrivals[i]
                    self.submit(Request(i, f, lo, hi, lv, t0 + ta))
                    i += 1
                self.step()
        finally:
            if gc_was_on:
                gc.enable()
        return self.done


def poisson_arrivals(rng, n, rate, fields_info, edge=(16, 256)):
    """n requests with exponential inter-arrival times (rate per second): a
    uniform field, a uniform progressive level 0..L and a box whose edge per
    axis is uniform in `edge` (clipped to the field) at a uniform origin."""
    t = 0.0
    out = []
    for _ in range(n):
        t += rng.exponential(1.0 / rate)
        k = int(rng.integers(0, len(fields_info)))
        inf = fields_info[k]
        dims = [int(v) for v in inf.dims]
        lo, hi = [], []
        for d in dims:
            e = min(d, int(rng.integers(edge[0], edge[1] + 1)))
            a = int(rng.integers(0, d - e + 1))
            lo.append(a)
            hi.append(a + e)
        lv = int(rng.integers(0, inf.levels + 1))
        out.append((t, k, lo, hi, lv))
    return out


def latency_stats(done):
    """Latency percentiles (nearest rank on the sorted latencies), mean and
    maximum, in ms, over the requests that succeeded."""
    lat = sorted((r.t_done - r.t_arrive) for r in done if r.status == stz.OK)
    if not lat:
        return {"p50_ms": None, "p99_ms": None, "p999_ms": None, "max_ms": None,
                "mean_ms": None}

    def pct(p):
        i = min(len(lat) - 1, max(0, int(round(p / 100.0 * (len(lat) - 1)))))
        return lat[i] * 1e3

    return {"p50_ms": round(pct(50), 3), "p99_ms": round(pct(99), 3),
            "p999_ms": round(pct(99.9), 3), "max_ms": round(lat[-1] * 1e3, 3),
            "mean_ms": round(sum(lat) / len(lat) * 1e3, 3)}
