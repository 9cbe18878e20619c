"""Benchmark of the STZ hot path on one MI355X.

Default workload: one 512^3 float32 turbulence-like field (random-phase
isotropic k^-5/3 spectrum, unit variance), value-range-relative error bound
1e-3, 32^3 blocks (5 levels). One step is the whole hot path over that field:
compress, full decompression, progressive decompression at every coarser level
and one random-access box decode. Inputs are resident in HBM before timing.

Prints one JSON line. `value` is field GB/s of a step (field bytes / step
time); per-operation rates, the dominant kernel's roofline and the CPU oracle
baseline are reported beside it.
"""
import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "comp/decomp GB/s & % HBM peak at rel eb 1e-3; batched vs plain; p99 ROI latency"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--eb", type=float, default=1e-3)
    ap.add_argument("--block", type=int, default=32)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="do not record per-kernel events in the timed region")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--batch-fields", type=int, default=256,
                    help="fields in the many-field batch (0 = skip)")
    ap.add_argument("--block-sweep", type=int, default=1,
                    help="batched CR and speed of the many-field batch per block edge (0 = skip)")
    ap.add_argument("--scale-n", type=int, default=1024,
                    help="edge of the 4 co-located variables (0 = skip)")
    ap.add_argument("--serve-fields", type=int, default=16, help="resident fields (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests per offered load")
    ap.add_argument("--serve-warmup", type=int, default=500,
                    help="uncounted requests before each offered load")
    ap.add_argument("--serve-rates", default="1000,4000,16000",
                    help="offered loads, requests per second")
    ap.add_argument("--f64-dims", default="256,256,2048",
                    help="dims of the float64 field (empty = skip)")
    ap.add_argument("--coding-n", type=int, default=512,
                    help="edge of the smooth field of the coding section (0 = skip)")
    ap.add_argument("--only", default="",
                    help="comma list of sections to run: plain,batch,scale,serve,f64,coding,roi")
    return ap.parse_args()


COPY_PROBE_BYTES = 1 << 30


def copy_probe():
    """A plain device-to-device copy of known size: FETCH_SIZE / WRITE_SIZE of
    this kernel against its 1 GiB read and 1 GiB write give the factor that
    turns those counters into HBM bytes. Two reductions then read only the
    first 64 and the first 32 bytes of every 128-byte line of the same 1 GiB:
    FETCH_SIZE equal to the copy's shows that every read fetches whole lines,
    so the factor holds for any access pattern."""
    import torch
    src = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    rows = src.view(-1, 32)  # one 128-byte line per row
    half = float(rows[:, :16].sum())
    quarter = float(rows[:, :8].sum())
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": COPY_PROBE_BYTES, "half_line_sum": half,
                      "quarter_line_sum": quarter}), flush=True)


def kernel_sources_digest():
    """Digest of the sources of the device kernels (counters recorded for an
    older digest no longer describe the built kernels)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2509_01626_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel_key):
    """HBM bytes per launch of `kernel_key` from the committed counter summary
    (profiles/traffic_512cube.txt), or None when it was taken on other sources."""
    path = os.path.join(ROOT, "profiles", "traffic_512cube.txt")
    try:
        with open(path) as f:
            lines = f.read().splitlines()
    except OSError:
        return None
    digest = None
    for ln in lines:
        if ln.startswith("sources_digest:"):
            digest = ln.split(":", 1)[1].strip()
    if digest != kernel_sources_digest():
        return None
    for ln in lines:
        if ln.startswith("traffic " + kernel_key + " "):
            return int(ln.split()[2])
    return None


def kernel_bytes(name, level, info, lvl_tab, N):
    """Algorithmic bytes one launch of a kernel must move: the inputs it has to
    read and the outputs it has to write, each counted once."""
    L = info.levels
    dims = [int(v) for v in info.dims]

    def grid(l):
        s = 1 << (L - l)
        n = 1
        for d in dims:
            n *= (d - 1) // s + 1
        return n

    if name == "minmax":
        return 4 * N
    if level is None:
        return None
    n_l = grid(level) - grid(level - 1)
    coarse = grid(level - 1)
    words = lvl_tab[level]["words"]
    outl = lvl_tab[level]["outl"]
    if name == "predict":
        return 4 * n_l + 4 * coarse + 2 * n_l
    if name == "decode":
        return 4 * coarse + 4 * words + 4 * outl + 4 * n_l
    if name == "pack":
        return 2 * n_l + 4 * words + 4 * outl
    if name == "lanelen":
        return 2 * n_l
    if name == "upcopy":
        return 8 * grid(level - 2) if level >= 2 else None
    return None


def level_table(comp_host):
    import struct
    L = struct.unpack_from("<I", comp_host, 36)[0]
    tab = {}
    for l in range(1, L + 1):
        off, nu, nl, ns, w, o = struct.unpack_from("<6Q", comp_host, 128 + 48 * (l - 1))
        tab[l] = dict(off=off, units=nu, lanes=nl, syms=ns, words=w, outl=o)
    return tab


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); the path has "
              "no multi-GPU mode", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2509_01626_amd import fields, stz

    lib = stz.lib()
    dev = torch.device("cuda:0")
    dims = (args.n, args.n, args.n)
    t0 = time.time()
    x = fields.spectral(dims, 5.0 / 3.0, seed=args.seed)
    print(f"[bench] field {dims} generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    N = x.size
    field_bytes = 4 * N
    xd = torch.from_numpy(x).to(dev)
    cfg = stz.config(block=args.block)
    cap = stz.stz_compress_bound(dims, cfg)
    comp_buf = torch.empty(cap, dtype=torch.uint8, device=dev)
    out_full = torch.empty(dims, dtype=torch.float32, device=dev)
    comp = stz.stz_compress(xd, stz.EB_REL, args.eb, cfg, out=comp_buf)
    info = stz.stz_info(comp)
    L = info.levels
    lvl_out = [torch.empty(stz.level_shape(info, l), dtype=torch.float32, device=dev)
               for l in range(L)]
    rng = np.random.default_rng(7)
    edge = min(64, args.n)
    lo = [int(rng.integers(0, n - edge + 1)) for n in dims]
    hi = [a + edge for a in lo]
    reg_out = torch.empty(edge ** 3, dtype=torch.float32, device=dev)
    timings = {"compress": 0.0, "decompress": 0.0, "levels": 0.0, "region": 0.0}

    def step(record):
        t = time.perf_counter()
        c = stz.stz_compress(xd, stz.EB_REL, args.eb, cfg, out=comp_buf)
        t1 = time.perf_counter()
        stz.stz_decompress(c, out=out_full, info=info)
        t2 = time.perf_counter()
        for l in range(L):
            stz.stz_decompress_level(c, l, out=lvl_out[l], info=info)
        t3 = time.perf_counter()
        stz.stz_decompress_region(c, lo, hi, L, out=reg_out, info=info)
        t4 = time.perf_counter()
        if record:
            timings["compress"] += t1 - t
            timings["decompress"] += t2 - t1
            timings["levels"] += t3 - t2
            timings["region"] += t4 - t3
        return c

    for _ in range(args.warmup):
        step(False)
    # Timed region: K steps, no instrumentation. Python's cyclic garbage
    # collector is paused meanwhile: a full collection over this process's
    # objects stalls one host call by milliseconds.
    gc.collect()
    gc.disable()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(args.steps):
        comp = step(True)
    torch.cuda.synchronize()
    te = time.perf_counter()
    gc.enable()
    ms_per_step = (te - ts) * 1e3 / args.steps
    K = args.steps
    # Second timed region of K steps with the library's per-kernel HIP events
    # recorded on the launch stream (for the roofline of the dominant kernel).
    if not args.no_profile:
        lib.stz_profile_reset()
        lib.stz_profile_enable(1)
        torch.cuda.synchronize()
        for _ in range(args.steps):
            step(False)
        torch.cuda.synchronize()
        lib.stz_profile_enable(0)

    comp_host = comp.cpu().numpy().tobytes()
    tab = level_table(comp_host)
    full = out_full.cpu().numpy()
    err = float(np.abs(full.astype(np.float64) - x.astype(np.float64)).max())
    rng_v = float(x.max()) - float(x.min())
    mse = float(np.mean((full.astype(np.float64) - x.astype(np.float64)) ** 2))
    psnr = 20 * np.log10(rng_v) - 10 * np.log10(mse) if mse > 0 else float("inf")

    # Per-kernel device time (HIP events on the library's stream, timed region).
    import ctypes as C
    prof = {}
    for i in range(lib.stz_profile_count()):
        name = C.create_string_buffer(64)
        n = C.c_uint64(0)
        ms = C.c_double(0)
        lib.stz_profile_entry(i, name, 64, C.byref(n), C.byref(ms))
        prof[name.value.decode()] = (n.value, ms.value)
    roofline = None
    kernels = {}
    if prof:
        for key, (n, ms) in prof.items():
            nm, _, lv = key.partition("@")
            lvl = int(lv) if lv else None
            b = kernel_bytes(nm, lvl, info, tab, N)
            avg = ms / n
            kernels[key] = {"launches": n, "avg_us": round(avg * 1e3, 2),
                            "share": None,
                            "gbs": round(b / (avg * 1e-3) / 1e9, 1) if b else None}
        tot = sum(ms for (_, ms) in prof.values())
        for key in kernels:
            kernels[key]["share"] = round(prof[key][1] / tot, 4)
        dom = max(prof, key=lambda k: prof[k][1])
        nm, _, lv = dom.partition("@")
        b = kernel_bytes(nm, int(lv) if lv else None, info, tab, N)
        n, ms = prof[dom]
        if b:
            ach = b / (ms / n * 1e-3) / 1e9
            roofline = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                        "traffic": recorded_traffic(dom), "bytes_per_launch": int(b),
                        "avg_us": round(ms / n * 1e3, 2), "device_ms_per_step": round(tot / K, 3)}

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        ocfg = O.config(block=args.block)
        t = time.perf_counter()
        want = O.compress(x, O.EB_REL, args.eb, ocfg)
        t1 = time.perf_counter()
        ref = O.decompress(want)
        t2 = time.perf_counter()
        for l in range(L):
            O.decompress_level(want, l)
        O.decompress_region(want, lo, hi, L)
        t3 = time.perf_counter()
        parity = (want == comp_host) and bool(np.array_equal(ref.view(np.uint32),
                                                             full.view(np.uint32)))
        cpu = {"value": round(field_bytes / (t3 - t) / 1e9, 4), "unit": "GB/s", "cores": 1,
               "kind": "oracle",
               "sample": f"one full step on the same {dims[0]}^3 field (single thread): "
                         f"compress {t1 - t:.2f}s, full decode {t2 - t1:.2f}s, "
                         f"levels+region {t3 - t2:.2f}s",
               "cpu": _cpu_model(), "host_cores": os.cpu_count()}

    res = {
        "metric": METRIC,
        "value": round(field_bytes / (ms_per_step * 1e-3) / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{dims[0]}^3 k^-5/3 spectral float32, rel eb {args.eb:g}, "
                               f"B={args.block}: compress + full + progressive(0..{L - 1}) + "
                               f"{edge}^3 region decode",
                   "dims": list(dims), "eb_rel": args.eb, "block": args.block, "levels": L},
        "compress_gbps": round(field_bytes * K / timings["compress"] / 1e9, 2),
        "decompress_gbps": round(field_bytes * K / timings["decompress"] / 1e9, 2),
        "levels_ms": round(timings["levels"] * 1e3 / K, 3),
        "region_ms": round(timings["region"] * 1e3 / K, 3),
        "compression_ratio": round(field_bytes / len(comp_host), 3),
        "max_err_over_eb": round(err / info.eb_abs, 6),
        "psnr_db": round(float(psnr), 2),
        "parity_with_oracle": parity,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
    }
    only = set(x for x in args.only.split(",") if x)

    def want(name):
        return not only or name in only

    if args.batch_fields > 0 and want("batch"):
        res["batched"] = bench_batched(args, dev, oracle_check=not args.no_cpu_baseline)
    if args.scale_n > 0 and want("scale"):
        res["scale"] = bench_scale(args, dev)
    if args.serve_fields > 0 and want("serve"):
        res["serving"] = bench_serve(args, dev)
    if args.f64_dims and want("f64"):
        res["f64"] = bench_f64(args, dev, oracle_check=not args.no_cpu_baseline)
    if want("roi"):
        res["roi"] = bench_roi(args, dev, comp, comp_host, oracle_check=not args.no_cpu_baseline)
    if args.coding_n > 0 and want("coding"):
        res["coding"] = bench_coding(args, dev, oracle_check=not args.no_cpu_baseline)
    print(json.dumps(res), flush=True)


def _sync_time(f, reps=1):
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        f()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps


def bench_roi(args, dev, comp, comp_host, oracle_check=True):
    """ROI selection (Sec. 3.3, flexible workflow) on the workload's field: per
    progressive level, the first selection of a (level, unit, statistic)
    decodes the level and keeps the per-unit statistics with the field; later
    selections (other thresholds or fractions) run from the kept statistics.
    Latency of both, host-clocked around the synchronous call."""
    import numpy as np

    from paper_2509_01626_amd import stz
    f = stz.Field(comp)
    L = f.info.levels
    out = {"field": f"{args.n}^3", "block": args.block, "levels": {}}
    for level in range(L + 1):
        row = {}
        for stat, sname in ((stz.ROI_MAX, "max"), (stz.ROI_RANGE, "range")):
            t = time.perf_counter()
            sel, st = stz.stz_roi_select(f, level, stz.ROI_BLOCKS, stat,
                                         stz.ROI_TOP_FRACTION, 0.1)
            first = time.perf_counter() - t
            reps = 20
            t = time.perf_counter()
            for i in range(reps):
                sel2, _ = stz.stz_roi_select(f, level, stz.ROI_BLOCKS, stat,
                                             stz.ROI_TOP_FRACTION, 0.05 + 0.01 * i)
            cached = (time.perf_counter() - t) / reps
            t = time.perf_counter()
            for i in range(reps):
                stz.stz_roi_select(f, level, stz.ROI_BLOCKS, stat, stz.ROI_THRESHOLD,
                                   float(st.mean()))
            thr = (time.perf_counter() - t) / reps
            row[sname] = {"first_ms": round(first * 1e3, 3), "cached_top_ms": round(cached * 1e3, 3),
                          "cached_threshold_ms": round(thr * 1e3, 3), "units": int(st.size),
                          "selected": int(sel.size)}
        out["levels"][str(level)] = row
    if oracle_check:
        from oracle import oracle as ora
        lv = max(0, L - 2)
        osel, ost = ora.roi_select(comp_host, lv, stz.ROI_BLOCKS, stz.ROI_RANGE,
                                   stz.ROI_TOP_FRACTION, 0.1)
        sel, st = stz.stz_roi_select(f, lv, stz.ROI_BLOCKS, stz.ROI_RANGE,
                                     stz.ROI_TOP_FRACTION, 0.1)
        out["oracle_equal_level"] = lv
        out["oracle_equal"] = bool(np.array_equal(sel, osel) and np.array_equal(st, ost))
    f.close()
    return out


def bench_batched(args, dev, oracle_check=True):
    """Many uneven fields: plain per-field calls vs one batched launch sequence
    (launch shapes from the autotuner), same bounds, same outputs."""
    import numpy as np
    import torch

    from paper_2509_01626_amd import fields, stz
    desc = fields.batch_fields(args.batch_fields, 32, 256, seed=1000)
    t0 = time.time()
    xs = [fields.make_t(kind, dims, seed, dev) for kind, dims, seed, _ in desc]
    torch.cuda.synchronize()
    print(f"[bench] batch: {len(xs)} fields generated in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    ebs = [eb for _, _, _, eb in desc]
    B = 32
    cfgs = [stz.config(block=B) for _ in xs]
    modes = [stz.EB_REL] * len(xs)
    nvals = sum(x.numel() for x in xs)
    fbytes = 4 * nvals
    outs = [torch.empty(stz.stz_compress_bound(x.shape, c), dtype=torch.uint8, device=dev)
            for x, c in zip(xs, cfgs)]
    outs_p = [torch.empty_like(o) for o in outs]
    # plain path: one call per field
    plain_sizes = [0] * len(xs)

    def plain_c():
        for i, x in enumerate(xs):
            c = stz.stz_compress(x, modes[i], ebs[i], cfgs[i], out=outs_p[i])
            plain_sizes[i] = c.numel()

    plain_c()
    t_pc = _sync_time(plain_c, args.steps)
    jobs = stz.make_jobs(xs, modes, ebs, cfgs, outs)
    report = stz.stz_autotune_batch(jobs)
    print("[bench] autotune:\n" + report, file=sys.stderr, flush=True)

    def batch_c():
        st = stz.lib().stz_compress_batch(jobs, len(xs), stz._stream())
        if st != stz.OK:
            raise stz.StzError(st, "stz_compress_batch")

    batch_c()
    t_bc = _sync_time(batch_c, args.steps)
    sizes = [jobs[i].out_size for i in range(len(xs))]
    same = sizes == plain_sizes and all(
        torch.equal(outs[i][:sizes[i]], outs_p[i][:sizes[i]]) for i in range(len(xs)))
    comps = [outs[i][:sizes[i]] for i in range(len(xs))]
    # decompression: plain per-field calls vs one batch of full-domain requests
    recon = [torch.empty_like(x) for x in xs]

    def plain_d():
        for c, r in zip(comps, recon):
            stz.stz_decompress(c, out=r)

    plain_d()
    t_pd = _sync_time(plain_d, args.steps)
    flds = [stz.Field(c) for c in comps]
    recon_b = [torch.empty_like(x) for x in xs]
    reqs = stz.make_requests([(f, [0, 0, 0], list(x.shape), f.info.levels, r)
                              for f, x, r in zip(flds, xs, recon_b)])

    def batch_d():
        stz.stz_decompress_batch(reqs)

    batch_d()
    t_bd = _sync_time(batch_d, args.steps)
    same_d = all(torch.equal(a.view(torch.int32), b.view(torch.int32))
                 for a, b in zip(recon, recon_b))
    ok_bound = all(float((r - x).abs().max()) <= f.info.eb_abs * (1 + 1e-6)
                   for r, x, f in zip(recon_b, xs, flds))
    # the same batches captured once in HIP graphs and replayed
    outs_g = [torch.empty_like(o) for o in outs]
    jobs_g = stz.make_jobs(xs, modes, ebs, cfgs, outs_g)
    plan_c = stz.BatchPlan(jobs=jobs_g)
    plan_c.run()
    t_gc = _sync_time(plan_c.run, args.steps)
    same_gc = plan_c.status() == stz.OK and all(
        jobs_g[i].out_size == sizes[i] and torch.equal(outs_g[i][:sizes[i]], comps[i])
        for i in range(len(xs)))
    plan_c.close()
    del outs_g
    recon_g = [torch.empty_like(x) for x in xs]
    reqs_g = stz.make_requests([(f, [0, 0, 0], list(x.shape), f.info.levels, r)
                                for f, x, r in zip(flds, xs, recon_g)])
    plan_d = stz.BatchPlan(reqs=reqs_g)
    plan_d.run()
    t_gd = _sync_time(plan_d.run, args.steps)
    same_gd = plan_d.status() == stz.OK and all(
        torch.equal(a.view(torch.int32), b.view(torch.int32)) for a, b in zip(recon, recon_g))
    plan_d.close()
    del recon_g
    oracle_ok = None
    if oracle_check:
        from oracle import oracle as O
        order = sorted(range(len(xs)), key=lambda i: xs[i].numel())[:2]
        oracle_ok = True
        for i in order:
            want = O.compress(xs[i].cpu().numpy(), O.EB_REL, ebs[i], O.config(block=B))
            oracle_ok = oracle_ok and want == comps[i].cpu().numpy().tobytes()
            ref = O.decompress(want).reshape(-1)
            oracle_ok = oracle_ok and np.array_equal(
                recon_b[i].reshape(-1).cpu().numpy().view(np.uint32), ref.view(np.uint32))
    for f in flds:
        f.close()
    # The block edge is part of the format (it changes the bytes), so it is the
    # caller's choice: batched compression ratio and speed per edge, launch
    # shapes at their defaults, to show what each choice costs.
    sweep = []
    if args.block_sweep:
        for Bs in (8, 16, 32, 64):
            cfg_s = [stz.config(block=Bs) for _ in xs]
            outs_s = [torch.empty(stz.stz_compress_bound(x.shape, c), dtype=torch.uint8,
                                  device=dev) for x, c in zip(xs, cfg_s)]
            jobs_s = stz.make_jobs(xs, modes, ebs, cfg_s, outs_s)

            def batch_s():
                st = stz.lib().stz_compress_batch(jobs_s, len(xs), stz._stream())
                if st != stz.OK:
                    raise stz.StzError(st, "stz_compress_batch")

            batch_s()
            t_s = _sync_time(batch_s, args.steps)
            comps_s = [outs_s[i][:jobs_s[i].out_size] for i in range(len(xs))]
            flds_s = [stz.Field(c) for c in comps_s]
            rec_s = [torch.empty_like(x) for x in xs]
            reqs_s = stz.make_requests([(f, [0, 0, 0], list(x.shape), f.info.levels, r)
                                        for f, x, r in zip(flds_s, xs, rec_s)])

            def batch_sd():
                stz.stz_decompress_batch(reqs_s)

            batch_sd()
            t_sd = _sync_time(batch_sd, args.steps)
            sweep.append({"block": Bs,
                          "compression_ratio": round(fbytes / sum(jobs_s[i].out_size
                                                                  for i in range(len(xs))), 3),
                          "compress_gbps": round(fbytes / t_s / 1e9, 2),
                          "decompress_gbps": round(fbytes / t_sd / 1e9, 2)})
            for f in flds_s:
                f.close()
            del outs_s, comps_s, rec_s
            torch.cuda.empty_cache()
            print(f"[bench] batch block sweep: {sweep[-1]}", file=sys.stderr, flush=True)
    cr = fbytes / sum(sizes)
    res = {
        "workload": f"{len(xs)} float32 fields, dims per axis U[32,256] (half Gaussian bumps, "
                    f"half k^-5/3 spectral), rel eb log-uniform [1e-4,1e-2], B={B}",
        "fields": len(xs), "values": nvals, "field_gb": round(fbytes / 1e9, 3),
        "compression_ratio": round(cr, 3),
        "compress_gbps": {"plain": round(fbytes / t_pc / 1e9, 2),
                          "batched": round(fbytes / t_bc / 1e9, 2),
                          "graph": round(fbytes / t_gc / 1e9, 2)},
        "decompress_gbps": {"plain": round(fbytes / t_pd / 1e9, 2),
                            "batched": round(fbytes / t_bd / 1e9, 2),
                            "graph": round(fbytes / t_gd / 1e9, 2)},
        "compress_ms": {"plain": round(t_pc * 1e3, 3), "batched": round(t_bc * 1e3, 3),
                        "graph": round(t_gc * 1e3, 3)},
        "decompress_ms": {"plain": round(t_pd * 1e3, 3), "batched": round(t_bd * 1e3, 3),
                          "graph": round(t_gd * 1e3, 3)},
        "batched_bytes_equal_plain": bool(same), "batched_decode_equal_plain": bool(same_d),
        "graph_bytes_equal_eager": bool(same_gc), "graph_decode_equal_eager": bool(same_gd),
        "within_bound": bool(ok_bound), "oracle_sample_equal": oracle_ok,
        "autotune": [ln for ln in report.splitlines() if "tuned" in ln or "default" in ln],
        "block_sweep": sweep,
    }
    del xs, outs, outs_p, recon, recon_b, comps
    torch.cuda.empty_cache()
    stz.stz_trim()
    return res


def bench_f64(args, dev, oracle_check=True):
    """A float64 field shaped like the paper's double-precision workload
    (256 x 256 x 2048, 1 GiB): k^-5/3 spectral synthesis kept in double, rel eb
    1e-3, B = 32; compress and full decompress rates (inputs resident)."""
    import numpy as np
    import torch

    from paper_2509_01626_amd import fields, stz
    dims = tuple(int(v) for v in args.f64_dims.split(","))
    t0 = time.time()
    x = fields.spectral64_t(dims, 5.0 / 3.0, 77, dev)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(f"[bench] f64: {dims} generated in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    cfg = stz.config(block=32)
    fbytes = 8 * x.numel()
    out = torch.empty(stz.stz_compress_bound(dims, cfg, torch.float64), dtype=torch.uint8,
                      device=dev)
    rec = torch.empty_like(x)
    holder = {}

    def comp():
        holder["c"] = stz.stz_compress(x, stz.EB_REL, args.eb, cfg, out=out)

    comp()
    t_c = _sync_time(comp, args.steps)
    c = holder["c"]
    inf = stz.stz_info(c)

    def decomp():
        stz.stz_decompress(c, out=rec, info=inf)

    decomp()
    t_d = _sync_time(decomp, args.steps)
    err = float((rec - x).abs().max())
    oracle_ok = None
    if oracle_check:
        # the same path on a crop of the field, against the oracle, in this run
        from oracle import oracle as O
        crop = x[:32, :48, :256].contiguous()
        want = O.compress(crop.cpu().numpy(), O.EB_REL, args.eb, O.config(block=32),
                          dtype=np.float64)
        got = stz.stz_compress(crop, stz.EB_REL, args.eb, cfg).cpu().numpy().tobytes()
        oracle_ok = got == want
    res = {
        "workload": f"{dims[0]}x{dims[1]}x{dims[2]} float64 k^-5/3 spectral (double "
                    f"synthesis), rel eb {args.eb:g}, B=32: compress + full decompress",
        "dims": list(dims), "field_gb": round(fbytes / 1e9, 3),
        "compress_gbps": round(fbytes / t_c / 1e9, 2),
        "decompress_gbps": round(fbytes / t_d / 1e9, 2),
        "compress_ms": round(t_c * 1e3, 3), "decompress_ms": round(t_d * 1e3, 3),
        "compression_ratio": round(fbytes / c.numel(), 3),
        "max_err_over_eb": round(err / inf.eb_abs, 6),
        "oracle_crop_equal": oracle_ok,
        "paper_context": "paper, 2x EPYC 7742, FP64 WarpX 256^2x2048: compress 0.43 GB/s "
                         "serial / 2.15 GB/s 8 threads, decompress 0.72 / 2.68 GB/s",
    }
    del x, out, rec, holder, c
    torch.cuda.empty_cache()
    stz.stz_trim()
    return res


def bench_coding(args, dev, oracle_check=True):
    """Entropy-coding stages on a smooth field (sum of 32 Gaussian bumps plus
    1e-3 noise, n^3), where most chunks are all-centre: compression ratio and
    rates of Huffman only vs zero chunks + Huffman, rel eb 1e-2 and 1e-3,
    B = 32. Both reconstruct the same values."""
    import torch

    from paper_2509_01626_amd import fields, stz
    n = args.coding_n
    dims = (n, n, n)
    x = fields.bumps_t(dims, 31, dev)
    torch.cuda.synchronize()
    fbytes = 4 * x.numel()
    rows = []
    for eb in (1e-2, 1e-3):
        recs = []
        for coding in (stz.CODING_HUFFMAN, stz.CODING_ZERO_CHUNKS):
            cfg = stz.config(block=32, coding=coding)
            out = torch.empty(stz.stz_compress_bound(dims, cfg), dtype=torch.uint8, device=dev)
            rec = torch.empty_like(x)
            holder = {}

            def comp():
                holder["c"] = stz.stz_compress(x, stz.EB_REL, eb, cfg, out=out)

            comp()
            t_c = _sync_time(comp, args.steps)
            c = holder["c"]
            inf = stz.stz_info(c)

            def decomp():
                stz.stz_decompress(c, out=rec, info=inf)

            decomp()
            t_d = _sync_time(decomp, args.steps)
            recs.append(rec)
            rows.append({"eb_rel": eb, "coding": "huffman" if coding == 1 else "zero_chunks",
                         "compression_ratio": round(fbytes / c.numel(), 2),
                         "compress_gbps": round(fbytes / t_c / 1e9, 2),
                         "decompress_gbps": round(fbytes / t_d / 1e9, 2)})
        rows[-1]["same_reconstruction"] = bool(
            torch.equal(recs[0].view(torch.int32), recs[1].view(torch.int32)))
    oracle_ok = None
    if oracle_check:
        from oracle import oracle as O
        crop = x[:64, :64, :64].contiguous()
        want = O.compress(crop.cpu().numpy(), O.EB_REL, 1e-2, O.config(block=32))
        oracle_ok = stz.stz_compress(crop, stz.EB_REL, 1e-2,
                                     stz.config(block=32)).cpu().numpy().tobytes() == want
    del x
    torch.cuda.empty_cache()
    stz.stz_trim()
    return {"workload": f"{n}^3 float32 sum of 32 Gaussian bumps + N(0,1e-6) noise, B=32",
            "runs": rows, "oracle_crop_equal": oracle_ok}


def bench_scale(args, dev):
    """4 co-located variables (log-normal density, three velocity components):
    plain per-variable calls vs one batch of 4 jobs, B = 64, rel eb 1e-3."""
    import numpy as np
    import torch

    from paper_2509_01626_amd import fields, stz
    n = args.scale_n
    dims = (n, n, n)
    t0 = time.time()
    xs = [fields.lognormal_t(dims, 2.0, 40, dev)] + \
         [fields.grf_t(dims, 3.0, 41 + i, dev) for i in range(3)]
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(f"[bench] scale: 4 x {n}^3 generated in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    cfg = stz.config(block=64)
    fbytes = 4 * sum(x.numel() for x in xs)
    outs = [torch.empty(stz.stz_compress_bound(dims, cfg), dtype=torch.uint8, device=dev)
            for _ in xs]
    sizes_p = [0] * 4

    def plain_c():
        for i, x in enumerate(xs):
            sizes_p[i] = stz.stz_compress(x, stz.EB_REL, 1e-3, cfg, out=outs[i]).numel()

    plain_c()
    t_pc = _sync_time(plain_c, 2)
    ref = [outs[i][:sizes_p[i]].clone() for i in range(4)]
    jobs = stz.make_jobs(xs, [stz.EB_REL] * 4, [1e-3] * 4, [cfg] * 4, outs)
    report = stz.stz_autotune_batch(jobs)
    print("[bench] scale autotune:\n" + report, file=sys.stderr, flush=True)

    def batch_c():
        st = stz.lib().stz_compress_batch(jobs, 4, stz._stream())
        if st != stz.OK:
            raise stz.StzError(st, "stz_compress_batch")

    batch_c()
    t_bc = _sync_time(batch_c, 2)
    sizes = [jobs[i].out_size for i in range(4)]
    same = sizes == sizes_p and all(torch.equal(outs[i][:sizes[i]], ref[i]) for i in range(4))
    # the batch captured in a HIP graph and replayed into the same buffers
    jobs_g = stz.make_jobs(xs, [stz.EB_REL] * 4, [1e-3] * 4, [cfg] * 4, outs)
    plan_c = stz.BatchPlan(jobs=jobs_g)
    plan_c.run()
    t_gc = _sync_time(plan_c.run, 2)
    same_gc = plan_c.status() == stz.OK and all(
        jobs_g[i].out_size == sizes[i] and torch.equal(outs[i][:sizes[i]], ref[i])
        for i in range(4))
    plan_c.close()
    del ref
    # oracle check on a 256^3 crop of the density (the same B and bound)
    from oracle import oracle as O
    crop = xs[0][:256, :256, :256].contiguous()
    c_crop = stz.stz_compress(crop, stz.EB_REL, 1e-3, cfg)
    want = O.compress(crop.cpu().numpy(), O.EB_REL, 1e-3, O.config(block=64))
    oracle_ok = c_crop.cpu().numpy().tobytes() == want
    oracle_ok = oracle_ok and np.array_equal(
        stz.stz_decompress(c_crop).cpu().numpy().view(np.uint32),
        O.decompress(want).view(np.uint32))
    del crop, c_crop, want
    comps = [outs[i][:sizes[i]] for i in range(4)]
    recon = torch.empty(dims, dtype=torch.float32, device=dev)
    err_ok = True

    def plain_d():
        for c in comps:
            stz.stz_decompress(c, out=recon)

    plain_d()
    t_pd = _sync_time(plain_d, 2)
    for c, x in zip(comps, xs):
        stz.stz_decompress(c, out=recon)
        e = float((recon - x).abs().max())
        err_ok = err_ok and e <= stz.stz_info(c).eb_abs * (1 + 1e-6)
    del xs
    torch.cuda.empty_cache()
    flds = [stz.Field(c) for c in comps]
    outs_d = [torch.empty(dims, dtype=torch.float32, device=dev) for _ in range(4)]
    reqs = stz.make_requests([(f, [0, 0, 0], list(dims), f.info.levels, o)
                              for f, o in zip(flds, outs_d)])

    def batch_d():
        stz.stz_decompress_batch(reqs)

    batch_d()
    t_bd = _sync_time(batch_d, 2)
    stz.stz_decompress(comps[3], out=recon)
    same_d = torch.equal(recon.view(torch.int32), outs_d[3].view(torch.int32))
    outs_d[3].fill_(0)
    plan_d = stz.BatchPlan(reqs=reqs)
    plan_d.run()
    t_gd = _sync_time(plan_d.run, 2)
    same_gd = plan_d.status() == stz.OK and torch.equal(recon.view(torch.int32),
                                                         outs_d[3].view(torch.int32))
    plan_d.close()
    for f in flds:
        f.close()
    res = {
        "workload": f"4 x {n}^3 float32: log-normal density exp(G), G with P(k)~k^-2; "
                    "3 Gaussian random velocity fields with P(k)~k^-3; rel eb 1e-3, B=64",
        "field_gb": round(fbytes / 1e9, 3),
        "compression_ratio": round(fbytes / sum(sizes), 3),
        "compress_gbps": {"plain": round(fbytes / t_pc / 1e9, 2),
                          "batched": round(fbytes / t_bc / 1e9, 2),
                          "graph": round(fbytes / t_gc / 1e9, 2)},
        "decompress_gbps": {"plain": round(fbytes / t_pd / 1e9, 2),
                            "batched": round(fbytes / t_bd / 1e9, 2),
                            "graph": round(fbytes / t_gd / 1e9, 2)},
        "batched_bytes_equal_plain": bool(same), "batched_decode_equal_plain": bool(same_d),
        "graph_bytes_equal_eager": bool(same_gc), "graph_decode_equal_eager": bool(same_gd),
        "oracle_crop_256_equal": bool(oracle_ok),
        "within_bound": bool(err_ok),
        "autotune": [ln for ln in report.splitlines() if "tuned" in ln or "default" in ln],
    }
    del outs, comps, recon, outs_d
    torch.cuda.empty_cache()
    stz.stz_trim()
    return res


def bench_serve(args, dev):
    """Resident compressed 512^3 fields; Poisson decode requests for random
    boxes at random progressive levels; continuous batching vs one request
    per launch."""
    import numpy as np
    import torch

    from paper_2509_01626_amd import fields, serve, stz
    nf = args.serve_fields
    dims = (512, 512, 512)
    cfg = stz.config(block=32)
    comps = []
    buf = torch.empty(stz.stz_compress_bound(dims, cfg), dtype=torch.uint8, device=dev)
    t0 = time.time()
    for i in range(nf):
        x = fields.spectral_t(dims, 5.0 / 3.0, 500 + i, dev)
        c = stz.stz_compress(x, stz.EB_REL, 1e-3, cfg, out=buf)
        comps.append(c.clone())
        del x
    del buf
    torch.cuda.empty_cache()
    print(f"[bench] serve: {nf} fields compressed in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    flds = [stz.Field(c) for c in comps]
    infos = [f.info for f in flds]
    rates = [float(r) for r in args.serve_rates.split(",") if r]
    points = []
    for rate in rates:
        pt = {"offered_rps": rate}
        for mode, slots, mb in (("batched", 2, 64), ("plain", 1, 1)):
            rng = np.random.default_rng(7)
            arr = serve.poisson_arrivals(rng, args.serve_requests, rate, infos)
            srv = serve.Server(flds, arena_bytes=8 << 30, slots=slots, max_batch=mb, device=dev)
            # scratch and staging sized for the largest request before serving
            srv.prewarm(0, 256, infos[0].levels)
            # warm-up requests (not counted)
            srv.run(serve.poisson_arrivals(np.random.default_rng(8), args.serve_warmup, rate,
                                           infos))
            srv.done = []
            srv.batch_sizes = []
            srv.batches = 0
            srv.trace = []
            t = time.perf_counter()
            done = srv.run(arr)
            wall = time.perf_counter() - t
            # the batch that took longest from launch to completion seen
            wb = max(srv.trace, key=lambda e: e[1] - e[0]) if srv.trace else (t, t, 0)
            st = serve.latency_stats(done)
            ok = sum(1 for r in done if r.status == stz.OK)
            pt[mode] = {"completed_rps": round(ok / wall, 1), "p50_ms": st["p50_ms"],
                        "p99_ms": st["p99_ms"], "p999_ms": st["p999_ms"],
                        "max_ms": st["max_ms"], "mean_ms": st["mean_ms"],
                        "launch_batches": srv.batches,
                        "mean_batch": round(sum(srv.batch_sizes) / max(1, len(srv.batch_sizes)),
                                            2),
                        "slowest_batch": {"ms": round((wb[1] - wb[0]) * 1e3, 3), "size": wb[2],
                                          "at_s": round(wb[0] - t, 3)}}
            del srv
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            stz.stz_trim()  # the server's streams are gone: drop their scratch
        print(f"[bench] serve rate {rate}: {pt}", file=sys.stderr, flush=True)
        points.append(pt)
    for f in flds:
        f.close()
    res = {
        "workload": f"{nf} resident compressed 512^3 k^-5/3 spectral fields (rel eb 1e-3, B=32); "
                    "Poisson requests: uniform field, level U{0..5}, box edge per axis U[16,256]",
        "requests_per_load": args.serve_requests,
        "warmup_requests": args.serve_warmup,
        "resident_compressed_gb": round(sum(c.numel() for c in comps) / 1e9, 3),
        "load_points": points,
    }
    del comps, flds
    torch.cuda.empty_cache()
    stz.stz_trim()
    return res


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
