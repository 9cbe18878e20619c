"""GPU: the batched compressor and the batched request decoder through the C
ABI. Every job of a batch must produce the same bytes as the plain call (and,
for the small fields checked here, as the CPU oracle); every request of a
batch must produce what the plain region / level decode of the same stream
produces and what the oracle's region decode produces; launch shapes chosen by
the autotuner must not change any output."""
import numpy as np
import pytest

from paper_2509_01626_amd import fields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    from paper_2509_01626_amd import stz
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    stz.lib()
    return torch.device("cuda:0")


def _stz():
    from paper_2509_01626_amd import stz
    return stz


def _uneven_batch(n, seed, lo=8, hi=48):
    """n fields with per-axis extents uniform in [lo, hi], alternating smooth
    bumps and power-law spectra, per-field relative bounds log-uniform in
    [1e-4, 1e-2] and block edges from {4, 8, 16, 32}."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        dims = tuple(int(v) for v in rng.integers(lo, hi + 1, size=3))
        x = fields.bumps(dims, seed=seed + i, n_bumps=6) if i % 2 == 0 else \
            fields.spectral(dims, 5 / 3, seed=seed + i)
        eb = float(10 ** rng.uniform(-4, -2))
        B = int(rng.choice([4, 8, 16, 32]))
        out.append((x, eb, B))
    return out


def _compress_batch(gpu, batch):
    import torch
    stz = _stz()
    xs = [torch.from_numpy(x).to(gpu) for x, _, _ in batch]
    cfgs = [stz.config(block=B) for _, _, B in batch]
    outs = [torch.empty(stz.stz_compress_bound(x.shape, c), dtype=torch.uint8, device=gpu)
            for x, c in zip(xs, cfgs)]
    comps, jobs = stz.stz_compress_batch(xs, [stz.EB_REL] * len(xs), [eb for _, eb, _ in batch],
                                         cfgs, outs)
    torch.cuda.synchronize()
    return xs, cfgs, outs, comps, jobs


def test_batch_compress_matches_plain_and_oracle(gpu, oracle):
    import torch
    stz = _stz()
    batch = _uneven_batch(24, seed=100)
    print(f"[case] batch compress of {len(batch)} fields", flush=True)
    xs, cfgs, outs, comps, jobs = _compress_batch(gpu, batch)
    for i, ((x, eb, B), xd, c, comp) in enumerate(zip(batch, xs, cfgs, comps)):
        assert jobs[i].status == stz.OK
        plain = stz.stz_compress(xd, stz.EB_REL, eb, c).cpu().numpy().tobytes()
        got = comp.cpu().numpy().tobytes()
        assert got == plain, (i, x.shape, B, eb)
        if i < 8:
            want = oracle.compress(x, oracle.EB_REL, eb, oracle.config(block=B))
            assert got == want, (i, x.shape, B, eb)
    torch.cuda.synchronize()


def test_batch_compress_statuses(gpu):
    import torch
    stz = _stz()
    x = torch.from_numpy(fields.spectral((20, 21, 22), 5 / 3, seed=4)).to(gpu)
    bad = x.clone()
    bad[3, 4, 5] = float("nan")
    cfg = stz.config(block=8)
    cap = stz.stz_compress_bound(x.shape, cfg)
    outs = [torch.empty(cap, dtype=torch.uint8, device=gpu) for _ in range(4)]
    outs[2] = torch.empty(64, dtype=torch.uint8, device=gpu)  # too small
    jobs = stz.make_jobs([x, bad, x, x], [stz.EB_REL] * 4, [1e-3, 1e-3, 1e-3, -1.0],
                         [cfg] * 4, outs)
    st = stz.lib().stz_compress_batch(jobs, 4, stz._stream())
    torch.cuda.synchronize()
    assert [jobs[i].status for i in range(4)] == [stz.OK, stz.ERR_NONFINITE, stz.ERR_BUFFER,
                                                  stz.ERR_ARG]
    assert st == stz.ERR_NONFINITE
    ref = stz.stz_compress(x, stz.EB_REL, 1e-3, cfg).cpu().numpy().tobytes()
    assert outs[0][:jobs[0].out_size].cpu().numpy().tobytes() == ref
    assert jobs[2].out_size > 64


def _random_requests(rng, flds, n):
    items = []
    for _ in range(n):
        k = int(rng.integers(0, len(flds)))
        f = flds[k]
        dims = [int(v) for v in f.info.dims]
        lo, hi = [], []
        for d in dims:
            e = int(rng.integers(1, d + 1))
            a = int(rng.integers(0, d - e + 1))
            lo.append(a)
            hi.append(a + e)
        level = int(rng.integers(0, f.info.levels + 1))
        items.append((k, lo, hi, level))
    return items


def test_batch_decode_matches_plain_region_and_oracle(gpu, oracle):
    import torch
    stz = _stz()
    batch = _uneven_batch(10, seed=300, lo=6, hi=40)
    _, _, _, comps, _ = _compress_batch(gpu, batch)
    hosts = [c.cpu().numpy().tobytes() for c in comps]
    flds = [stz.Field(c) for c in comps]
    rng = np.random.default_rng(5)
    reqs = _random_requests(rng, flds, 60)
    # whole-domain requests at every level of two fields, too
    for k in (0, 3):
        for lv in range(flds[k].info.levels + 1):
            reqs.append((k, [0, 0, 0], [int(v) for v in flds[k].info.dims], lv))
    items, outs = [], []
    for k, lo, hi, lv in reqs:
        shp = stz.region_shape(flds[k].info, lo, hi, lv)
        o = torch.full((max(1, shp[0] * shp[1] * shp[2]),), -7.0, dtype=torch.float32,
                       device=gpu)
        outs.append(o)
        items.append((flds[k], lo, hi, lv, o))
    print(f"[case] batch decode of {len(items)} requests", flush=True)
    arr = stz.make_requests(items)
    stz.stz_decompress_batch(arr)
    torch.cuda.synchronize()
    for i, (k, lo, hi, lv) in enumerate(reqs):
        want = stz.stz_decompress_region(comps[k], lo, hi, lv, info=flds[k].info)
        n = want.numel()
        assert tuple(arr[i].out_dims) == tuple(want.shape)
        got = outs[i][:n].cpu().numpy()
        assert np.array_equal(got.view(np.uint32), want.reshape(-1).cpu().numpy().view(np.uint32)), \
            (i, k, lo, hi, lv)
        ref = oracle.decompress_region(hosts[k], lo, hi, lv).reshape(-1)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), ("oracle", i, k, lo, hi, lv)
    for f in flds:
        f.close()


def test_batch_decode_async_flags_and_errors(gpu):
    import torch
    stz = _stz()
    x = torch.from_numpy(fields.bumps((30, 26, 34), seed=8, n_bumps=5)).to(gpu)
    comp = stz.stz_compress(x, stz.EB_REL, 1e-3, stz.config(block=8))
    f = stz.Field(comp)
    good = torch.empty(30 * 26 * 34, dtype=torch.float32, device=gpu)
    small = torch.empty(5, dtype=torch.float32, device=gpu)
    items = [(f, [0, 0, 0], [30, 26, 34], 3, good),
             (f, [0, 0, 0], [30, 26, 34], 3, small),       # buffer too small
             (f, [0, 0, 0], [31, 26, 34], 3, good),        # box outside the field
             (f, [0, 0, 0], [30, 26, 34], 9, good)]        # level above L
    arr = stz.make_requests(items)
    flags = torch.full((4,), 77, dtype=torch.int32, device=gpu)
    st = stz.stz_decompress_batch(arr, flags=flags, check=False)
    torch.cuda.synchronize()
    assert st == stz.ERR_BUFFER
    assert [arr[i].status for i in range(4)] == [stz.OK, stz.ERR_BUFFER, stz.ERR_ARG, stz.ERR_ARG]
    assert flags.cpu().tolist() == [0, 0, 0, 0]
    ref = stz.stz_decompress(comp).reshape(-1)
    assert torch.equal(good.view(torch.int32), ref.view(torch.int32))
    f.close()


def test_batch_decode_reports_corruption(gpu):
    import torch
    stz = _stz()
    x = torch.from_numpy(fields.spectral((32, 32, 32), 5 / 3, seed=9)).to(gpu)
    comp = stz.stz_compress(x, stz.EB_REL, 1e-3, stz.config(block=8))
    bad = comp.clone()
    info = stz.stz_info(comp)
    f_ok = stz.Field(comp)
    f_bad = stz.Field(bad)   # header and code table intact
    # flip payload bits of the finest level after opening (the table is cached)
    tail = bad[-4096:]
    tail ^= 0x5A
    o1 = torch.empty(32 ** 3, dtype=torch.float32, device=gpu)
    o2 = torch.empty(32 ** 3, dtype=torch.float32, device=gpu)
    arr = stz.make_requests([(f_ok, [0, 0, 0], [32, 32, 32], info.levels, o1),
                             (f_bad, [0, 0, 0], [32, 32, 32], info.levels, o2)])
    plain = stz.decode_status(bad, "decompress")
    st = stz.stz_decompress_batch(arr, check=False)
    torch.cuda.synchronize()
    assert arr[0].status == stz.OK
    assert arr[1].status == plain
    assert st == plain
    assert torch.equal(o1.view(torch.int32), stz.stz_decompress(comp).reshape(-1).view(torch.int32))
    f_ok.close()
    f_bad.close()


def test_autotuned_shapes_keep_outputs(gpu):
    import torch
    stz = _stz()
    batch = _uneven_batch(12, seed=700, lo=16, hi=64)
    xs, cfgs, outs, comps, jobs = _compress_batch(gpu, batch)
    before = [c.cpu().numpy().tobytes() for c in comps]
    report = stz.stz_autotune_batch(jobs)
    print(report, flush=True)
    assert "compress tuned" in report and "decode tuned" in report
    # every candidate shape must reproduce the default output exactly
    assert "changed the output" not in report
    comps2, jobs2 = stz.stz_compress_batch(xs, [stz.EB_REL] * len(xs), [eb for _, eb, _ in batch],
                                           cfgs, outs)
    torch.cuda.synchronize()
    assert [c.cpu().numpy().tobytes() for c in comps2] == before
    # decode with the tuned shapes equals the plain decode
    flds = [stz.Field(c) for c in comps2]
    items, outs_d = [], []
    for f, (x, _, _) in zip(flds, batch):
        o = torch.empty(x.size, dtype=torch.float32, device=gpu)
        outs_d.append(o)
        items.append((f, [0, 0, 0], list(x.shape), f.info.levels, o))
    stz.stz_decompress_batch(stz.make_requests(items))
    torch.cuda.synchronize()
    for o, c in zip(outs_d, comps2):
        assert torch.equal(o.view(torch.int32), stz.stz_decompress(c).reshape(-1).view(torch.int32))
    for f in flds:
        f.close()


def test_batch_decode_large_request_direct_path(gpu):
    """A request with many blocks per level takes the plain launch inside the
    batch; results still equal the plain decoder's."""
    import torch
    stz = _stz()
    xa = torch.from_numpy(fields.spectral((128, 96, 80), 5 / 3, seed=21)).to(gpu)  # 1920 blocks
    xb = torch.from_numpy(fields.bumps((20, 30, 40), seed=22, n_bumps=4)).to(gpu)
    ca = stz.stz_compress(xa, stz.EB_REL, 1e-3, stz.config(block=8))
    cb = stz.stz_compress(xb, stz.EB_REL, 1e-3, stz.config(block=8))
    fa, fb = stz.Field(ca), stz.Field(cb)
    oa = torch.empty(xa.numel(), dtype=torch.float32, device=gpu)
    ob = torch.empty(xb.numel(), dtype=torch.float32, device=gpu)
    oc = torch.empty(xa.numel(), dtype=torch.float32, device=gpu)
    lo, hi = [3, 5, 7], [120, 90, 77]
    arr = stz.make_requests([(fa, [0, 0, 0], [128, 96, 80], 3, oa),
                             (fb, [0, 0, 0], [20, 30, 40], 3, ob),
                             (fa, lo, hi, 3, oc)])
    print("[case] direct-path batch", flush=True)
    stz.stz_decompress_batch(arr)
    torch.cuda.synchronize()
    assert torch.equal(oa.view(torch.int32), stz.stz_decompress(ca).reshape(-1).view(torch.int32))
    assert torch.equal(ob.view(torch.int32), stz.stz_decompress(cb).reshape(-1).view(torch.int32))
    want = stz.stz_decompress_region(ca, lo, hi, 3).reshape(-1)
    assert torch.equal(oc[:want.numel()].view(torch.int32), want.view(torch.int32))
    fa.close()
    fb.close()


def test_batch_with_large_job_matches_plain_and_oracle(gpu, oracle):
    """A job with 1331 blocks of 32^3 points at its finest level runs that
    level's predictor as a plain launch inside the batch (interior and shell
    kernels); its bytes and its neighbours' must equal the plain calls' and
    the oracle's."""
    import torch

    from paper_2509_01626_amd import stz
    big = fields.spectral((336, 336, 336), 5 / 3, seed=61)
    small = [fields.bumps((40, 33, 50), seed=62, n_bumps=4), fields.spectral((70, 64, 96), 5 / 3,
                                                                              seed=63)]
    xs = [big] + small
    ebs = [1e-3, 1e-2, 1e-4]
    cfgs = [stz.config(block=32)] * 3
    xds = [torch.from_numpy(x).to(gpu) for x in xs]
    outs = [torch.empty(stz.stz_compress_bound(x.shape, c), dtype=torch.uint8, device=gpu)
            for x, c in zip(xds, cfgs)]
    print("[case] batch with a 336^3 job", flush=True)
    comps, jobs = stz.stz_compress_batch(xds, [stz.EB_REL] * 3, ebs, cfgs, outs)
    torch.cuda.synchronize()
    for i in range(3):
        assert jobs[i].status == stz.OK
        got = comps[i].cpu().numpy().tobytes()
        plain = stz.stz_compress(xds[i], stz.EB_REL, ebs[i], cfgs[i]).cpu().numpy().tobytes()
        assert got == plain, i
        want = oracle.compress(xs[i], oracle.EB_REL, ebs[i], oracle.config(block=32))
        assert got == want, i


def test_batch_with_whole_gpu_job_matches_plain(gpu):
    """A job of 512^3 values fills the GPU by itself and runs its plain launch
    sequence inside the batch, eager and captured; its bytes and its small
    neighbours' equal the plain calls' (the plain 512^3 compression equals
    the oracle's in the full-size tests)."""
    import torch

    from paper_2509_01626_amd import stz
    big = fields.spectral_t((512, 512, 512), 5 / 3, 5, gpu)
    small = [torch.from_numpy(fields.bumps((40, 33, 50), seed=72, n_bumps=4)).to(gpu),
             torch.from_numpy(fields.spectral((70, 64, 96), 5 / 3, seed=73)).to(gpu)]
    xds = [big] + small
    ebs = [1e-3, 1e-2, 1e-4]
    cfgs = [stz.config(block=32)] * 3
    plain = [stz.stz_compress(x, stz.EB_REL, eb, c).cpu().numpy().tobytes()
             for x, eb, c in zip(xds, ebs, cfgs)]
    outs = [torch.empty(stz.stz_compress_bound(x.shape, c), dtype=torch.uint8, device=gpu)
            for x, c in zip(xds, cfgs)]
    print("[case] batch with a 512^3 job", flush=True)
    comps, jobs = stz.stz_compress_batch(xds, [stz.EB_REL] * 3, ebs, cfgs, outs)
    torch.cuda.synchronize()
    for i in range(3):
        assert jobs[i].status == stz.OK
        assert comps[i].cpu().numpy().tobytes() == plain[i], i
    outs_g = [torch.zeros_like(o) for o in outs]
    jobs_g = stz.make_jobs(xds, [stz.EB_REL] * 3, ebs, cfgs, outs_g)
    plan = stz.BatchPlan(jobs=jobs_g)
    for rep in range(2):
        print(f"[case] 512^3 job, captured replay {rep}", flush=True)
        plan.run()
        assert plan.status() == stz.OK
        torch.cuda.synchronize()
        for i in range(3):
            assert outs_g[i][:jobs_g[i].out_size].cpu().numpy().tobytes() == plain[i], (rep, i)
    plan.close()
