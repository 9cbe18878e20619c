"""GPU: the allocation-free region decode (stz_decompress_region_noalloc)
through the C ABI against the allocating stz_decompress_region, bit for bit,
on two calls in a row (the second with a smaller stream and box, so stale
contents of the shared scratch from the first call must not leak into it),
plus full-field and progressive-level boxes, a corrupt stream, the value-type
check and the scratch-size limit."""
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


def _both(stz, torch, gpu, comp, lo, hi, level):
    want = stz.stz_decompress_region(comp, lo, hi, level)
    out = torch.full((want.numel() + 37,), -3.0, dtype=torch.float32, device=gpu)
    print(f"[noalloc] lo={lo} hi={hi} level={level}", flush=True)
    st, od = stz.stz_decompress_region_noalloc(comp, lo, hi, level, out)
    torch.cuda.synchronize()
    assert st == stz.OK, st
    assert od == tuple(want.shape)
    got = out[:want.numel()]
    assert torch.equal(got.view(torch.int32), want.reshape(-1).view(torch.int32))
    assert bool((out[want.numel():] == -3.0).all())


def test_noalloc_region_matches_region(gpu):
    import torch

    from paper_2509_01626_amd import stz
    big = torch.from_numpy(fields.spectral((160, 144, 176), 5 / 3, seed=61)).to(gpu)
    small = torch.from_numpy(fields.bumps((40, 36, 52), seed=62, n_bumps=8)).to(gpu)
    cb = stz.stz_compress(big, stz.EB_REL, 1e-3, stz.config(block=32))
    cs = stz.stz_compress(small, stz.EB_REL, 1e-2, stz.config(block=8))
    # first call: a large box of the large field; second: a smaller stream
    _both(stz, torch, gpu, cb, [3, 10, 20], [150, 140, 170], 5)
    _both(stz, torch, gpu, cs, [5, 1, 7], [30, 20, 40], 3)
    # whole fields and progressive levels, alternating sizes
    _both(stz, torch, gpu, cb, [0, 0, 0], [160, 144, 176], 5)
    _both(stz, torch, gpu, cs, [0, 0, 0], [40, 36, 52], 2)
    _both(stz, torch, gpu, cb, [64, 0, 100], [65, 144, 101], 4)
    _both(stz, torch, gpu, cs, [39, 35, 51], [40, 36, 52], 3)
    rng = np.random.default_rng(3)
    for _ in range(6):
        lo = [int(rng.integers(0, n)) for n in (160, 144, 176)]
        hi = [int(rng.integers(a + 1, n + 1)) for a, n in zip(lo, (160, 144, 176))]
        _both(stz, torch, gpu, cb, lo, hi, int(rng.integers(0, 6)))


def test_noalloc_errors(gpu):
    import torch

    from paper_2509_01626_amd import stz
    x = torch.from_numpy(fields.spectral((48, 40, 36), 5 / 3, seed=63)).to(gpu)
    comp = stz.stz_compress(x, stz.EB_REL, 1e-3, stz.config(block=16))
    out = torch.empty(48 * 40 * 36, dtype=torch.float32, device=gpu)
    # box outside the field, level above L, buffer too small
    assert stz.stz_decompress_region_noalloc(comp, [0, 0, 0], [49, 40, 36], 4, out)[0] == \
        stz.ERR_ARG
    assert stz.stz_decompress_region_noalloc(comp, [0, 0, 0], [48, 40, 36], 5, out)[0] == \
        stz.ERR_ARG
    assert stz.stz_decompress_region_noalloc(comp, [0, 0, 0], [48, 40, 36], 4, out[:10])[0] == \
        stz.ERR_BUFFER
    # a corrupt payload gives the same status as the allocating decoder
    bad = comp.clone()
    bad[-2048:] ^= 0x3C
    want = stz.decode_status(bad, "region", 4, (0, 0, 0), (48, 40, 36))
    assert want == stz.ERR_CORRUPT
    assert stz.stz_decompress_region_noalloc(bad, [0, 0, 0], [48, 40, 36], 4, out)[0] == want
    # float64 streams are rejected
    c64 = stz.stz_compress(x.double(), stz.EB_REL, 1e-3, stz.config(block=16))
    assert stz.stz_decompress_region_noalloc(c64, [0, 0, 0], [8, 8, 8], 4, out)[0] == stz.ERR_ARG
    # still correct after the failures
    _both(stz, torch, gpu, comp, [1, 2, 3], [47, 39, 35], 4)


def test_noalloc_scratch_limit(gpu):
    """A decode whose cone grids exceed the fixed scratch is refused; a box
    of the same stream that fits decodes exactly."""
    import torch

    from paper_2509_01626_amd import stz
    n = 512  # level-4 grid 256^3 * 4 B = 67 MB > 64 MiB
    x = torch.zeros((n, n, n), dtype=torch.float32, device=gpu)
    x[::7, ::5, ::3] = 1.0
    comp = stz.stz_compress(x, stz.EB_ABS, 0.25, stz.config(block=32))
    out = torch.empty(n * n * n, dtype=torch.float32, device=gpu)
    st, _ = stz.stz_decompress_region_noalloc(comp, [0, 0, 0], [n, n, n], 5, out)
    assert st == stz.ERR_NOMEM
    del out
    _both(stz, torch, gpu, comp, [100, 37, 250], [229, 300, 262], 5)
    _both(stz, torch, gpu, comp, [0, 0, 0], [n, n, n], 4)
