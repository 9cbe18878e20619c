"""GPU parity at the benchmark's full size and launch configuration: the 512^3
k^-5/3 spectral field, 32^3 blocks, relative bounds 1e-2, 1e-3 and 1e-4.
Compressed bytes and the full reconstruction must equal the CPU oracle's bit
for bit; progressive levels and a region are checked against the full
reconstruction (properties that hold at any size)."""
import numpy as np
import pytest

from paper_2509_01626_amd import fields

pytestmark = pytest.mark.gpu

N = 512


@pytest.fixture(scope="module")
def field512():
    import torch

    from paper_2509_01626_amd import stz
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    stz.lib()
    x = fields.spectral((N, N, N), 5.0 / 3.0, seed=2)
    return x, torch.from_numpy(x).to("cuda:0")


@pytest.mark.parametrize("eb", [1e-2, 1e-3, 1e-4])
def test_512cube_matches_oracle(field512, oracle, eb):
    import torch

    from paper_2509_01626_amd import stz
    x, xd = field512
    print(f"[case] 512^3 spectral rel eb {eb}", flush=True)
    cfg = stz.config(block=32)
    comp = stz.stz_compress(xd, stz.EB_REL, eb, cfg)
    got = comp.cpu().numpy().tobytes()
    want = oracle.compress(x, oracle.EB_REL, eb, oracle.config(block=32))
    assert len(got) == len(want)
    assert got == want
    full = stz.stz_decompress(comp)
    ref = oracle.decompress(want)
    fh = full.cpu().numpy()
    assert np.array_equal(fh.view(np.uint32), ref.view(np.uint32))
    info = stz.stz_info(comp)
    err = float(np.abs(fh.astype(np.float64) - x.astype(np.float64)).max())
    assert err <= info.eb_abs
    for lv in range(info.levels):
        s = 1 << (info.levels - lv)
        g = stz.stz_decompress_level(comp, lv, info=info)
        assert torch.equal(g, full[::s, ::s, ::s].contiguous()), lv
    # a small box, and one of 3360 blocks off the origin that holds interior
    # and boundary blocks (the decoder takes those in separate kernels)
    for lo, hi in (([100, 37, 250], [229, 300, 262]), ([20, 40, 33], [500, 470, 490])):
        r = stz.stz_decompress_region(comp, lo, hi, info.levels, info=info)
        assert torch.equal(r, full[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]].contiguous()), (lo, hi)
    torch.cuda.synchronize()
