"""GPU parity on 2-D fields (nz = 1): bytes, full, progressive and region
decodes equal the oracle's, for several plane sizes, blocks and bounds."""
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


@pytest.mark.parametrize("shape,B", [((1, 256, 256), 32), ((1, 100, 73), 16), ((1, 513, 31), 8)])
@pytest.mark.parametrize("eb", [1e-2, 1e-4])
def test_2d_matches_oracle(gpu, oracle, shape, B, eb):
    import torch

    from paper_2509_01626_amd import stz
    print(f"[case] 2d {shape} B={B} eb={eb}", flush=True)
    x = fields.spectral(shape, 5 / 3, seed=shape[1] + B)
    comp = stz.stz_compress(torch.from_numpy(x).to(gpu), stz.EB_REL, eb, stz.config(block=B))
    want = oracle.compress(x, oracle.EB_REL, eb, oracle.config(block=B))
    assert comp.cpu().numpy().tobytes() == want
    inf = stz.stz_info(comp)
    full = stz.stz_decompress(comp).cpu().numpy()
    assert np.array_equal(full.view(np.uint32), oracle.decompress(want).view(np.uint32))
    for lv in range(inf.levels + 1):
        g = stz.stz_decompress_level(comp, lv, info=inf).cpu().numpy()
        assert np.array_equal(g, oracle.decompress_level(want, lv))
    lo, hi = [0, shape[1] // 3, 5], [1, shape[1] // 3 + 17, min(shape[2], 29)]
    r = stz.stz_decompress_region(comp, lo, hi, inf.levels, info=inf).cpu().numpy()
    assert np.array_equal(r, oracle.decompress_region(want, lo, hi, inf.levels))
