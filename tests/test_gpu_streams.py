"""GPU: the plain calls on a caller's stream. The binding passes the current
torch stream (or an explicit one) to the library; compression and every
decode run there in stream order, with results equal to the default
stream's and the oracle's, also when one stream buffer is decoded on two
streams in turn (kept headers and decoder tables are per device, not per
stream)."""
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


def _bits(t):
    return t.cpu().numpy().view(np.uint32)


def test_calls_on_a_side_stream(gpu, oracle):
    import torch

    from paper_2509_01626_amd import stz
    x = fields.spectral((40, 33, 47), 5 / 3, seed=61)
    want = oracle.compress(x, oracle.EB_REL, 1e-3, oracle.config(block=16))
    xd = torch.from_numpy(x).to(gpu)
    cfg = stz.config(block=16)
    ref = stz.stz_compress(xd, stz.EB_REL, 1e-3, cfg)
    torch.cuda.synchronize()
    assert ref.cpu().numpy().tobytes() == want
    info = stz.stz_info(ref)
    lo, hi = [4, 7, 3], [29, 30, 41]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # the current stream: picked up by the binding
        c1 = stz.stz_compress(xd, stz.EB_REL, 1e-3, cfg)
        f1 = stz.stz_decompress(c1, info=info)
        l1 = stz.stz_decompress_level(c1, info.levels - 1, info=info)
        r1 = stz.stz_decompress_region(c1, lo, hi, info.levels, info=info)
    side.synchronize()
    assert c1.cpu().numpy().tobytes() == want
    assert np.array_equal(_bits(f1), oracle.decompress(want).view(np.uint32))
    assert np.array_equal(_bits(l1), oracle.decompress_level(want, info.levels - 1).view(np.uint32))
    assert np.array_equal(_bits(r1),
                          oracle.decompress_region(want, lo, hi, info.levels).view(np.uint32))
    # an explicit stream argument, and one buffer decoded on two streams in turn
    out = torch.empty(tuple(int(v) for v in info.dims), dtype=torch.float32, device=gpu)
    for k in range(4):
        st = side if k % 2 == 0 else None
        print(f"[streams] decode {k} on {'side' if st is not None else 'current'}", flush=True)
        out.fill_(-1.0)
        if st is not None:
            st.wait_stream(torch.cuda.current_stream())
        got = stz.stz_decompress(c1, out=out, stream=st, info=info)
        if st is not None:
            st.synchronize()
        else:
            torch.cuda.synchronize()
        assert np.array_equal(_bits(got), _bits(f1)), k
