"""GPU: plain decodes keep the parsed header of the streams they were given
(per device, stream address and size) and check it on the device before
trusting it. A buffer whose contents change between calls (another stream,
another value type, a corrupted header or payload) must decode exactly as a
call that reads the header first: the oracle's values, or the oracle's
status."""
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


def _put(buf, stream):
    """Copy stream bytes to the front of the device buffer (same address,
    same size for every call)."""
    import torch
    buf.zero_()
    buf[:len(stream)].copy_(torch.frombuffer(bytearray(stream), dtype=torch.uint8))


def _same(a, b):
    return np.array_equal(np.ascontiguousarray(a).view(np.uint8), np.ascontiguousarray(b).view(np.uint8))


def test_streams_swapped_in_one_buffer(gpu, oracle):
    import torch

    from paper_2509_01626_amd import stz
    xa = fields.spectral((33, 28, 41), 5 / 3, seed=11)
    xb = fields.bumps((40, 36, 22), seed=12, n_bumps=5)
    sa = oracle.compress(xa, oracle.EB_REL, 1e-3, oracle.config(block=16))
    sb = oracle.compress(xb, oracle.EB_REL, 1e-2, oracle.config(block=8))
    buf = torch.zeros(max(len(sa), len(sb)) + 64, dtype=torch.uint8, device=gpu)
    lo, hi = [3, 5, 2], [19, 22, 17]
    for rep in range(3):
        for tag, s in (("a", sa), ("b", sb)):
            print(f"[kept] rep {rep} stream {tag}", flush=True)
            _put(buf, s)
            info = stz.stz_info(buf)
            for k in range(2):  # the first call may read the header, the second keeps it
                got = stz.stz_decompress(buf, info=info).cpu().numpy()
                assert _same(got, oracle.decompress(s)), (rep, tag, k)
            L = info.levels
            for lv in (0, L - 1):
                got = stz.stz_decompress_level(buf, lv, info=info).cpu().numpy()
                assert _same(got, oracle.decompress_level(s, lv)), (rep, tag, lv)
            got = stz.stz_decompress_region(buf, lo, hi, L, info=info).cpu().numpy()
            assert _same(got, oracle.decompress_region(s, lo, hi, L)), (rep, tag)


def test_value_type_swapped_in_one_buffer(gpu, oracle):
    import torch

    from paper_2509_01626_amd import stz
    x = fields.spectral((26, 30, 24), 5 / 3, seed=21)
    s32 = oracle.compress(x, oracle.EB_REL, 1e-3, oracle.config(block=8))
    s64 = oracle.compress(x.astype(np.float64), oracle.EB_REL, 1e-3, oracle.config(block=8),
                          dtype=np.float64)
    buf = torch.zeros(max(len(s32), len(s64)) + 16, dtype=torch.uint8, device=gpu)
    for rep in range(2):
        for s, dt in ((s64, torch.float64), (s32, torch.float32)):
            print(f"[kept] rep {rep} value type {dt}", flush=True)
            _put(buf, s)
            info = stz.stz_info(buf)
            for k in range(2):
                out = torch.empty(tuple(int(v) for v in info.dims), dtype=dt, device=gpu)
                got = stz.stz_decompress(buf, out=out, info=info).cpu().numpy()
                assert _same(got, oracle.decompress(s)), (rep, str(dt), k)
            # the other value type's call is rejected, as on a fresh read
            other = torch.float32 if dt == torch.float64 else torch.float64
            assert stz.decode_status(buf, dtype=other) == stz.ERR_ARG


def test_header_and_payload_changes_after_a_kept_decode(gpu, oracle):
    import torch

    from paper_2509_01626_amd import stz
    x = fields.spectral((30, 30, 30), 5 / 3, seed=31)
    s = oracle.compress(x, oracle.EB_REL, 1e-3, oracle.config(block=8))
    ref = oracle.decompress(s)
    buf = torch.zeros(len(s), dtype=torch.uint8, device=gpu)
    rng = np.random.default_rng(5)
    nsym = 2 * 512 + 2
    for i in range(40):
        _put(buf, s)
        for _ in range(2):  # keep the clean header
            assert stz.decode_status(buf) == stz.OK
        c = bytearray(s)
        # alternate flips inside the header (fixed part and code lengths)
        # with flips anywhere in the stream
        k = int(rng.integers(0, min(len(c), 512 + nsym))) if i % 2 == 0 else \
            int(rng.integers(0, len(c)))
        c[k] ^= 1 << int(rng.integers(0, 8))
        print(f"[kept] flip byte {k}", flush=True)
        _put(buf, bytes(c))
        st_gpu = stz.decode_status(buf)
        st_ref = oracle.decode_status(bytes(c))
        assert (st_gpu == stz.OK) == (st_ref == oracle.OK), (k, st_gpu, st_ref)
        if st_gpu == stz.OK:
            got = stz.stz_decompress(buf, info=stz.stz_info(buf)).cpu().numpy()
            assert _same(got, oracle.decompress(bytes(c))), k
    _put(buf, s)
    assert _same(stz.stz_decompress(buf, info=stz.stz_info(buf)).cpu().numpy(), ref)
