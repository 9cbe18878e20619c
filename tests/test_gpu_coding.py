"""GPU parity of the entropy-coding stages: Huffman only and zero chunks
(the default). Smooth fields make most chunks all-centre, so the zero-chunk
token dominates; streams must equal the oracle's byte for byte for every
block size (lane packer for small blocks, chunked unit packer for 32^3 and
64^3 blocks, partial edge blocks with any M_y), and both codings must
reconstruct the same values."""
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


CASES = [
    ((64, 64, 64), 16, 1e-2),
    ((70, 45, 101), 32, 1e-2),
    ((45, 70, 131), 64, 1e-3),
    ((33, 29, 40), 8, 1e-2),
    ((1, 200, 150), 32, 1e-3),
    ((20, 21, 22), 4, 1e-2),
]


@pytest.mark.parametrize("shape,B,eb", CASES)
@pytest.mark.parametrize("coding", [1, 2])
def test_coding_matches_oracle(gpu, oracle, shape, B, eb, coding):
    import torch

    from paper_2509_01626_amd import stz
    print(f"[case] coding={coding} {shape} B={B} eb={eb}", flush=True)
    x = fields.bumps(shape, seed=sum(shape) + B, n_bumps=8)
    comp = stz.stz_compress(torch.from_numpy(x).to(gpu), stz.EB_REL, eb,
                            stz.config(block=B, coding=coding))
    want = oracle.compress(x, oracle.EB_REL, eb, oracle.config(block=B, coding=coding))
    got = comp.cpu().numpy().tobytes()
    assert len(got) == len(want)
    assert got == want
    inf = stz.stz_info(comp)
    assert inf.coding == coding
    full = stz.stz_decompress(comp, info=inf).cpu().numpy()
    assert np.array_equal(full.view(np.uint32), oracle.decompress(want).view(np.uint32))
    for lv in range(inf.levels + 1):
        g = stz.stz_decompress_level(comp, lv, info=inf).cpu().numpy()
        assert np.array_equal(g, oracle.decompress_level(want, lv))
    rng = np.random.default_rng(B + coding)
    for _ in range(3):
        lo = [int(rng.integers(0, n)) for n in shape]
        hi = [int(rng.integers(a + 1, n + 1)) for a, n in zip(lo, shape)]
        lv = int(rng.integers(0, inf.levels + 1))
        r = stz.stz_decompress_region(comp, lo, hi, lv, info=inf).cpu().numpy()
        assert np.array_equal(r, oracle.decompress_region(want, lo, hi, lv)), (lo, hi, lv)


def test_zero_chunks_are_lossless_and_smaller(gpu):
    import torch

    from paper_2509_01626_amd import stz
    x = torch.from_numpy(fields.bumps((96, 96, 96), seed=4, n_bumps=16)).to(gpu)
    a = stz.stz_compress(x, stz.EB_REL, 1e-2, stz.config(coding=stz.CODING_HUFFMAN))
    b = stz.stz_compress(x, stz.EB_REL, 1e-2, stz.config())
    assert stz.stz_info(b).coding == stz.CODING_ZERO_CHUNKS
    assert b.numel() < a.numel() / 2
    assert torch.equal(stz.stz_decompress(a).view(torch.int32),
                       stz.stz_decompress(b).view(torch.int32))


def test_batch_with_both_codings(gpu, oracle):
    """A batch mixing the two codings: every job equals the plain call and a
    sample equals the oracle."""
    import torch

    from paper_2509_01626_amd import stz
    shapes = [(40, 50, 60), (33, 33, 33), (64, 20, 70), (17, 90, 31)]
    xs = [torch.from_numpy(fields.bumps(s, seed=i, n_bumps=6)).to(gpu)
          for i, s in enumerate(shapes)]
    cfgs = [stz.config(block=16, coding=1 + (i & 1)) for i in range(len(xs))]
    outs = [torch.empty(stz.stz_compress_bound(x.shape, c), dtype=torch.uint8, device=gpu)
            for x, c in zip(xs, cfgs)]
    views, _ = stz.stz_compress_batch(xs, [stz.EB_REL] * 4, [1e-2] * 4, cfgs, outs)
    for i, x in enumerate(xs):
        ref = stz.stz_compress(x, stz.EB_REL, 1e-2, cfgs[i])
        assert torch.equal(views[i], ref)
    want = oracle.compress(xs[1].cpu().numpy(), oracle.EB_REL, 1e-2,
                           oracle.config(block=16, coding=2))
    assert views[1].cpu().numpy().tobytes() == want


def test_corrupt_zero_chunk_streams_match_oracle_status(gpu, oracle):
    """Bit flips in the payload of a stream full of zero-chunk tokens: the GPU
    decoder reports corruption exactly when the oracle does (a token that is
    not at a chunk's first row included), and equal values otherwise."""
    import torch

    from paper_2509_01626_amd import stz
    x = fields.bumps((24, 24, 24), seed=3, n_bumps=4)
    want = oracle.compress(x, oracle.EB_REL, 1e-2, oracle.config(block=8))
    assert oracle.info(want).coding == 2
    rng = np.random.default_rng(5)
    payload_from = len(want) // 3
    for i in range(60):
        c = bytearray(want)
        k = int(rng.integers(payload_from, len(c)))
        c[k] ^= 1 << int(rng.integers(0, 8))
        print(f"[corrupt] byte {k}", flush=True)
        d = torch.frombuffer(bytearray(c), dtype=torch.uint8).to(gpu)
        st_gpu = stz.decode_status(d)
        st_ref = oracle.decode_status(bytes(c))
        assert (st_gpu == stz.OK) == (st_ref == oracle.OK), (k, st_gpu, st_ref)
        if st_ref == oracle.OK:
            got = stz.stz_decompress(d).cpu().numpy()
            assert np.array_equal(got.view(np.uint32), oracle.decompress(bytes(c)).view(np.uint32))
