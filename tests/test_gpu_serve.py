"""GPU: the continuous-batching decode server. Requests arriving while other
batches are on the device are admitted as arena memory frees up and decoded
in shared launches; every result must be bit-identical to decoding the same
request alone with the plain region decoder."""
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


def test_mix_equals_alone(gpu):
    import torch

    from paper_2509_01626_amd import serve, stz
    shapes = [(48, 40, 56), (33, 64, 20), (64, 64, 64)]
    comps, flds = [], []
    for i, shp in enumerate(shapes):
        x = torch.from_numpy(fields.spectral(shp, 5 / 3, seed=40 + i)).to(gpu)
        c = stz.stz_compress(x, stz.EB_REL, 1e-3, stz.config(block=16 if i != 1 else 8))
        comps.append(c)
        flds.append(stz.Field(c))
    rng = np.random.default_rng(11)
    arrivals = serve.poisson_arrivals(rng, 300, rate=20000.0,
                                      fields_info=[f.info for f in flds], edge=(4, 64))
    results = {}

    def keep(r, view):
        results[r.rid] = view.clone()

    # A small arena (1 MiB) forces requests to wait for memory.
    srv = serve.Server(flds, arena_bytes=1 << 20, slots=2, max_batch=16, device=gpu,
                       on_done=keep)
    print(f"[case] serve {len(arrivals)} requests", flush=True)
    done = srv.run(arrivals)
    torch.cuda.synchronize()
    assert len(done) == len(arrivals)
    assert all(r.status == stz.OK for r in done)
    assert srv.batches < len(arrivals)          # requests shared launches
    assert max(srv.batch_sizes) > 1
    for r in done:
        t, k, lo, hi, lv = arrivals[r.rid]
        alone = stz.stz_decompress_region(comps[k], lo, hi, lv, info=flds[k].info)
        got = results[r.rid]
        assert tuple(got.shape) == tuple(alone.shape), r.rid
        assert torch.equal(got.view(torch.int32), alone.view(torch.int32)), (r.rid, k, lo, hi, lv)
    st = serve.latency_stats(done)
    assert st["p50_ms"] is not None and st["p99_ms"] >= st["p50_ms"]
    for f in flds:
        f.close()


def test_oversized_request_rejected(gpu):
    import torch

    from paper_2509_01626_amd import serve, stz
    x = torch.from_numpy(fields.bumps((64, 64, 64), seed=3, n_bumps=4)).to(gpu)
    c = stz.stz_compress(x, stz.EB_REL, 1e-3, stz.config(block=16))
    f = stz.Field(c)
    srv = serve.Server([f], arena_bytes=1 << 16, slots=1, max_batch=4, device=gpu)
    done = srv.run([(0.0, 0, [0, 0, 0], [64, 64, 64], 4), (0.0, 0, [0, 0, 0], [8, 8, 8], 4)])
    st = {r.rid: r.status for r in done}
    assert st[0] == stz.ERR_NOMEM and st[1] == stz.OK
    f.close()
