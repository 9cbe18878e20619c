"""Host logic of the decode server: the arena allocator, arrival generation
and latency percentiles (no GPU)."""
import numpy as np

from paper_2509_01626_amd import serve


def test_arena_first_fit_and_merge():
    a = serve.Arena(64 * 10, "cpu")
    x = a.alloc(100)      # 2 granules
    y = a.alloc(64)       # 1 granule
    z = a.alloc(64 * 7)   # the rest
    assert x == (0, 128) and y == (128, 64) and z == (192, 448)
    assert a.alloc(1) is None
    a.release(*y)
    assert a.alloc(65) is None       # one free granule only
    a.release(*x)
    assert a.free == [(0, 192)]      # merged
    a.release(*z)
    assert a.free == [(0, 640)]


class _Info:
    def __init__(self, dims, levels):
        self.dims = dims
        self.levels = levels


def test_poisson_arrivals_shape():
    rng = np.random.default_rng(0)
    arr = serve.poisson_arrivals(rng, 2000, rate=100.0,
                                 fields_info=[_Info((512, 512, 512), 5), _Info((40, 30, 20), 3)])
    ts = [a[0] for a in arr]
    assert ts == sorted(ts)
    gaps = np.diff([0.0] + ts)
    assert abs(gaps.mean() - 0.01) < 0.002           # mean inter-arrival 1/rate
    for t, k, lo, hi, lv in arr:
        dims = (512, 512, 512) if k == 0 else (40, 30, 20)
        for d in range(3):
            assert 0 <= lo[d] < hi[d] <= dims[d]
            assert hi[d] - lo[d] >= min(16, dims[d])
        assert 0 <= lv <= (5 if k == 0 else 3)


class _R:
    def __init__(self, a, d):
        self.t_arrive, self.t_done, self.status = a, d, 0


def test_latency_percentiles():
    done = [_R(0.0, i / 1000.0) for i in range(1, 101)]
    st = serve.latency_stats(done)
    assert st["p50_ms"] == 51.0 or st["p50_ms"] == 50.0
    assert st["p99_ms"] == 99.0
    assert st["p999_ms"] == 100.0 and st["max_ms"] == 100.0
