"""GPU ROI selection (Sec. 3.3, flexible scientific workflow) through the C ABI
against the oracle's: identical per-unit statistics and selections for blocks
and slices, max and range, threshold and top fraction; the selected blocks
then decode at full resolution as a batch, equal to the plain region decode."""
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


@pytest.mark.parametrize("unit", [0, 1, 2, 3])
@pytest.mark.parametrize("stat", [0, 1])
def test_roi_matches_oracle(gpu, oracle, unit, stat):
    import torch

    from paper_2509_01626_amd import stz
    x = fields.bumps((45, 38, 52), seed=31, n_bumps=10)
    comp = stz.stz_compress(torch.from_numpy(x).to(gpu), stz.EB_REL, 1e-3, stz.config(block=8))
    host = comp.cpu().numpy().tobytes()
    f = stz.Field(comp)
    print(f"[case] roi unit={unit} stat={stat}", flush=True)
    for level in range(f.info.levels + 1):
        for rule, value in ((1, 0.1), (1, 1.0), (0, None)):
            osel, ost = oracle.roi_select(host, level, unit, stat, rule,
                                          value if value is not None else 0.0)
            if value is None:  # threshold at the oracle's median statistic
                value = float(np.median(ost))
                osel, ost = oracle.roi_select(host, level, unit, stat, rule, value)
            sel, st = stz.stz_roi_select(f, level, unit, stat, rule, value)
            assert np.array_equal(st, ost), (level, rule)
            assert np.array_equal(sel, osel), (level, rule)
    f.close()


def test_roi_blocks_decode_as_batch(gpu, oracle):
    import torch

    from paper_2509_01626_amd import stz
    x = fields.spectral((64, 48, 80), 5 / 3, seed=12)
    comp = stz.stz_compress(torch.from_numpy(x).to(gpu), stz.EB_REL, 1e-3, stz.config(block=16))
    host = comp.cpu().numpy().tobytes()
    f = stz.Field(comp)
    sel, _ = stz.stz_roi_select(f, 2, stz.ROI_BLOCKS, stz.ROI_RANGE, stz.ROI_TOP_FRACTION, 0.25)
    osel, _ = oracle.roi_select(host, 2, stz.ROI_BLOCKS, stz.ROI_RANGE, stz.ROI_TOP_FRACTION, 0.25)
    assert np.array_equal(sel, osel)
    boxes = stz.roi_block_boxes(f.info, sel)
    assert len(boxes) == int(np.ceil(0.25 * 4 * 3 * 5))
    items, outs = [], []
    for lo, hi in boxes:
        o = torch.empty(16 ** 3, dtype=torch.float32, device=gpu)
        outs.append(o)
        items.append((f, lo, hi, f.info.levels, o))
    stz.stz_decompress_batch(stz.make_requests(items))
    torch.cuda.synchronize()
    for (lo, hi), o in zip(boxes, outs):
        want = stz.stz_decompress_region(comp, lo, hi, f.info.levels).reshape(-1)
        assert torch.equal(o[:want.numel()].view(torch.int32), want.view(torch.int32))
        ref = oracle.decompress_region(host, lo, hi, f.info.levels).reshape(-1)
        assert np.array_equal(o[:ref.size].cpu().numpy().view(np.uint32), ref.view(np.uint32))
    f.close()


@pytest.mark.parametrize("dtype,edge", [(np.float32, 128), (np.float64, 128),
                                        (np.float32, 256)])
def test_roi_many_units_ties_and_cache(gpu, oracle, dtype, edge):
    """4096 blocks (one-work-group selection, several compaction chunks of 1024)
    and 32768 blocks (grid-wide digit histograms and chunked compaction), a
    field with a large constant region (many equal statistics: ties go to the
    smaller index), selections repeated from the kept statistics, and a second
    field whose statistics are kept apart."""
    import torch

    from paper_2509_01626_amd import stz
    x = fields.bumps((edge, edge, edge), seed=77, n_bumps=5).astype(dtype)
    x[:, :edge // 2, :] = 1.0
    comp = stz.stz_compress(torch.from_numpy(x).to(gpu), stz.EB_REL, 1e-3, stz.config(block=8))
    host = comp.cpu().numpy().tobytes()
    y = fields.spectral((40, 40, 40), 5 / 3, seed=78).astype(dtype)
    comp2 = stz.stz_compress(torch.from_numpy(y).to(gpu), stz.EB_REL, 1e-3, stz.config(block=8))
    host2 = comp2.cpu().numpy().tobytes()
    f, f2 = stz.Field(comp), stz.Field(comp2)
    L = f.info.levels
    for rep in range(2):
        top = L if edge <= 128 else L - 2   # the oracle decodes this level on the CPU
        for level, stat, rule, value in ((top, 1, 1, 0.3), (top, 1, 1, 0.75), (top, 0, 0, 1.0),
                                         (top - 1, 0, 1, 0.5), (top, 1, 1, 1.0),
                                         (top, 1, 1, 1e-4)):
            print(f"[case] roi many rep={rep} {dtype.__name__} lv={level} stat={stat} "
                  f"rule={rule} value={value}", flush=True)
            osel, ost = oracle.roi_select(host, level, 0, stat, rule, value)
            sel, st = stz.stz_roi_select(f, level, 0, stat, rule, value)
            assert np.array_equal(st, ost)
            assert np.array_equal(sel, osel)
            osel2, _ = oracle.roi_select(host2, level if level <= f2.info.levels else
                                         f2.info.levels, 0, stat, rule, value)
            sel2, _ = stz.stz_roi_select(f2, level if level <= f2.info.levels else
                                         f2.info.levels, 0, stat, rule, value)
            assert np.array_equal(sel2, osel2)
    f.close()
    f2.close()
