"""The measurement entry point: the sustained int8 matrix-core rate."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_mfma_peak_is_plausible():
    from paper_1706_00037_amd import ubqp
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = ubqp.Context(0)
    tops = ctx.mfma_peak()
    # a single compute unit at 2.4 GHz already exceeds 10 TOP/s; the published dense
    # int8 peak of the whole device is 5000 TOP/s
    assert 10.0 < tops < 5500.0, tops


def test_read_peak_levels_are_ordered():
    """Streaming reads from a buffer that each XCD's L2 holds are faster than from
    one that only the Infinity Cache holds, and those faster than HBM streaming;
    HBM streaming stays below the published 8 TB/s."""
    from paper_1706_00037_amd import ubqp
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = ubqp.Context(0)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    l2 = ctx.read_peak(2 << 20, 2 << 20, 4 << 20)
    mall = ctx.read_peak(128 << 20, 64 << 10, 1 << 20)
    hbm = ctx.read_peak(8 * cus * (2 << 20), 2 << 20, 2 << 20)
    assert 100.0 < hbm < 8000.0, hbm
    assert l2 > mall > hbm, (l2, mall, hbm)
    with pytest.raises(ubqp.UbqpError):
        ctx.read_peak(1000, 1000, 1 << 15)
    with pytest.raises(ubqp.UbqpError):
        ctx.read_peak(2 << 20, 3 << 12, 1 << 15)      # a window that does not divide the buffer
