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
