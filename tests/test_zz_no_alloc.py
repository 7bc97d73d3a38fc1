"""ubqp_screen_noalloc (the screen whose partials live in the library's static
device scratch) against ubqp_screen, through the C ABI: bit-exact on two calls in
a row, the second with fewer candidates, so the second call runs over a scratch
still holding the first call's partials; sizes beyond the scratch are rejected
with nothing launched."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1706_00037_amd import ubqp
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return ubqp.Context(0)


def _both(ctx, f_host, lam):
    M = f_host.shape[0]
    f = torch.from_numpy(f_host).cuda()
    out = []
    for name in ("screen", "screen_noalloc"):
        idx = torch.full((M,), -7, dtype=torch.int32, device="cuda")
        npass = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        sm = torch.full((2,), -1, dtype=torch.int64, device="cuda")
        getattr(ctx, name)(f, lam[0], lam[1], idx, npass, sm)
        torch.cuda.synchronize()
        out.append((idx.cpu().numpy(), int(npass.item()), sm.cpu().numpy()))
    return out


@pytest.mark.parametrize("sizes", [(4_000_003, 5000), (100_003, 2049), (2048, 1)])
@pytest.mark.parametrize("lam", [(1, 2), (3, 10)])
def test_noalloc_screen_equals_screen_twice(ctx, sizes, lam):
    rng = np.random.default_rng(sizes[0] + lam[0])
    for M in sizes:                              # second call smaller than the first
        f = rng.integers(-10**9, 10**9, size=M, dtype=np.int64)
        (i0, p0, s0), (i1, p1, s1) = _both(ctx, f, lam)
        assert p0 == p1 and p0 >= 0, M
        assert np.array_equal(s0, s1), M
        assert np.array_equal(i0[:p0], i1[:p1]), M
        assert (i1[p1:] == -7).all(), M          # nothing written past the passers


def test_noalloc_screen_rejects_beyond_its_scratch(ctx):
    from paper_1706_00037_amd import ubqp
    L = ubqp.load()
    M = ubqp.UBQP_SCREEN_NOALLOC_MAX_M + 1
    f = torch.zeros(8, dtype=torch.int64, device="cuda")
    idx = torch.zeros(8, dtype=torch.int32, device="cuda")
    npass = torch.full((1,), -5, dtype=torch.int64, device="cuda")
    sm = torch.zeros(2, dtype=torch.int64, device="cuda")
    P = ctypes.c_void_p
    rc = L.ubqp_screen_noalloc(ctx.h, P(f.data_ptr()), M, 1, 2, P(idx.data_ptr()), P(npass.data_ptr()),
                               P(sm.data_ptr()))
    assert rc == ubqp.UBQP_EINVAL
    assert b"static screen scratch" in L.ubqp_last_error(ctx.h)
    torch.cuda.synchronize()
    assert int(npass.item()) == -5                # nothing was launched
