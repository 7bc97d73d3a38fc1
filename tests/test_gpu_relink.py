"""Parity of path relinking (ubqp_relink through the C ABI) with the oracle's
orc_relink_many: every path's steps, intermediate value, polished value and
final row, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1706_00037_amd.inputs import make_instance, pack_bits, random_candidates, unpack_bits

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ub():
    from paper_1706_00037_amd import ubqp
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return ubqp


@pytest.fixture(scope="module")
def ctx(ub):
    return ub.Context(0)


def _elite(n, E, seed):
    X = random_candidates(E, n, seed)
    if E >= 4:
        X[2] = X[0]                                           # identical: no intermediate
        X[3] = pack_bits((1 - unpack_bits(X[1], n))[None, :])[0]   # the complement: |D| = n
    return X


def _check(ctx, Q, elite, mf=0, pairs_idx=None):
    prob = ctx.problem(Q)
    r = ctx.relink_elite(prob, elite, max_flips=mf)
    pairs = r["pairs"]
    sel = np.arange(len(pairs)) if pairs_idx is None else np.asarray(pairs_idx)
    o = oracle.relink_many(Q, elite, pairs[sel], max_flips=mf, threads=8)
    assert np.array_equal(r["steps"][sel], o["steps"])
    assert np.array_equal(r["f_mid"][sel], o["f_mid"])
    assert np.array_equal(r["f_out"][sel], o["f_out"])
    assert np.array_equal(r["X"][sel], o["X"])
    return r


@pytest.mark.parametrize("n,d,lo,hi,E,mf", [
    (1, 1.0, -100, 100, 3, 0),
    (2, 1.0, -100, 100, 4, 0),
    (63, 0.5, -128, 127, 6, 0),
    (130, 0.3, -100, 100, 6, 0),
    (300, 0.5, -32768, 32767, 5, 0),        # two planes
    (257, 0.2, -100, 100, 5, 4),            # capped ascent after the walk
    (1100, 0.3, -100, 100, 5, 0),
    (4500, 0.1, -30000, 30000, 4, 0),       # two planes, five column blocks
])
def test_relink_matches_oracle(ctx, n, d, lo, hi, E, mf):
    Q = make_instance(n, d, lo, hi, 8800 + n)
    _check(ctx, Q, _elite(n, E, 90 + n), mf)


def test_relink_more_paths_than_one_chunk(ctx):
    """71 elite rows: 4970 ordered pairs, more than one chunk of 4096 paths."""
    n = 100
    Q = make_instance(n, 0.5, -100, 100, 5)
    _check(ctx, Q, _elite(n, 71, 6))


@pytest.mark.parametrize("n,lo,hi,d", [(7000, -100, 100, 0.5), (8192, -32768, 32767, 0.1)])
def test_relink_largest_shapes_sampled(ctx, n, lo, hi, d):
    """The headline size (seven column blocks) and the largest n with two planes
    (eight blocks): a sample of the paths against the oracle."""
    Q = make_instance(n, d, lo, hi, 77)
    E = 6
    r = _check(ctx, Q, _elite(n, E, 78), pairs_idx=[0, 5, 6, 11, 17, 29])
    assert (r["f_out"][r["steps"] > 0] >= r["f_mid"][r["steps"] > 0]).all()


@pytest.mark.parametrize("P,lo,hi", [(512, -100, 100), (513, -100, 100), (300, -32768, 32767)])
def test_relink_team_threshold(ctx, P, lo, hi):
    """At most 512 paths with n_pad > 3072 are walked by teams of four waves, more
    by one wave each; both give the oracle's steps, values and rows."""
    n = 3100
    Q = make_instance(n, 0.2, lo, hi, 8900 + P)
    elite = _elite(n, 24, 8901)
    pairs = np.array([(a, b) for a in range(24) for b in range(24) if a != b], np.int32)[:P]
    prob = ctx.problem(Q)
    X = torch.empty((P, prob.W), dtype=torch.int64, device="cuda")
    fm = torch.empty(P, dtype=torch.int64, device="cuda")
    fo = torch.empty(P, dtype=torch.int64, device="cuda")
    st = torch.empty(P, dtype=torch.int32, device="cuda")
    ctx.relink(prob, torch.from_numpy(elite.view(np.int64)).cuda(), torch.from_numpy(pairs).cuda(), X, fm, fo, st)
    ctx.sync()
    o = oracle.relink_many(Q, elite, pairs, threads=8)
    assert np.array_equal(st.cpu().numpy(), o["steps"])
    assert np.array_equal(fm.cpu().numpy(), o["f_mid"])
    assert np.array_equal(fo.cpu().numpy(), o["f_out"])
    assert np.array_equal(X.cpu().numpy().view(np.uint64), o["X"])


@pytest.mark.parametrize("n", [70, 3100])                 # one wave per path; a team of four
def test_relink_rejects_bad_arguments(ctx, ub, n):
    prob = ctx.problem(make_instance(n, 0.5, -100, 100, 1))
    W = prob.W
    elite = torch.zeros((3, W), dtype=torch.int64, device="cuda")
    X = torch.zeros((2, W), dtype=torch.int64, device="cuda")
    f = torch.zeros(2, dtype=torch.int64, device="cuda")
    st = torch.zeros(2, dtype=torch.int32, device="cuda")
    with pytest.raises(ub.UbqpError):
        ctx.relink(prob, elite, torch.zeros((2, 2), dtype=torch.int32, device="cuda"), X, f, f, st, max_flips=-1)
    # a pair index outside the elite set is reported by the next synchronisation
    ctx.relink(prob, elite, torch.tensor([[0, 1], [0, 3]], dtype=torch.int32, device="cuda"), X, f, f.clone(), st)
    with pytest.raises(ub.UbqpError):
        ctx.sync()
    ctx.sync()


def test_relink_single_pair_of_identical_rows(ctx):
    """A pair whose two solutions coincide: no intermediate, the row unchanged."""
    n = 90
    Q = make_instance(n, 0.5, -100, 100, 3)
    elite = random_candidates(1, n, 4)
    prob = ctx.problem(Q)
    ed = torch.from_numpy(elite.view(np.int64)).cuda()
    pairs = torch.tensor([[0, 0]], dtype=torch.int32, device="cuda")
    X = torch.full((1, prob.W), -1, dtype=torch.int64, device="cuda")
    fm = torch.zeros(1, dtype=torch.int64, device="cuda")
    fo = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    ctx.relink(prob, ed, pairs, X, fm, fo, st)
    ctx.sync()
    assert st.item() == 0 and fm.item() == np.iinfo(np.int64).min and fo.item() == fm.item()
    assert np.array_equal(X.cpu().numpy().view(np.uint64), elite)
