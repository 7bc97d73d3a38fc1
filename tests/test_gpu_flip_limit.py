"""The ascent's flip limit (ubqp_problem_set_flip_limit): an ascent to a local
optimum that reaches it stops, and every call that reports the device's checks
returns UBQP_ELIMIT instead of a result cut short.  The limit is forced from the
host (a few flips against ascents of dozens); every kernel still ends normally.
Capped ascents (max_flips > 0) are unaffected, and the default limit gives the
oracle's results."""
import numpy as np
import pytest

import oracle
from paper_1706_00037_amd.inputs import make_instance, random_candidates

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1706_00037_amd import ubqp
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return ubqp.Context(0)


def dev(a):
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a.view(np.int64) if a.dtype == np.uint64 else a).cuda()


@pytest.mark.parametrize("n,lo,hi", [(500, -100, 100), (700, -32768, 32767),
                                     (4000, -100, 100),       # a team of four waves per passer
                                     (4000, -32768, 32767)])  # the same with two planes
def test_step_ascent_reports_the_limit(ctx, n, lo, hi):
    from paper_1706_00037_amd import ubqp
    M = 32
    Q = make_instance(n, 0.3, lo, hi, 71 + n)
    X = random_candidates(M, n, 72)
    f = oracle.eval_many(Q, X, threads=8)
    _, _, want_flips = oracle.ascent_many(Q, X, np.arange(M, dtype=np.int32), f, threads=8)
    assert want_flips.min() > 3                    # every ascent needs more than the limit
    prob = ctx.problem(Q)
    idx = dev(np.arange(M, dtype=np.int32))
    cnt = dev(np.array([M], np.int64))
    prob.set_flip_limit(3)
    fl = torch.zeros(M, dtype=torch.int32, device="cuda")
    ctx.ascent(prob, dev(X), idx, cnt, dev(f), fl)
    with pytest.raises(ubqp.UbqpError) as e:
        ctx.sync()
    assert e.value.code == ubqp.UBQP_ELIMIT
    assert (fl.cpu().numpy() == 3).all()
    # a capped ascent stops at its cap without error, whatever the limit
    Xd, fd = dev(X), dev(f)
    ctx.ascent(prob, Xd, idx, cnt, fd, fl, max_flips=2)
    ctx.sync()
    Xo, fo, _ = oracle.ascent_many(Q, X, np.arange(M, dtype=np.int32), f, max_flips=2)
    assert np.array_equal(fd.cpu().numpy(), fo) and np.array_equal(Xd.cpu().numpy().view(np.uint64), Xo)
    # back to the default: the oracle's local optima
    prob.set_flip_limit(0)
    Xd, fd = dev(X), dev(f)
    ctx.ascent(prob, Xd, idx, cnt, fd, fl)
    ctx.sync()
    Xo, fo, flo = oracle.ascent_many(Q, X, np.arange(M, dtype=np.int32), f)
    assert np.array_equal(fd.cpu().numpy(), fo) and np.array_equal(fl.cpu().numpy(), flo)


def test_runs_and_batches_report_the_limit(ctx):
    from paper_1706_00037_amd import ubqp
    Qa = make_instance(400, 0.3, -100, 100, 81)
    Qb = make_instance(300, 0.3, -100, 100, 82)
    pa, pb = ctx.problem(Qa), ctx.problem(Qb)
    kw = dict(M=600, H=10, lam_num=1, lam_den=2, G=2, run_seed=3)
    pa.set_flip_limit(2)
    with pytest.raises(ubqp.UbqpError) as e:
        ctx.multistart(pa, **kw)
    assert e.value.code == ubqp.UBQP_ELIMIT
    # in a batch only the instance whose ascent hit the limit fails
    b = ctx.batch([pb, pa], [kw, kw])
    b.step(2)
    rb = b.result(0)
    o = oracle.multistart(Qb, threads=8, **kw)
    assert rb["best_f"] == o["best_f"] and np.array_equal(rb["stats"], o["stats"])
    with pytest.raises(ubqp.UbqpError) as e:
        b.result(1)
    assert e.value.code == ubqp.UBQP_ELIMIT
    b.close()
    pa.set_flip_limit(0)
    r = ctx.multistart(pa, **kw)
    o = oracle.multistart(Qa, threads=8, **kw)
    assert r["best_f"] == o["best_f"] and np.array_equal(r["best_x"], o["best_x"])


def test_sequential_reports_the_limit(ctx):
    from paper_1706_00037_amd import ubqp
    Q = make_instance(300, 0.3, -100, 100, 83)
    o = oracle.sequential(Q, 50, 100, 300, 0, 1, run_seed=1)
    assert o["flips"] > o["passers"] > 0           # some ascent takes two flips or more
    prob = ctx.problem(Q)
    prob.set_flip_limit(1)
    with pytest.raises(ubqp.UbqpError) as e:
        ctx.sequential(prob, iterations=50, samples=100, H=0, lam_num=0, lam_den=1, run_seed=1)
    assert e.value.code == ubqp.UBQP_ELIMIT
