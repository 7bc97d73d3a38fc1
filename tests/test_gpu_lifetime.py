"""Lifetime of a context and of what is created on it: ubqp_destroy may come
before the problems, runs, batches and servers made on the context are
destroyed; the context then lives until the last of them is gone.  Python's
collector relies on this: objects that end in one reference cycle (a test's
frame held by the traceback of an exception it caught, say) are finalized in no
set order, the context's handle possibly first."""
import gc

import numpy as np
import pytest

import oracle
from paper_1706_00037_amd.inputs import make_instance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RUN = dict(M=256, H=10, lam_num=1, lam_den=2, G=2, run_seed=3)


@pytest.fixture(scope="module")
def ubqp():
    from paper_1706_00037_amd import ubqp
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return ubqp


@pytest.fixture(scope="module")
def Q():
    return make_instance(300, 0.3, -100, 100, 41)


def test_context_released_before_its_holders(ubqp, Q):
    ctx = ubqp.Context(0)
    prob = ctx.problem(Q)
    run = ctx.run(prob, **RUN)
    run.step(RUN["G"])
    batch = ctx.batch([prob], [RUN])
    srv = ctx.server(pool_bytes=64 << 20, max_active=2)
    ctx.close()                      # ubqp_destroy with four holders alive
    r = run.result()                 # the run's own state is still there
    o = oracle.multistart(Q, **RUN)
    assert r["best_f"] == o["best_f"] and np.array_equal(r["stats"], o["stats"])
    srv.close()
    prob.close()
    batch.close()
    run.close()                      # the last holder frees the context
    # a fresh context afterwards gives the oracle's result
    ctx2 = ubqp.Context(0)
    r2 = ctx2.multistart(ctx2.problem(Q), **RUN)
    assert r2["best_f"] == o["best_f"] and np.array_equal(r2["best_x"], o["best_x"])
    ctx2.close()


def test_reference_cycles_collected_in_any_order(ubqp, Q):
    for _ in range(4):
        ctx = ubqp.Context(0)
        prob = ctx.problem(Q)
        run = ctx.run(prob, **RUN)
        cyc = [ctx, prob, run]
        cyc.append(cyc)
        del ctx, prob, run, cyc
        gc.collect()
    ctx = ubqp.Context(0)
    r = ctx.multistart(ctx.problem(Q), **RUN)
    assert r["best_f"] == oracle.multistart(Q, **RUN)["best_f"]
