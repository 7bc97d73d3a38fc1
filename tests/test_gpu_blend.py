"""Parity of the blending diversification (HIP path through the C ABI) with the
oracle: the step kernel alone, and multi-start runs that use it (alone, batched
beside Glover instances, replayed as a graph, served as requests).
Every comparison is bit-exact."""
import numpy as np
import pytest

import oracle
from paper_1706_00037_amd.inputs import WORKLOADS, make_instance, random_candidates

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def host_u64(t):
    return t.cpu().numpy().view(np.uint64)


def oracle_flags(ub, flags):
    return (oracle.FLAG_DERIV_START if flags & ub.UBQP_DERIV_START else 0) | \
           (oracle.FLAG_BLEND if flags & ub.UBQP_BLEND else 0)


def _same(r, o, tag):
    assert r["have_best"] == o["have_best"], tag
    assert np.array_equal(r["stats"], o["stats"]), (tag, r["stats"], o["stats"])
    assert r["best_f"] == o["best_f"], tag
    if o["have_best"]:
        assert np.array_equal(r["best_x"], o["best_x"]), tag


@pytest.mark.parametrize("n,S,M,g,rs", [(1, 3, 55, 0, 1), (5, 1, 12, 3, 2), (64, 7, 133, 1, 3), (65, 7, 140, 9, 4),
                                        (500, 50, 1001, 2, 5), (300, 2, 1500, 2**31 - 1, 6),
                                        (8192, 3, 9, 4, 7), (7000, 820, 16384, 0, 8), (2500, 3277, 65536, 19, 9)])
def test_blend_matches_oracle(ctx, n, S, M, g, rs):
    """Ragged word tails (n = 1, 5, 65), one seed, odd M, the largest g, the
    largest n, and the seed counts of the headline shapes (n=7000, M=16384 with
    H=10 and n=2500, M=65536)."""
    seeds = random_candidates(S, n, 80 + n)
    Xd = torch.full((M, (n + 63) // 64), -1, dtype=torch.int64, device="cuda")
    ctx.blend(n, dev(seeds), Xd, g, rs)
    torch.cuda.synchronize()
    assert np.array_equal(host_u64(Xd), oracle.blend(n, seeds, M, g, rs))


def test_blend_rejects_bad_arguments(ctx, ub):
    seeds = dev(random_candidates(2, 70, 1))
    X = torch.zeros((4, 2), dtype=torch.int64, device="cuda")
    with pytest.raises(ub.UbqpError):
        ctx.blend(70, seeds, X, -1, 0)
    with pytest.raises(ub.UbqpError):
        ctx.blend(70, seeds, X, 2**31, 0)
    with pytest.raises(ub.UbqpError):
        ctx.blend(70, seeds[:0], X, 0, 0)


BLEND_CASES = [
    dict(n=200, d=0.5, lo=-32768, hi=32767, M=300, H=10, lam=(1, 2), G=4, mf=0, fl=0),
    dict(n=333, d=0.2, lo=-100, hi=100, M=999, H=7, lam=(3, 10), G=3, mf=0, fl=1),
    dict(n=64, d=0.9, lo=-128, hi=127, M=129, H=1, lam=(4, 5), G=6, mf=0, fl=0),
    dict(n=150, d=0.5, lo=-100, hi=100, M=201, H=10, lam=(1, 2), G=3, mf=3, fl=0),
    dict(n=90, d=0.5, lo=-100, hi=100, M=100, H=5, lam=(1, 1), G=2, mf=0, fl=0),     # nobody passes
    dict(n=1100, d=0.3, lo=-100, hi=100, M=2000, H=10, lam=(1, 2), G=3, mf=0, fl=0),
    dict(n=1, d=1.0, lo=-100, hi=100, M=7, H=3, lam=(1, 2), G=3, mf=0, fl=0),
]


@pytest.mark.parametrize("c", BLEND_CASES)
def test_multistart_blend_matches_oracle(ctx, ub, c):
    Q = make_instance(c["n"], c["d"], c["lo"], c["hi"], 6100 + c["n"])
    kw = dict(M=c["M"], H=c["H"], lam_num=c["lam"][0], lam_den=c["lam"][1], G=c["G"], max_flips=c["mf"],
              run_seed=13)
    fl = ub.UBQP_BLEND | (ub.UBQP_DERIV_START if c["fl"] else 0)
    r = ctx.multistart(ctx.problem(Q), flags=fl, **kw)
    o = oracle.multistart(Q, threads=8, flags=oracle_flags(ub, fl), **kw)
    _same(r, o, c)
    if c["lam"] == (1, 1):
        assert not r["have_best"]


def test_multistart_blend_dump_matches_oracle(ctx, ub):
    """The objectives of every generation's blended candidates, as dumped."""
    n, M, G = 400, 700, 4
    Q = make_instance(n, 0.4, -100, 100, 31)
    kw = dict(M=M, H=6, lam_num=1, lam_den=2, G=G, run_seed=3)
    dump = torch.zeros(G * M, dtype=torch.int64, device="cuda")
    ctx.multistart(ctx.problem(Q), flags=ub.UBQP_BLEND, f_dump=dump, **kw)
    o = oracle.multistart(Q, threads=8, flags=oracle.FLAG_BLEND, dump=True, **kw)
    assert np.array_equal(dump.cpu().numpy().reshape(G, M), o["f_all"])


def test_blend_graph_replay_equals_direct_launches(ctx, ub):
    """The generation index is read on the device, so replays of one captured
    generation blend with the right g."""
    Q = make_instance(900, 0.3, -100, 100, 78)
    prob = ctx.problem(Q)
    kw = dict(M=3000, H=10, lam_num=1, lam_den=2, G=5, run_seed=6)
    a = ctx.multistart(prob, flags=ub.UBQP_BLEND, **kw)
    b = ctx.multistart(prob, flags=ub.UBQP_BLEND | ub.UBQP_NO_GRAPH, **kw)
    _same(a, b, "graph")


def test_run_in_steps_with_blend_equals_one_call(ctx, ub):
    Q = make_instance(500, 0.3, -100, 100, 79)
    prob = ctx.problem(Q)
    kw = dict(M=1000, H=10, lam_num=1, lam_den=2, G=5, run_seed=8, flags=ub.UBQP_BLEND)
    whole = ctx.multistart(prob, **kw)
    run = ctx.run(prob, **kw)
    for k in (2, 1, 2):
        run.step(k)
    _same(run.result(), whole, "steps")
    run.close()


def test_batch_mixing_blend_and_glover(ctx, ub):
    """Blending and Glover instances in one batch (one- and two-plane): each gives
    what it gives alone and what the oracle gives."""
    cases = [(300, 0.5, -100, 100, 500, 10, ub.UBQP_BLEND), (129, 0.3, -32768, 32767, 260, 5, ub.UBQP_BLEND),
             (1100, 0.1, -100, 100, 4500, 10, 0), (64, 0.9, -128, 127, 128, 2, ub.UBQP_BLEND | ub.UBQP_DERIV_START),
             (700, 0.5, -1000, 1000, 1000, 10, 0)]
    G = 3
    probs, params, Qs = [], [], []
    for k, (n, d, lo, hi, M, H, fl) in enumerate(cases):
        Q = make_instance(n, d, lo, hi, 7100 + k)
        Qs.append(Q)
        probs.append(ctx.problem(Q))
        params.append(dict(M=M, H=H, lam_num=1, lam_den=2, G=G, run_seed=60 + k, flags=fl))
    res = ctx.multistart_batched(probs, params)
    for k, (prob, pr, r) in enumerate(zip(probs, params, res)):
        _same(r, ctx.multistart(prob, **pr), k)
        o = oracle.multistart(Qs[k], threads=8, **dict(pr, flags=oracle_flags(ub, pr["flags"])))
        _same(r, o, k)


def test_served_blend_requests_match_oracle(ctx, ub):
    cases = []
    for k, (n, dt, lo, hi, M, fl) in enumerate([(300, np.int8, -100, 100, 600, ub.UBQP_BLEND),
                                                 (129, np.int16, -32768, 32767, 260, ub.UBQP_BLEND),
                                                 (450, np.int16, -30000, 30000, 1500,
                                                  ub.UBQP_BLEND | ub.UBQP_DERIV_START),
                                                 (200, np.int8, -100, 100, 300, 0)]):
        Q = make_instance(n, 0.4, lo, hi, 9300 + k).astype(dt)
        cases.append((Q, dict(M=M, H=10, lam_num=1, lam_den=2, G=4, run_seed=70 + k, flags=fl)))
    srv = ub.Server(ctx, pool_bytes=1 << 30, max_active=8)
    try:
        ids = [srv.submit(Q, **pr) for Q, pr in cases]
        got = {}
        while len(got) < len(ids):
            for d in srv.wait(timeout_s=60.0):
                got[d["id"]] = d
    finally:
        srv.close()
    for (Q, pr), i in zip(cases, ids):
        assert got[i]["status"] == ub.UBQP_OK
        o = oracle.multistart(Q.astype(np.int32), threads=8, **dict(pr, flags=oracle_flags(ub, pr["flags"])))
        _same(got[i], o, i)


def test_multistart_blend_full_size_sampled(ctx, ub):
    """n=7000, M=16384 (the headline shape) with blending, two generations: the
    generation-0 candidates rebuilt by the oracle from the random seeds and their
    objectives compared on a sample; each generation's screen statistics
    recomputed from the dumped objectives; the incumbent checked."""
    c = WORKLOADS["n7000_d0.50_M16384"]
    n, M, H, G = c["n"], c["M"], c["H"], 2
    lam = tuple(c["lam"])
    Q = make_instance(n, c["density"], c["lo"], c["hi"], c["inst_seed"])
    dump = torch.zeros(G * M, dtype=torch.int64, device="cuda")
    r = ctx.multistart(ctx.problem(Q), M=M, H=H, lam_num=lam[0], lam_den=lam[1], G=G, run_seed=c["run_seed"],
                       flags=ub.UBQP_BLEND, f_dump=dump)
    fd = dump.cpu().numpy().reshape(G, M)
    S = -(-M // (2 * H))
    seeds = np.stack([oracle.random_solution(n, c["run_seed"], 0, S, s) for s in range(S)])
    X0 = oracle.blend(n, seeds, M, 0, c["run_seed"])
    rng = np.random.default_rng(9)
    for cnd in np.unique(np.concatenate([[0, 1, 2 * S - 1, 2 * S, M - 1], rng.choice(M, 20, replace=False)])):
        assert oracle.f(Q, X0[cnd]) == fd[0, cnd], int(cnd)
    for g in range(G):
        idx, sm, mx = oracle.screen(fd[g], lam[0], lam[1])
        assert (r["stats"][g, 0], r["stats"][g, 1], r["stats"][g, 2]) == (sm, mx, len(idx)), g
    assert r["have_best"] and oracle.f(Q, r["best_x"]) == r["best_f"] == r["stats"][-1, 4]
    assert (oracle.delta(Q, r["best_x"]) <= 0).all()


def test_unknown_flags_rejected(ctx, ub):
    prob = ctx.problem(make_instance(50, 0.5, -100, 100, 1))
    with pytest.raises(ub.UbqpError):
        ctx.multistart(prob, M=20, H=2, lam_num=1, lam_den=2, G=1, flags=1 << 10)


def test_blend_single_candidate(ctx):
    n = 200
    seeds = random_candidates(3, n, 12)
    Xd = torch.full((1, (n + 63) // 64), -1, dtype=torch.int64, device="cuda")
    ctx.blend(n, dev(seeds), Xd, 5, 21)
    torch.cuda.synchronize()
    assert np.array_equal(host_u64(Xd), oracle.blend(n, seeds, 1, 5, 21))
