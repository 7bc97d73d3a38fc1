"""Pins of the oracle's sequential main loop (Fig. 2 with one candidate per
iteration; orc_sequential).

The checks do not repeat the loop.  They recompute what it must have done from
its outputs with separate code: objectives by numpy products, the screen
against T rebuilt from the improvement history, candidates rebuilt from the
seeds that are known (the starting solution before the first improvement, the
final incumbent after the last one), and the special values of lambda whose
outcome is fixed."""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1706_00037_amd.inputs import make_instance, unpack_bits, pack_bits


def f_np(Q, xd):
    xd = np.asarray(xd, np.int64)
    return int(xd @ np.asarray(Q, np.int64) @ xd)


def start_np(Q):
    return (np.asarray(Q, np.int64).sum(axis=1) > 0).astype(np.int64)


def candidate_np(seed_dense, i, H):
    """Iteration i >= 1: flip j = 0, h, 2h, ... with h = ((i-1)//2 mod H) + 1,
    complement when i-1 is odd."""
    x = seed_dense.copy()
    c = i - 1
    h = (c // 2) % H + 1
    x[::h] ^= 1
    if c % 2:
        x ^= 1
    return x


def run(Q, **kw):
    kw.setdefault("threads", 4)
    return oracle.sequential(Q, **kw)


CASES = [(40, 0.5, -50, 50, 300, 20, 7, (1, 2), 0),
         (130, 0.2, -100, 100, 400, 50, 13, (3, 10), 0),
         (65, 0.9, -128, 127, 250, 7, 3, (4, 5), 0),
         (100, 0.5, -100, 100, 300, 30, 100, (1, 2), 2),
         (1, 1.0, -100, 100, 9, 5, 2, (1, 2), 0)]


@pytest.mark.parametrize("n,d,lo,hi,I,Ms,H,lam,mf", CASES)
def test_sequential_consistent_with_its_outputs(n, d, lo, hi, I, Ms, H, lam, mf):
    Q = make_instance(n, d, lo, hi, 300 + n)
    r = run(Q, iterations=I, samples=Ms, H=H, lam_num=lam[0], lam_den=lam[1], max_flips=mf, run_seed=5)
    # Mean and the starting value, by numpy
    samples = np.stack([unpack_bits(oracle.random_solution(n, 5, 0, Ms, s), n) for s in range(Ms)])
    assert r["sample_sum"] == int(((samples.astype(np.int64) @ Q.astype(np.int64)) * samples).sum())
    x0 = start_np(Q)
    assert r["start_f"] == f_np(Q, x0)
    # history: strictly increasing iterations and values, ending at the incumbent
    hist = r["history"]
    assert len(hist) == r["improvements"]
    if len(hist):
        assert (np.diff(hist[:, 0]) > 0).all() and (np.diff(hist[:, 1]) > 0).all()
        assert r["have_best"] and hist[-1, 1] == r["best_f"]
    else:
        assert not r["have_best"]
    # candidates whose seed is known
    fd = r["f_dump"]
    assert fd[0] == r["start_f"]
    first = hist[0, 0] if len(hist) else I - 1
    for i in range(1, min(first, 60) + 1):
        assert fd[i] == f_np(Q, candidate_np(x0, i, H)), i
    if r["have_best"]:
        xb = unpack_bits(r["best_x"], n).astype(np.int64)
        assert f_np(Q, xb) == r["best_f"]
        assert mf > 0 or brute.is_local_optimum(Q, xb)
        for i in range(max(hist[-1, 0] + 1, I - 60), I):
            assert fd[i] == f_np(Q, candidate_np(xb, i, H)), i
    # the screen: T rebuilt from Mean and the Max in force at each iteration
    num, den = lam
    mx = np.full(I, r["start_f"], dtype=object)
    for it, v in hist:
        mx[it + 1:] = int(v)
    passed = [den * Ms * int(fd[i]) > (den - num) * r["sample_sum"] + num * Ms * int(mx[i]) for i in range(I)]
    assert sum(passed) == r["passers"]
    assert all(passed[int(it)] for it, _ in hist)


def test_lambda_one_makes_every_passer_an_improvement():
    Q = make_instance(120, 0.3, -100, 100, 1)
    r = run(Q, iterations=500, samples=30, H=60, lam_num=1, lam_den=1, run_seed=2)
    assert r["passers"] == r["improvements"] > 0


def test_lambda_zero_screens_against_the_mean():
    Q = make_instance(90, 0.5, -100, 100, 2)
    I, Ms = 300, 40
    r = run(Q, iterations=I, samples=Ms, H=45, lam_num=0, lam_den=1, run_seed=3)
    assert r["passers"] == int((Ms * r["f_dump"] > r["sample_sum"]).sum())


def test_single_iteration_is_the_ascent_of_the_starting_solution():
    Q = make_instance(150, 0.3, -100, 100, 4)
    r = run(Q, iterations=1, samples=100, H=10, lam_num=1, lam_den=2, run_seed=1)
    x0 = start_np(Q)
    mean_below = 100 * r["start_f"] > r["sample_sum"]
    assert r["passers"] == int(mean_below)
    assert mean_below
    xa, fa, flips = oracle.ascent(Q, pack_bits(x0[None, :])[0])
    assert r["best_f"] == fa and r["flips"] == flips and np.array_equal(r["best_x"], xa)
    assert r["f_dump"][0] == f_np(Q, x0)


@pytest.mark.parametrize("n,seed", [(7, 1), (10, 2), (12, 3)])
def test_sequential_bounded_by_brute_force(n, seed):
    Q = make_instance(n, 0.7, -20, 20, seed)
    opt = brute.optimum(Q)[0]
    r = run(Q, iterations=60, samples=10, H=n, lam_num=1, lam_den=2, run_seed=seed)
    if r["have_best"]:
        assert r["best_f"] <= opt
        assert brute.is_local_optimum(Q, unpack_bits(r["best_x"], n).astype(np.int64))


def test_history_cap_keeps_the_first_entries():
    Q = make_instance(120, 0.3, -100, 100, 1)
    full = run(Q, iterations=500, samples=30, H=60, lam_num=1, lam_den=1, run_seed=2)
    cut = oracle.sequential(Q, iterations=500, samples=30, H=60, lam_num=1, lam_den=1, run_seed=2, history_cap=2)
    assert cut["improvements"] == full["improvements"] and np.array_equal(cut["history"], full["history"][:2])
