"""Pins of the oracle's blending diversification (a reading: the paper reports
blending two solutions without a rule; see the oracle's orc_blend).

The crossover invariants hold for any correct uniform crossover; the parent
pairs come from a hand-worked fixture; the mask bits are checked against the
separately pinned SplitMix64; multistart runs with blending are checked against
brute force and against their own dumps."""
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1706_00037_amd.inputs import make_instance, unpack_bits

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "blend_parents.txt")


def _golden():
    cases = []
    for line in open(GOLDEN):
        if not line.strip() or line.startswith("#"):
            continue
        head, tail = line.split(":")
        S, M, g = (int(v) for v in head.split())
        pairs = [tuple(int(v) for v in t.split(",")) for t in tail.split()]
        cases.append((S, M, g, pairs))
    return cases


def _seeds(n, S, seed):
    return np.stack([oracle.random_solution(n, seed, 0, S, s) for s in range(S)])


def _parents_of(even, odd, seeds):
    """All (a, b) with even ^ odd == a ^ b and even & odd == a & b (the children
    of a and b under some mask)."""
    out = []
    for a in range(len(seeds)):
        for b in range(len(seeds)):
            if np.array_equal(even ^ odd, seeds[a] ^ seeds[b]) and np.array_equal(even & odd, seeds[a] & seeds[b]):
                out.append((a, b))
    return out


@pytest.mark.parametrize("S,M,g,pairs", _golden())
def test_blend_parents_match_hand_worked_pairs(S, M, g, pairs):
    n = 130
    seeds = _seeds(n, S, 40 + S)
    X = oracle.blend(n, seeds, M, g, run_seed=9)
    assert len(pairs) == (M + 1) // 2
    for k, (a, b) in enumerate(pairs):
        even = X[2 * k]
        odd = X[2 * k + 1] if 2 * k + 1 < M else None
        if odd is None:                       # a lone last child: its bits come from a or b
            assert np.array_equal(even & ~(seeds[a] | seeds[b]), np.zeros_like(even))
            assert np.array_equal((seeds[a] & seeds[b]) & ~even, np.zeros_like(even))
            continue
        if a == b:
            assert np.array_equal(even, seeds[a]) and np.array_equal(odd, seeds[a])
        else:
            # children of distinct random seeds identify their parents (up to order)
            found = _parents_of(even, odd, seeds)
            assert (a, b) in found and len({frozenset(p) for p in found}) == 1, (k, found)


def test_blend_mask_bits_are_splitmix_outputs():
    n, S, M, g, rs = 200, 5, 23, 4, 77
    seeds = _seeds(n, S, 3)
    X = oracle.blend(n, seeds, M, g, rs)
    W, pairs = oracle.words(n), (M + 1) // 2
    for k in range(pairs):
        a, b = k % S, (k % S + 1 + k // S + g) % S
        if a == b:
            continue
        for w in range(W):
            m = oracle.splitmix64(rs, (1 << 62) + (g * pairs + k) * W + w)
            diff = int(seeds[a][w] ^ seeds[b][w])
            even = int(X[2 * k][w])
            # where the parents differ, the even child shows parent a exactly where m = 1
            assert (even ^ int(seeds[b][w])) & diff == m & diff, (k, w)
            if 2 * k + 1 < M:
                odd = int(X[2 * k + 1][w])
                assert (odd ^ int(seeds[a][w])) & diff == m & diff, (k, w)


def test_blend_crossover_invariants_and_padding():
    n, S, M, g = 157, 7, 60, 2
    seeds = _seeds(n, S, 11)
    X = oracle.blend(n, seeds, M, g, run_seed=5)
    W = oracle.words(n)
    pad = ~np.uint64((1 << (n - 64 * (W - 1))) - 1)
    for c in range(M):
        assert (X[c][W - 1] & pad) == 0
    for k in range(M // 2):
        found = _parents_of(X[2 * k], X[2 * k + 1], seeds)
        assert found, k


def test_blend_single_seed_reproduces_it():
    n = 90
    seeds = _seeds(n, 1, 8)
    X = oracle.blend(n, seeds, 9, 3, run_seed=1)
    assert all(np.array_equal(x, seeds[0]) for x in X)


@pytest.mark.parametrize("n,seed", [(6, 1), (9, 2), (11, 3)])
def test_multistart_blend_bounded_by_brute_force(n, seed):
    Q = make_instance(n, 0.7, -20, 20, seed)
    opt = brute.optimum(Q)[0]
    r = oracle.multistart(Q, M=40, H=3, lam_num=1, lam_den=3, G=6, run_seed=seed, flags=oracle.FLAG_BLEND)
    if r["have_best"]:
        assert r["best_f"] <= opt
        assert oracle.f(Q, r["best_x"]) == r["best_f"]
        assert brute.is_local_optimum(Q, unpack_bits(r["best_x"], n).astype(np.int64))


def test_multistart_blend_uses_blending_of_its_seeds():
    """Every generation's objectives are those of the blend of that generation's
    seeds (dumped), and the statistics agree with the dump."""
    n, M, H, G, rs = 70, 90, 5, 4, 12
    Q = make_instance(n, 0.4, -50, 50, 21)
    r = oracle.multistart(Q, M=M, H=H, lam_num=1, lam_den=2, G=G, run_seed=rs, flags=oracle.FLAG_BLEND,
                          dump=True)
    for g in range(G):
        X = oracle.blend(n, r["seeds_all"][g], M, g, rs)
        assert np.array_equal(oracle.eval_many(Q, X), r["f_all"][g]), g
        assert r["stats"][g, 0] == r["f_all"][g].sum() and r["stats"][g, 1] == r["f_all"][g].max()
    glover = oracle.multistart(Q, M=M, H=H, lam_num=1, lam_den=2, G=G, run_seed=rs)
    assert not np.array_equal(glover["stats"], r["stats"])      # a different generator
