"""Pins of the oracle's path relinking (greedy relinking; orc_relink_path).

The walk is rebuilt by brute force: every step re-evaluates f(x xor e_k) for
every free k with a numpy product (no deltas) and takes the largest, lowest k on
ties.  Besides: the intermediate lies between the two solutions at the reported
distance, the two delta modes agree, the degenerate distances have closed
forms, and the polished result is a local optimum no worse than the
intermediate."""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1706_00037_amd.inputs import make_instance, pack_bits, random_candidates, unpack_bits

I64_MIN = np.iinfo(np.int64).min


def f_np(Q, xd):
    xd = np.asarray(xd, np.int64)
    return int(xd @ np.asarray(Q, np.int64) @ xd)


def walk_brute(Q, xi, xg):
    """(steps, x_mid, f_mid) by direct evaluation."""
    x = xi.astype(np.int64).copy()
    free = [k for k in range(len(x)) if xi[k] != xg[k]]
    best, best_step, best_x = None, 0, xi.copy()
    for s in range(1, len(free)):
        vals = []
        for k in free:
            y = x.copy(); y[k] ^= 1
            vals.append((f_np(Q, y), -k))
        fv, negk = max(vals)
        k = -negk
        x[k] ^= 1
        free.remove(k)
        if best is None or fv > best:
            best, best_step, best_x = fv, s, x.copy()
    return best_step, best_x, (I64_MIN if best is None else best)


@pytest.mark.parametrize("n,d,lo,hi,seed", [(9, 0.8, -20, 20, 1), (14, 0.5, -50, 50, 2), (23, 0.9, -10, 10, 3),
                                            (66, 0.3, -100, 100, 4), (70, 1.0, -3, 3, 5)])
def test_relink_path_matches_brute_force_walk(n, d, lo, hi, seed):
    Q = make_instance(n, d, lo, hi, seed)
    X = random_candidates(6, n, seed + 10)
    for a in range(3):
        for b in range(3, 6):
            xi, xg = unpack_bits(X[a], n), unpack_bits(X[b], n)
            st, xm, fm = oracle.relink_path(Q, X[a], X[b])
            bst, bx, bf = walk_brute(Q, xi, xg)
            assert (st, fm) == (bst, bf), (a, b)
            assert np.array_equal(unpack_bits(xm, n), bx)


def test_relink_intermediate_lies_between_and_modes_agree():
    n = 150
    Q = make_instance(n, 0.3, -100, 100, 7)
    X = random_candidates(8, n, 8)
    for a in range(4):
        for b in range(4, 8):
            st, xm, fm = oracle.relink_path(Q, X[a], X[b])
            assert st >= 1
            xi, xg, xd = unpack_bits(X[a], n), unpack_bits(X[b], n), unpack_bits(xm, n)
            same = xi == xg
            assert np.array_equal(xd[same], xi[same])
            assert int((xd != xi).sum()) == st and int((xd != xg).sum()) == int((xi != xg).sum()) - st
            assert fm == f_np(Q, xd)
            st1, xm1, fm1 = oracle.relink_path(Q, X[a], X[b], mode=1)
            assert (st1, fm1) == (st, fm) and np.array_equal(xm1, xm)


def test_relink_degenerate_distances():
    n = 40
    Q = make_instance(n, 0.5, -100, 100, 9)
    x = random_candidates(1, n, 10)[0]
    xd = unpack_bits(x, n)
    # distance 0 and 1: no intermediate
    for k in (None, 17):
        g = xd.copy()
        if k is not None:
            g[k] ^= 1
        st, xm, fm = oracle.relink_path(Q, x, pack_bits(g[None, :])[0])
        assert st == 0 and fm == I64_MIN and np.array_equal(xm, x)
    # distance 2 (variables i < j): the single intermediate is the better single flip, i on ties
    i, j = 5, 31
    g = xd.copy(); g[i] ^= 1; g[j] ^= 1
    yi, yj = xd.copy(), xd.copy()
    yi[i] ^= 1; yj[j] ^= 1
    fi, fj = f_np(Q, yi), f_np(Q, yj)
    st, xm, fm = oracle.relink_path(Q, x, pack_bits(g[None, :])[0])
    assert st == 1 and fm == max(fi, fj)
    assert np.array_equal(unpack_bits(xm, n), yi if fi >= fj else yj)


def test_relink_toward_the_complement_takes_n_minus_one_steps_at_most():
    n = 60
    Q = make_instance(n, 0.4, -100, 100, 11)
    x = random_candidates(1, n, 12)[0]
    comp = pack_bits((1 - unpack_bits(x, n))[None, :])[0]
    st, xm, fm = oracle.relink_path(Q, x, comp)
    bst, bx, bf = walk_brute(Q, unpack_bits(x, n), unpack_bits(comp, n))
    assert 1 <= st <= n - 1 and (st, fm) == (bst, bf)


@pytest.mark.parametrize("mf", [0, 3])
def test_relink_many_polishes_each_intermediate(mf):
    n = 45
    Q = make_instance(n, 0.5, -100, 100, 13)
    E = 5
    elite = random_candidates(E, n, 14)
    elite[3] = elite[1]                                     # an identical pair: no intermediate
    pairs = np.array([(a, b) for a in range(E) for b in range(E) if a != b], np.int32)
    r = oracle.relink_many(Q, elite, pairs, max_flips=mf, threads=2)
    for p, (a, b) in enumerate(pairs):
        st, xm, fm = oracle.relink_path(Q, elite[a], elite[b])
        assert r["steps"][p] == st and r["f_mid"][p] == fm
        if st == 0:
            assert r["f_out"][p] == I64_MIN and np.array_equal(r["X"][p], elite[a])
            continue
        xa, fa, _ = oracle.ascent(Q, xm, fm, max_flips=mf)
        assert r["f_out"][p] == fa >= fm and np.array_equal(r["X"][p], xa)
        if mf == 0:
            assert brute.is_local_optimum(Q, unpack_bits(r["X"][p], n).astype(np.int64))
    assert (r["steps"][[p for p, (a, b) in enumerate(pairs) if {a, b} == {1, 3}]] == 0).all()
