"""CPU oracle for the diversified multi-start UBQP method (arXiv:1706.00037).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py``; never by the product package.

``ubqp_oracle.c`` holds the arithmetic (plain scalar C, int64/int128); this module
builds it with gcc and wraps it with ctypes over numpy arrays.  ``brute`` is a
second, independent numpy implementation used to pin it on tiny instances.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ubqp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ubqp_oracle.c into liboracle.so with gcc (plain -O2, OpenMP only
    to partition independent candidates across threads)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-fvisibility=hidden", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("H", ctypes.c_int32), ("lam_num", ctypes.c_int32),
                ("lam_den", ctypes.c_int32), ("G", ctypes.c_int32), ("max_flips", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("run_seed", ctypes.c_uint64)]


class SeqParams(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("samples", ctypes.c_int64), ("H", ctypes.c_int64),
                ("lam_num", ctypes.c_int32), ("lam_den", ctypes.c_int32), ("max_flips", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("run_seed", ctypes.c_uint64)]


class SeqOut(ctypes.Structure):
    _fields_ = [("best_f", ctypes.c_int64), ("have_best", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("sample_sum", ctypes.c_int64), ("start_f", ctypes.c_int64), ("passers", ctypes.c_int64),
                ("flips", ctypes.c_int64), ("improvements", ctypes.c_int64)]


class Dump(ctypes.Structure):
    _fields_ = [("f", ctypes.c_void_p), ("fa", ctypes.c_void_p), ("pass_", ctypes.c_void_p),
                ("xa", ctypes.c_void_p), ("seeds", ctypes.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        sig = {
            "orc_splitmix64": (u64, [u64, u64]),
            "orc_random_solution": (None, [i32, u64, i64, i64, i64, P]),
            "orc_f": (i64, [i32, P, P]),
            "orc_eval": (None, [i32, P, P, i64, P, i32]),
            "orc_diversify": (None, [i32, P, i64, i32, P, i64]),
            "orc_blend": (None, [i32, P, i64, i64, i64, u64, P]),
            "orc_sequential": (None, [i32, P, P, P, P, P, P, i64, i32]),
            "orc_relink_path": (i64, [i32, P, P, P, i32, P, P]),
            "orc_relink_many": (None, [i32, P, P, P, i64, i32, P, P, P, P, i32]),
            "orc_screen": (i64, [P, i64, i32, i32, P, P, P]),
            "orc_delta_recompute": (None, [i32, P, P, P]),
            "orc_delta": (None, [i32, P, P, P]),
            "orc_ascent": (i64, [i32, P, P, P, i32, i32]),
            "orc_ascent_many": (None, [i32, P, P, P, i64, P, i32, P, i32]),
            "orc_derivative_start": (None, [i32, P, P]),
            "orc_multistart": (i32, [i32, P, ctypes.POINTER(Params), P, P, P, ctypes.POINTER(Dump),
                                     i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _q(Q):
    Q = np.ascontiguousarray(Q, dtype=np.int32)
    assert Q.ndim == 2 and Q.shape[0] == Q.shape[1]
    return Q


def words(n: int) -> int:
    return (n + 63) // 64


def splitmix64(seed: int, i: int) -> int:
    return int(lib().orc_splitmix64(seed, i))


def random_solution(n, run_seed, g, S, s):
    x = np.zeros(words(n), np.uint64)
    lib().orc_random_solution(n, run_seed, g, S, s, _p(x))
    return x


def f(Q, x) -> int:
    Q = _q(Q)
    x = np.ascontiguousarray(x, np.uint64)
    return int(lib().orc_f(Q.shape[0], _p(Q), _p(x)))


def eval_many(Q, X, threads: int = 1):
    Q = _q(Q)
    X = np.ascontiguousarray(X, np.uint64)
    M = X.shape[0]
    out = np.zeros(M, np.int64)
    lib().orc_eval(Q.shape[0], _p(Q), _p(X), M, _p(out), threads)
    return out


def diversify(n, seeds, H, M):
    seeds = np.ascontiguousarray(seeds, np.uint64)
    X = np.zeros((M, words(n)), np.uint64)
    lib().orc_diversify(n, _p(seeds), seeds.shape[0], H, _p(X), M)
    return X


def blend(n, seeds, M, g, run_seed):
    """Blending diversification of generation g (pairs of seeds, SplitMix64 masks)."""
    seeds = np.ascontiguousarray(seeds, np.uint64)
    X = np.zeros((M, words(n)), np.uint64)
    lib().orc_blend(n, _p(seeds), seeds.shape[0], M, g, run_seed, _p(X))
    return X


def screen(fv, lam_num, lam_den):
    fv = np.ascontiguousarray(fv, np.int64)
    M = fv.shape[0]
    idx = np.zeros(M, np.int32)
    s = np.zeros(1, np.int64)
    m = np.zeros(1, np.int64)
    P = lib().orc_screen(_p(fv), M, lam_num, lam_den, _p(idx), _p(s), _p(m))
    return idx[:P].copy(), int(s[0]), int(m[0])


def delta(Q, x, recompute: bool = False):
    Q = _q(Q)
    x = np.ascontiguousarray(x, np.uint64)
    d = np.zeros(Q.shape[0], np.int64)
    fn = lib().orc_delta_recompute if recompute else lib().orc_delta
    fn(Q.shape[0], _p(Q), _p(x), _p(d))
    return d


def ascent(Q, x, fx=None, max_flips: int = 0, mode: int = 0):
    """Returns (x_after, f_after, flips)."""
    Q = _q(Q)
    x = np.array(x, np.uint64, copy=True)
    fv = np.array([f(Q, x) if fx is None else fx], np.int64)
    flips = lib().orc_ascent(Q.shape[0], _p(Q), _p(x), _p(fv), max_flips, mode)
    return x, int(fv[0]), int(flips)


def ascent_many(Q, X, idx, fv, max_flips: int = 0, threads: int = 1):
    """Ascends rows idx of X in place (copies returned): (X, f, flips)."""
    Q = _q(Q)
    X = np.array(X, np.uint64, copy=True)
    fv = np.array(fv, np.int64, copy=True)
    idx = np.ascontiguousarray(idx, np.int32)
    flips = np.zeros(X.shape[0], np.int64)
    lib().orc_ascent_many(Q.shape[0], _p(Q), _p(X), _p(idx), idx.shape[0], _p(fv), max_flips,
                          _p(flips), threads)
    return X, fv, flips


def derivative_start(Q):
    Q = _q(Q)
    x = np.zeros(words(Q.shape[0]), np.uint64)
    lib().orc_derivative_start(Q.shape[0], _p(Q), _p(x))
    return x


FLAG_DERIV_START, FLAG_BLEND = 1, 2


def multistart(Q, M, H, lam_num, lam_den, G, max_flips=0, run_seed=0, flags=0, threads=1,
               dump=False):
    """Returns dict(best_f, best_x, have_best, stats[G,5]); with dump=True also
    f_all[G,M], fa_all[G,M], pass_all[G,M], xa_all[G,M,W], seeds_all[G,S,W]."""
    Q = _q(Q)
    n = Q.shape[0]
    W = words(n)
    S = -(-M // (2 * H))
    pr = Params(M, H, lam_num, lam_den, G, max_flips, flags, run_seed)
    bf = np.zeros(1, np.int64)
    bx = np.zeros(W, np.uint64)
    st = np.zeros((G, 5), np.int64)
    d = None
    if dump:
        arrs = dict(f_all=np.zeros((G, M), np.int64), fa_all=np.zeros((G, M), np.int64),
                    pass_all=np.zeros((G, M), np.uint8), xa_all=np.zeros((G, M, W), np.uint64),
                    seeds_all=np.zeros((G, S, W), np.uint64))
        d = Dump(arrs["f_all"].ctypes.data, arrs["fa_all"].ctypes.data, arrs["pass_all"].ctypes.data,
                 arrs["xa_all"].ctypes.data, arrs["seeds_all"].ctypes.data)
    have = lib().orc_multistart(n, _p(Q), ctypes.byref(pr), _p(bf), _p(bx), _p(st),
                                ctypes.byref(d) if dump else None, threads)
    out = dict(best_f=int(bf[0]), best_x=bx, have_best=bool(have), stats=st)
    if dump:
        out.update(arrs)
    return out


def sequential(Q, iterations, samples, H, lam_num, lam_den, max_flips=0, run_seed=0, threads=1,
               history_cap=1 << 16):
    """The main loop of Fig. 2 one candidate per iteration (orc_sequential).
    Returns dict(best_f, best_x, have_best, sample_sum, start_f, passers, flips,
    improvements, history[k, 2] = (iteration, value), f_dump[iterations])."""
    Q = _q(Q)
    n = Q.shape[0]
    pr = SeqParams(iterations, samples, H, lam_num, lam_den, max_flips, 0, run_seed)
    out = SeqOut()
    bx = np.zeros(words(n), np.uint64)
    fd = np.zeros(iterations, np.int64)
    hist = np.zeros((history_cap, 2), np.int64)
    lib().orc_sequential(n, _p(Q), ctypes.byref(pr), ctypes.byref(out), _p(bx), _p(fd), _p(hist), history_cap,
                         threads)
    k = min(out.improvements, history_cap)
    return dict(best_f=out.best_f, best_x=bx, have_best=bool(out.have_best), sample_sum=out.sample_sum,
                start_f=out.start_f, passers=out.passers, flips=out.flips, improvements=out.improvements,
                history=hist[:k].copy(), f_dump=fd)


def relink_path(Q, x_init, x_guide, mode=0):
    """Greedy relinking from x_init toward x_guide: (steps, x_mid, f_mid)."""
    Q = _q(Q)
    n = Q.shape[0]
    xi = np.ascontiguousarray(x_init, np.uint64)
    xg = np.ascontiguousarray(x_guide, np.uint64)
    xm = np.zeros(words(n), np.uint64)
    fm = np.zeros(1, np.int64)
    st = lib().orc_relink_path(n, _p(Q), _p(xi), _p(xg), mode, _p(xm), _p(fm))
    return int(st), xm, int(fm[0])


def relink_many(Q, elite, pairs, max_flips=0, threads=1):
    """Relinking of pairs (rows of [P, 2] indices into elite), then ascent:
    dict(X, f_mid, f_out, steps)."""
    Q = _q(Q)
    n = Q.shape[0]
    elite = np.ascontiguousarray(elite, np.uint64)
    pairs = np.ascontiguousarray(pairs, np.int32).reshape(-1, 2)
    P = pairs.shape[0]
    X = np.zeros((P, words(n)), np.uint64)
    fm = np.zeros(P, np.int64)
    fo = np.zeros(P, np.int64)
    st = np.zeros(P, np.int64)
    lib().orc_relink_many(n, _p(Q), _p(elite), _p(pairs), P, max_flips, _p(X), _p(fm), _p(fo), _p(st), threads)
    return dict(X=X, f_mid=fm, f_out=fo, steps=st)
