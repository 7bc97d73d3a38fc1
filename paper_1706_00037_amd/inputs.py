"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module only draws inputs: symmetric integer Q matrices shaped like the
paper's benchmark instances, random bit-packed candidate matrices and seed
vectors.  It holds none of the method's arithmetic (no objective, no screening,
no ascent), so both the GPU path and the CPU oracle can consume its outputs.

Instances (stand-ins for ORLIB b2500 and Palubeckis p5000-p7000, which are not
available here): for every i <= j the entry is nonzero with probability
`density`; a nonzero value is uniform over the integers of [lo, hi] other than
0; the upper triangle (diagonal included) is mirrored.  numpy PCG64, one seed
per instance.
"""
from __future__ import annotations

import numpy as np


def words(n: int) -> int:
    return (n + 63) // 64


def make_instance(n: int, density: float, lo: int, hi: int, seed: int) -> np.ndarray:
    """Symmetric int32 n x n matrix (see module docstring)."""
    assert n >= 1 and lo <= 0 <= hi and (lo < 0 or hi > 0)
    rng = np.random.Generator(np.random.PCG64(seed))
    Q = np.zeros((n, n), dtype=np.int32)
    iu, ju = np.triu_indices(n)
    keep = rng.random(iu.shape[0]) < density
    iu, ju = iu[keep], ju[keep]
    # uniform over [lo, hi] \ {0}: draw from [lo, hi-1] and shift non-negatives up by one
    v = rng.integers(lo, hi, size=iu.shape[0], endpoint=False, dtype=np.int64)
    v = np.where(v >= 0, v + 1, v).astype(np.int32)
    Q[iu, ju] = v
    Q[ju, iu] = v
    return Q


def pack_bits(B: np.ndarray) -> np.ndarray:
    """Dense 0/1 array [..., n] -> uint64 words [..., ceil(n/64)], bit j of a row in
    word j//64 at position j%64, padding bits zero."""
    B = np.asarray(B).astype(np.uint8)
    n = B.shape[-1]
    W = words(n)
    pad = np.zeros(B.shape[:-1] + (W * 64 - n,), np.uint8)
    Bp = np.concatenate([B, pad], axis=-1)
    by = np.packbits(Bp.reshape(B.shape[:-1] + (W * 8, 8)), axis=-1, bitorder="little")[..., 0]
    return np.ascontiguousarray(by).view(np.uint64).reshape(B.shape[:-1] + (W,))


def unpack_bits(X: np.ndarray, n: int) -> np.ndarray:
    """Inverse of pack_bits: uint64 words [..., W] -> 0/1 uint8 [..., n]."""
    X = np.ascontiguousarray(X, np.uint64)
    by = X.view(np.uint8)
    bits = np.unpackbits(by, axis=-1, bitorder="little")
    return bits[..., :n]


def random_candidates(M: int, n: int, seed: int, p_one: float = 0.5) -> np.ndarray:
    """M bit-packed Bernoulli(p_one) solutions, uint64 [M, ceil(n/64)]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if p_one == 0.5:
        X = rng.integers(0, 2**64, size=(M, words(n)), dtype=np.uint64)
        r = n % 64
        if r:
            X[:, -1] &= np.uint64((1 << r) - 1)
        return X
    return pack_bits(rng.random((M, n)) < p_one)


# The workloads (instance seed, run seed and shapes) used by tests and bench.
WORKLOADS = {
    "n500_d0.10_M1000": dict(n=500, density=0.10, lo=-100, hi=100, inst_seed=1001, run_seed=1,
                             M=1000, H=10, lam=(1, 2), G=20),
    "n2500_d0.10_M65536": dict(n=2500, density=0.10, lo=-100, hi=100, inst_seed=2001, run_seed=2,
                               M=65536, H=10, lam=(1, 2), G=20),
    "n7000_d0.50_M16384": dict(n=7000, density=0.50, lo=-100, hi=100, inst_seed=3001, run_seed=3,
                               M=16384, H=10, lam=(1, 2), G=20),
}


# Request stream of the serving workload: request r has n ~ U{500..7000}, density
# ~ U[0.05, 1] (both from one PCG64 stream, seed 5), coefficients uniform in
# [-100, 100] \ {0}, instance seed 5000 + r, run seed 5000 + r, M = 4096, H = 10,
# lambda = 1/2, G = 10.
SERVE_PARAMS = dict(M=4096, H=10, lam_num=1, lam_den=2, G=10)


def serving_requests(count: int, seed: int = 5):
    """The first `count` requests of the serving workload: list of dicts with n,
    density, inst_seed and run_seed (the instance itself is make_instance(n,
    density, -100, 100, inst_seed))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.integers(500, 7001, size=count)
    ds = rng.uniform(0.05, 1.0, size=count)
    return [dict(n=int(ns[r]), density=float(ds[r]), inst_seed=5000 + r, run_seed=5000 + r) for r in range(count)]


# A subset of the batched workload's shape drawn host-side: int16 coefficients
# over the whole range (two int8 planes), n spread over [1000, 7000], the three
# densities, M = 4096, H = 10, lambda = 1/2, G = 10, instance seed 4001 + k, run
# seed 4000 + k.
BATCH_SUBSET = [dict(n=1000, density=0.1), dict(n=2900, density=1.0), dict(n=4800, density=0.5),
                dict(n=7000, density=0.1)]
BATCH_PARAMS = dict(M=4096, H=10, lam_num=1, lam_den=2, G=10)
