"""Brute force over all 2^n binary x for tiny n (n <= 20), in numpy.

TEST INFRASTRUCTURE ONLY.  Independent of ubqp_oracle.c: it forms every x as a
dense 0/1 matrix and evaluates x^T Q x with a library matrix product, which is
the definition of the objective of problem (P) and nothing more.
"""
from __future__ import annotations

import numpy as np


def all_solutions(n: int) -> np.ndarray:
    """Rows are all 2^n binary vectors; row r has bit j of r in column j."""
    r = np.arange(1 << n, dtype=np.int64)
    return ((r[:, None] >> np.arange(n, dtype=np.int64)[None, :]) & 1).astype(np.int64)


def objective_all(Q: np.ndarray) -> np.ndarray:
    """f(x) = x^T Q x for every x of all_solutions(n), int64."""
    Q = np.asarray(Q, dtype=np.int64)
    X = all_solutions(Q.shape[0])
    return ((X @ Q) * X).sum(axis=1)


def optimum(Q: np.ndarray):
    """(max f, the lowest-numbered x attaining it as a dense 0/1 vector)."""
    fv = objective_all(Q)
    r = int(np.argmax(fv))
    n = np.asarray(Q).shape[0]
    return int(fv[r]), ((r >> np.arange(n)) & 1).astype(np.int64)


def is_local_optimum(Q: np.ndarray, x_dense: np.ndarray) -> bool:
    """True iff no single flip increases f (checked by direct re-evaluation)."""
    Q = np.asarray(Q, dtype=np.int64)
    x = np.asarray(x_dense, dtype=np.int64)
    f0 = x @ Q @ x
    for i in range(x.shape[0]):
        y = x.copy()
        y[i] ^= 1
        if y @ Q @ y > f0:
            return False
    return True
