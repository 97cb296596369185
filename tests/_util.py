"""Shared helpers of the test-suite (matching of eigenvalue sets)."""
import numpy as np
from scipy.optimize import linear_sum_assignment


def match_sets(a, b):
    """Optimal one-to-one matching of two equal-size complex sets; returns the
    largest |a_i - b_j| used."""
    a = np.asarray(a)
    b = np.asarray(b)
    assert len(a) == len(b), (len(a), len(b))
    if len(a) == 0:
        return 0.0
    cost = np.abs(a[:, None] - b[None, :])
    r, c = linear_sum_assignment(cost)
    return float(cost[r, c].max())


def subspace_gap(V, W):
    """sin of the largest principal angle between span(V) and span(W)
    (orthonormalised first)."""
    qv, _ = np.linalg.qr(V)
    qw, _ = np.linalg.qr(W)
    s = np.linalg.svd(qv.conj().T @ qw, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - min(s) ** 2)))
