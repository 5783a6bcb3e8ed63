"""Small test-side helpers: random problems of controlled structure.

Inputs only; no precoding arithmetic lives here.
"""
from __future__ import annotations

import numpy as np


def random_problem(rng, nt, k, lo=None, hi=None, nlos=True, xi=None, disjoint=False):
    """A random drop with contiguous VRs. ``disjoint`` places the VRs so that
    no two overlap (requires sum of lengths <= nt)."""
    lo = max(0, nt // 4 if lo is None else lo)
    hi = max(lo, nt // 2 if hi is None else hi)
    if disjoint:
        seg = nt // k
        vl = rng.integers(max(0, min(lo, seg) // 2), seg + 1, size=k).astype(np.int32)
        vs = np.array([i * seg + rng.integers(0, seg - vl[i] + 1) for i in range(k)], dtype=np.int32)
        perm = rng.permutation(k)
        vs, vl = vs[perm], vl[perm]
    else:
        vl = rng.integers(lo, min(hi, nt) + 1, size=k).astype(np.int32)
        vs = np.array([rng.integers(0, nt - L + 1) for L in vl], dtype=np.int32)
    H = np.zeros((k, nt), dtype=np.complex128)
    for i in range(k):
        a, L = vs[i], vl[i]
        if L:
            H[i, a:a + L] = (rng.standard_normal(L) + 1j * rng.standard_normal(L)) * 0.3
            if not nlos:
                H[i, a:a + L] = np.exp(2j * np.pi * rng.random(L)) * 0.1
    if xi is None:
        xi = float(k / 10.0)
    return H, vs, vl, float(xi)


def qpsk(rng, shape):
    b = rng.integers(0, 2, size=tuple(shape) + (2,))
    v = (2.0 * b - 1.0) / np.sqrt(2.0)
    return v[..., 0] + 1j * v[..., 1]


def rzf_numpy(H, S, xi):
    """RZF via numpy.linalg.solve (the textbook library routine)."""
    M = H @ H.conj().T + xi * np.eye(H.shape[0])
    V = np.linalg.solve(M, np.atleast_2d(S).T).T
    X = V @ H.conj()
    return X, V


def augmented(H, xi):
    """A = [H, sqrt(xi) I] of the consistent system."""
    return np.hstack([H, np.sqrt(xi) * np.eye(H.shape[0])])
