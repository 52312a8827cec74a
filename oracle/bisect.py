"""Slicing the spectrum (Algorithm 1) with inertia reuse (oracle).

Algorithm 1 (Sec. 2): starting from [a, b] containing lambda_k, repeat while
b_k - a_k >= eps_ev: mu = (a_k + b_k)/2; if nu(A - mu I) >= k then b_k = mu
else a_k = mu.  Return (a_k + b_k)/2, which is within eps_ev/2 of lambda_k
when every inertia is correct (Eq. error-bound).

Inertia reuse (Sec. 4.2, first bullet): a recorded pair (mu, v) with v < k
proves lambda_k >= mu, and v >= k proves lambda_k < mu, so the starting
interval of k shrinks to [max{mu : v < k}, min{mu : v >= k}] intersected with
[a, b].

Default starting interval when none is given: the Gershgorin interval of the
kernel matrix, [min_i(A_ii - sum_{j!=i}|A_ij|), max_i(A_ii + sum_{j!=i}|A_ij|)],
widened by 10*eps*normA on both sides to cover the H^2 approximation error.
"""
from __future__ import annotations

import numpy as np


def bisect_kth(nu_fn, k: int, a: float, b: float, tol: float, cache: list | None = None):
    """Algorithm 1.  nu_fn(mu) -> #{lambda < mu}.  Returns (lambda~, (a_k, b_k), steps)."""
    ak, bk = float(a), float(b)
    if cache:
        for mu, v in cache:
            if v < k and mu > ak:
                ak = mu
            if v >= k and mu < bk:
                bk = mu
    steps = 0
    while bk - ak >= tol:
        mu = 0.5 * (ak + bk)
        v = int(nu_fn(mu))
        steps += 1
        if cache is not None:
            cache.append((mu, v))
        if v >= k:
            bk = mu
        else:
            ak = mu
    return 0.5 * (ak + bk), (ak, bk), steps


def expected_steps(width: float, tol: float) -> int:
    """Number of halvings Algorithm 1 performs on an interval of this width:
    the smallest s with width / 2^s < tol."""
    s = 0
    w = float(width)
    while w >= tol:
        w *= 0.5
        s += 1
    return s


def gershgorin(X: np.ndarray, kern, margin: float = 0.0):
    """Exact Gershgorin interval of the kernel matrix (row chunks)."""
    n = X.shape[0]
    lo, hi = np.inf, -np.inf
    allc = np.arange(n)
    for c0 in range(0, n, 256):
        rows = np.arange(c0, min(n, c0 + 256))
        blk = kern.block(X, rows, allc)
        d = blk[np.arange(len(rows)), rows]
        rad = np.abs(blk).sum(axis=1) - np.abs(d)
        lo = min(lo, float(np.min(d - rad)))
        hi = max(hi, float(np.max(d + rad)))
    return lo - margin, hi + margin


def kth_eigs(H, ks, tol: float, ab=None, nu_fn=None):
    """lambda~_k for every k (1-based), sharing one inertia cache."""
    from .factor import inertia
    if nu_fn is None:
        nu_fn = lambda mu: inertia(H, mu)
    if ab is None:
        ab = gershgorin(H.X, H.kern, 10.0 * H.eps * H.normA)
    cache = []
    out = []
    for k in ks:
        lam, _, _ = bisect_kth(nu_fn, int(k), ab[0], ab[1], tol, cache)
        out.append(lam)
    return np.array(out)
