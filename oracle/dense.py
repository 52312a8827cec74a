"""Brute-force checkers for the oracle (dense, small n).

  * ``dense_inertia``: #{lambda(A) < sigma} from LAPACK's symmetric
    eigensolver (NumPy eigvalsh) -- the plain definition of the inertia count
    of Sec. 2.
  * ``jacobi_eigvalsh``: cyclic Jacobi eigenvalue algorithm (Golub & Van
    Loan, Matrix Computations, Sec. 8.5), an independent eigensolver for
    n <= 512.
  * ``tridiag_eigs`` / ``tridiag_inertia``: the closed-form spectrum
    2 - 2cos(j*pi/(n+1)), j = 1..n, of tridiag(-1, 2, -1).
"""
from __future__ import annotations

import math

import numpy as np


def dense_inertia(A: np.ndarray, sigma: float) -> int:
    return int(np.sum(np.linalg.eigvalsh(A) < sigma))


def jacobi_eigvalsh(A: np.ndarray, tol: float = 1e-14, max_sweeps: int = 60) -> np.ndarray:
    """Cyclic-by-row Jacobi: annihilate a_pq with the symmetric Schur rotation
    for every p < q, sweep until off(A) <= tol * ||A||_F."""
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    fro = np.linalg.norm(A)
    for _ in range(max_sweeps):
        off = math.sqrt(max(0.0, np.sum(A * A) - np.sum(np.diag(A) ** 2)))
        if off <= tol * fro:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = A[p, q]
                if apq == 0.0:
                    continue
                tau = (A[q, q] - A[p, p]) / (2.0 * apq)
                t = (1.0 if tau >= 0 else -1.0) / (abs(tau) + math.sqrt(1.0 + tau * tau))
                c = 1.0 / math.sqrt(1.0 + t * t)
                s = t * c
                ap, aq = A[:, p].copy(), A[:, q].copy()
                A[:, p] = c * ap - s * aq
                A[:, q] = s * ap + c * aq
                ap, aq = A[p, :].copy(), A[q, :].copy()
                A[p, :] = c * ap - s * aq
                A[q, :] = s * ap + c * aq
    return np.sort(np.diag(A))


def tridiag_eigs(n: int) -> np.ndarray:
    j = np.arange(1, n + 1)
    return 2.0 - 2.0 * np.cos(j * np.pi / (n + 1))


def tridiag_inertia(n: int, sigma: float) -> int:
    """#{j : 2 - 2cos(j pi/(n+1)) < sigma} in closed form."""
    if sigma <= 0.0:
        return 0
    if sigma > 4.0:
        return n
    t = (n + 1) * math.acos(1.0 - sigma / 2.0) / math.pi
    v = math.ceil(t) - 1
    # guard the boundary j == t exactly (lambda_j == sigma is not counted)
    return int(min(n, max(0, v)))
