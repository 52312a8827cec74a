"""Kernel-matrix entries A_ij = f(|x_i - x_j|) (i != j), A_ii = diag.

The paper's synthetic test uses the regularised Laplace kernel
1/(|x_i - x_j| + 1e-3) (Sec. 5.1).  The other kinds are the workloads this
library is measured on.  Kind codes match the C ABI.
"""
from __future__ import annotations

import numpy as np

LAPLACE, YUKAWA, GAUSS_DAMPED, REG_LAPLACE, TRIDIAG_1D = 0, 1, 2, 3, 4


class Kernel:
    def __init__(self, kind: int, diag: float, p0: float = 0.0, p1: float = 0.0):
        self.kind, self.diag, self.p0, self.p1 = int(kind), float(diag), float(p0), float(p1)

    def f(self, r: np.ndarray) -> np.ndarray:
        """Off-diagonal kernel value at distance r (no diagonal handling)."""
        k = self.kind
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            if k == LAPLACE:
                return 1.0 / r
            if k == YUKAWA:
                return np.exp(-r) / r
            if k == GAUSS_DAMPED:
                return np.exp(-r * r / self.p0) / (r + self.p1)
            if k == REG_LAPLACE:
                return 1.0 / (r + self.p0)
            if k == TRIDIAG_1D:
                return np.where(np.abs(r - self.p0) < 1e-9 * self.p0, -1.0, 0.0)
        raise ValueError("unknown kernel kind %d" % k)

    def block(self, X: np.ndarray, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
        """Dense block A(rows, cols) for original point indices rows, cols."""
        P, Q = X[rows], X[cols]
        d = P[:, None, :] - Q[None, :, :]
        r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
        out = self.f(r)
        same = rows[:, None] == cols[None, :]
        out = np.where(same, self.diag, out)
        return out

    def dense(self, X: np.ndarray) -> np.ndarray:
        idx = np.arange(X.shape[0])
        return self.block(X, idx, idx)
