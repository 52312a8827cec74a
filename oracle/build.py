"""H^2 construction with nested orthonormal bases (oracle).

Follows Sec. 3.1: the shared basis of a row at a level spans all low-rank
blocks of that row (Eq. shared-bases), parent bases are transfer matrices
acting on the children's skeleton coordinates (Eq. transfer-matrices), bases
are orthonormal, and the split [U^R U^S] separates the redundant part from
the skeleton part, with the criterion |U^S U^S^T A_{l;i,+} - A_{l;i,+}| <= eps_H2.
The paper allows QR, SVD or an interpolative decomposition (ID) for the
rank-revealing step; this reading uses an ID by column-pivoted QR, then
orthonormalises it (Sec. 3.1: "Orthogonalization of the shared bases can
also be done in O(n)"):

  * rows of cluster i at the leaf level are its points; at a parent level they
    are the children's skeleton points, in child order.
  * columns (the far field A_{l;i,+}): every point of every cluster in the
    interaction list of i or of one of its ancestors, at every size.
  * pivoted QR on the rows of that block with freshly computed remaining
    norms; the first maximum wins ties; stop when the Frobenius norm of the
    whole remaining block is <= tau_i = tau * sqrt(|tau_i| / n), with
    tau = eps * normA and |tau_i| the number of points of cluster i.  The
    pivots are the skeleton points s_i and M ~= X_i M(s_i, :) with
    X_i(s_i, :) = I; the residual M - X_i M(s_i, :) is that remaining block,
    so its norm is at most tau_i: the criterion of Sec. 3.1 for the block row
    of i at level l.  The budget tau_i shrinks with the cluster so that the
    block rows of one level, which partition the rows of A, have residuals
    whose squares sum to at most tau^2: the whole level then errs by at most
    tau in the 2-norm, at every n (a fixed tau per block row lets the error
    of a level grow like sqrt(2^l) * tau).
  * orthonormalisation: leaf X_i = U_i T_i (QR); parent
    blkdiag(T_c1, T_c2) X_p = E_p^S T_p.  Completed to square orthonormal
    matrices ordered [redundant | skeleton].
  * coupling of an admissible pair: C_ij = T_i A(s_i, s_j) T_j^T.
  * dense (near) leaf blocks in skeleton coordinates:
    B_ij = [U^R U^S]_i^T A_ij [U^R U^S]_j (Eq. dense_skeleton).
  * normA = max(mean of the row sums A*1 over rows i = 0 mod s, |A_ii|),
    s = max(1, n // 16384); tau = eps * normA.
"""
from __future__ import annotations

import math

import numpy as np

from .kernels import Kernel
from .tree import Tree


def pivoted_rows_id(M: np.ndarray, tol: float):
    """Row interpolative decomposition M ~= X @ M[s] by column-pivoted QR of M^T.

    Returns (s, X) with s the selected row indices (pivot order) and X of shape
    (M.shape[0], len(s)) with X[s] = I.  Remaining norms are recomputed from
    scratch at every step (slow, but the pivot rule is exactly
    "largest remaining row norm, first index on ties").  The loop stops once
    the Frobenius norm of the remaining block, which equals the Frobenius norm
    of the residual M - X M[s], is <= tol."""
    m, ncol = M.shape
    A = np.array(M.T, dtype=np.float64, copy=True)    # ncol x m: columns = rows of M
    perm = np.arange(m)
    kmax = min(m, ncol)
    r = 0
    for k in range(kmax):
        sq = np.sum(A[k:, k:] * A[k:, k:], axis=0)
        if not math.sqrt(float(np.sum(sq))) > tol:
            break
        j = int(np.argmax(sq))
        j += k
        if j != k:
            A[:, [k, j]] = A[:, [j, k]]
            perm[[k, j]] = perm[[j, k]]
        # Householder reflector zeroing A[k+1:, k]
        x = A[k:, k].copy()
        alpha = -np.copysign(np.linalg.norm(x), x[0] if x[0] != 0 else 1.0)
        v = x
        v[0] -= alpha
        vn = np.dot(v, v)
        if vn > 0:
            A[k:, k:] -= np.outer(v, (2.0 / vn) * (v @ A[k:, k:]))
        r = k + 1
    if r == 0:
        return np.zeros(0, dtype=np.int64), np.zeros((m, 0))
    R11 = np.triu(A[:r, :r])
    R12 = A[:r, r:]
    Tm = np.linalg.solve(R11, R12) if R12.shape[1] else np.zeros((r, 0))
    X = np.zeros((m, r))
    X[perm[:r], :] = np.eye(r)
    X[perm[r:], :] = Tm.T
    return perm[:r].copy(), X


def complete_basis(Y: np.ndarray):
    """QR of Y (m x r, full column rank) completed to a square orthonormal
    matrix ordered [redundant | skeleton]; returns (Q, T) with Y = Q[:, m-r:] T."""
    m, r = Y.shape
    if r == 0:
        return np.eye(m), np.zeros((0, 0))
    Qc, Rc = np.linalg.qr(Y, mode="complete")
    Q = np.concatenate([Qc[:, r:], Qc[:, :r]], axis=1)
    return Q, Rc[:r, :r]


def far_columns(tree: Tree, l: int, i: int) -> np.ndarray:
    """Every point of the far field of cluster i at level l (original indices)."""
    cols = []
    for (lv, q) in tree.far_field(l, i):
        cols.append(tree.pts(lv, q))
    if not cols:
        return np.zeros(0, dtype=np.int64)
    return np.concatenate(cols)


def estimate_norm(X: np.ndarray, kern: Kernel) -> float:
    n = X.shape[0]
    s = max(1, n // 16384)
    rows = np.arange(0, n, s)
    allc = np.arange(n)
    tot = 0.0
    for c0 in range(0, len(rows), 256):
        rr = rows[c0:c0 + 256]
        tot += float(kern.block(X, rr, allc).sum())
    return max(tot / len(rows), abs(kern.diag))


class H2:
    """An H^2 matrix built from points + kernel (oracle's own construction)."""

    def __init__(self, X, kern: Kernel, leaf: int, eta: float, eps: float):
        self.tree = T = Tree(X, leaf, eta)
        self.X = T.X
        self.kern, self.eps = kern, float(eps)
        self.normA = estimate_norm(self.X, kern)
        self.tau = self.eps * self.normA
        L = T.L
        self.r = [None] * (L + 1)       # original skeleton rank per cluster
        self.skel = [None] * (L + 1)    # skeleton points (original indices)
        self.Tf = [None] * (L + 1)      # triangular factor T
        self.Q = [None] * (L + 1)       # leaf: square basis; parent: transfer matrix E
        self.m = [None] * (L + 1)       # cluster dimension at the start of its level
        for l in range(L, -1, -1):
            N = 1 << l
            rl, sl, tl, ql, ml = [], [], [], [], []
            for i in range(N):
                if l == L:
                    rows = T.idx[L][i]
                else:
                    rows = np.concatenate([self.skel[l + 1][2 * i], self.skel[l + 1][2 * i + 1]])
                cols = far_columns(T, l, i)
                if len(cols) and len(rows):
                    M = kern.block(self.X, rows, cols)
                    piv, Xi = pivoted_rows_id(M, self.cluster_tol(l, i))
                else:
                    piv, Xi = np.zeros(0, dtype=np.int64), np.zeros((len(rows), 0))
                if l < L:
                    c1, c2 = 2 * i, 2 * i + 1
                    r1, r2 = self.r[l + 1][c1], self.r[l + 1][c2]
                    Tb = np.zeros((r1 + r2, r1 + r2))
                    Tb[:r1, :r1] = self.Tf[l + 1][c1]
                    Tb[r1:, r1:] = self.Tf[l + 1][c2]
                    Y = Tb @ Xi
                else:
                    Y = Xi
                Qi, Ti = complete_basis(Y)
                rl.append(len(piv))
                sl.append(rows[piv])
                tl.append(Ti)
                ql.append(Qi)
                ml.append(len(rows))
            self.r[l], self.skel[l], self.Tf[l], self.Q[l], self.m[l] = rl, sl, tl, ql, ml
        # couplings of admissible pairs (both orientations)
        self.C = [dict() for _ in range(L + 1)]
        for l in range(1, L + 1):
            for i in range(1 << l):
                for j in T.far[l][i]:
                    A_ss = kern.block(self.X, self.skel[l][i], self.skel[l][j])
                    self.C[l][(i, j)] = self.Tf[l][i] @ A_ss @ self.Tf[l][j].T
        # leaf near blocks in skeleton coordinates (Eq. dense_skeleton)
        self.B = {}
        for i in range(1 << L):
            for j in T.near[L][i]:
                Aij = kern.block(self.X, T.idx[L][i], T.idx[L][j])
                self.B[(i, j)] = self.Q[L][i].T @ Aij @ self.Q[L][j]

    def cluster_tol(self, l: int, i: int) -> float:
        """Truncation budget of cluster i at level l: tau * sqrt(|cluster| / n)."""
        return self.tau * math.sqrt(len(self.tree.pts(l, i)) / self.tree.n)

    # ------------------------------------------------------------------ checks
    def nested_basis(self, l: int, i: int) -> np.ndarray:
        """Explicit orthonormal skeleton basis of cluster i at level l, rows in the
        cluster's tree order (n_i x r_i)."""
        L = self.tree.L
        if l == L:
            return self.Q[L][i][:, self.m[L][i] - self.r[L][i]:]
        c1, c2 = 2 * i, 2 * i + 1
        U1, U2 = self.nested_basis(l + 1, c1), self.nested_basis(l + 1, c2)
        blk = np.zeros((U1.shape[0] + U2.shape[0], U1.shape[1] + U2.shape[1]))
        blk[:U1.shape[0], :U1.shape[1]] = U1
        blk[U1.shape[0]:, U1.shape[1]:] = U2
        E = self.Q[l][i]
        rp = self.r[l][i]
        return blk @ E[:, E.shape[1] - rp:]

    def dense(self) -> np.ndarray:
        """The H^2 matrix A~ assembled densely, in original point order."""
        T, L, n = self.tree, self.tree.L, self.tree.n
        A = np.zeros((n, n))
        for i in range(1 << L):
            for j in T.near[L][i]:
                A[np.ix_(T.idx[L][i], T.idx[L][j])] = self.kern.block(self.X, T.idx[L][i], T.idx[L][j])
        for l in range(1, L + 1):
            for i in range(1 << l):
                for j in T.far[l][i]:
                    Ui, Uj = self.nested_basis(l, i), self.nested_basis(l, j)
                    A[np.ix_(T.pts(l, i), T.pts(l, j))] = Ui @ self.C[l][(i, j)] @ Uj.T
        return A
