"""Cluster tree, block tree and colouring (oracle).

Sec. 3.1 indexes same-level blocks A_{level;row,col} of a binary subdivision.
The paper leaves the clustering rule and the strong-admissibility condition
unstated; the readings used here are:

  * clustering: every cluster of level l < L is split at the median of its
    longest bounding-box axis (lowest axis on ties, stable sort by that
    coordinate, left child = first floor(|tau|/2) points).  L is the smallest
    depth at which every cluster holds at most ``leaf`` points, so all leaves
    sit at level L.  Children of cluster p are 2p and 2p+1.
  * admissibility ("strong", Secs. 1 and 3.4): clusters i != j are admissible
    iff eta * |c_i - c_j| >= rho_i + rho_j, with c the bounding-box centre and
    rho half the bounding-box diagonal, and |c_i - c_j| > 0.
  * block tree: level-synchronous from N_0 = {(0,0)}; the candidate pairs of
    level l are the children pairs of the near pairs of level l-1; admissible
    candidates form the interaction list I_l, the rest the near list N_l
    (dense blocks).  Non-near pairs of level l whose parents are not near are
    "inherited far": they are represented through an ancestor's coupling.
  * colouring: greedy over the near graph of each level in ascending cluster
    index, smallest colour not used by an already coloured near neighbour.
    Clusters are eliminated colour-major, index-minor.
"""
from __future__ import annotations

import numpy as np


class Tree:
    """Cluster tree + block tree of a point set (oracle's own)."""

    def __init__(self, X: np.ndarray, leaf: int, eta: float):
        X = np.asarray(X, dtype=np.float64)
        if X.ndim == 1:
            X = X.reshape(-1, 1)
        n = X.shape[0]
        self.X, self.n, self.leaf, self.eta = X, n, int(leaf), float(eta)
        L = 0
        while -(-n // (1 << L)) > leaf:
            L += 1
        self.L = L
        # idx[l][i]: original point indices of cluster i at level l, in tree order
        idx = [[np.arange(n)]]
        for l in range(1, L + 1):
            nxt = []
            for a in idx[l - 1]:
                P = X[a]
                ext = P.max(axis=0) - P.min(axis=0)
                ax = int(np.argmax(ext))
                order = np.argsort(P[:, ax], kind="stable")
                half = len(a) // 2
                nxt.append(a[order[:half]])
                nxt.append(a[order[half:]])
            idx.append(nxt)
        self.idx = idx
        self.center, self.radius = [], []
        for l in range(L + 1):
            cs, rs = [], []
            for a in idx[l]:
                P = X[a]
                lo, hi = P.min(axis=0), P.max(axis=0)
                cs.append(0.5 * (lo + hi))
                rs.append(0.5 * float(np.linalg.norm(hi - lo)))
            self.center.append(np.array(cs))
            self.radius.append(np.array(rs))
        # block tree
        self.near = [[[0]]]          # near[l][i]: sorted near neighbours (incl. i)
        self.far = [[[]]]            # far[l][i]: sorted interaction list I_l(i)
        for l in range(1, L + 1):
            N = 1 << l
            near = [[] for _ in range(N)]
            far = [[] for _ in range(N)]
            for p in range(N >> 1):
                for q in self.near[l - 1][p]:
                    for c in (2 * p, 2 * p + 1):
                        for d in (2 * q, 2 * q + 1):
                            if self.admissible(l, c, d):
                                far[c].append(d)
                            else:
                                near[c].append(d)
            self.near.append([sorted(v) for v in near])
            self.far.append([sorted(v) for v in far])
        self.near_set = [[set(v) for v in lv] for lv in self.near]
        # colouring and elimination order
        self.colour, self.order = [], []
        for l in range(L + 1):
            N = 1 << l
            col = [-1] * N
            for i in range(N):
                used = {col[j] for j in self.near[l][i] if j < i}
                c = 0
                while c in used:
                    c += 1
                col[i] = c
            self.colour.append(col)
            self.order.append(sorted(range(N), key=lambda i: (col[i], i)))

    def admissible(self, l: int, i: int, j: int) -> bool:
        if i == j:
            return False
        d = float(np.linalg.norm(self.center[l][i] - self.center[l][j]))
        return d > 0.0 and self.eta * d >= self.radius[l][i] + self.radius[l][j]

    def nclusters(self, l: int) -> int:
        return 1 << l

    def far_field(self, l: int, i: int):
        """Clusters (level, index) making up the far field of cluster i at level l:
        the interaction lists of i and of all its ancestors (Sec. 3.1: the shared
        basis of a row spans every low-rank block of that row)."""
        out = []
        a = i
        for lv in range(l, 0, -1):
            for q in self.far[lv][a]:
                out.append((lv, q))
            a >>= 1
        return out

    def pts(self, l: int, i: int) -> np.ndarray:
        """Original point indices of cluster i at level l in tree order (the
        concatenation of its leaves, left to right)."""
        s = self.L - l
        return np.concatenate(self.idx[self.L][i << s:(i + 1) << s])

    def perm(self) -> np.ndarray:
        """Original point indices in leaf order."""
        return np.concatenate(self.idx[self.L])
