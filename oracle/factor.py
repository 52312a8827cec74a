"""Generalized H^2-LDL of A~ - sigma*I, inertia only (oracle).

Secs. 3.2-3.4 and 4, written as plainly as possible with dense NumPy blocks
held in dictionaries keyed by ordered cluster pairs (both orientations stored).

State at level l, in every cluster's current coordinates (redundant part
first, skeleton part last, Eq. dense_skeleton):
  S[(j,k)]  dense near blocks (Eq. dense_skeleton; after the merge, the
            Eq. hss_dense_skeleton blocks of the parent level);
  F[(j,k)]  explicit fill-in on non-near pairs (Sec. 3.4, the "orange
            blocks"); admissible pairs keep their coupling C separately, whose
            redundant rows are zero (Eq. lr_skeleton).

For every cluster i, in colour-major / index-minor order:
  (i)   recompression (Sec. 3.4 displaymath): the products to concatenate are
        the R_i rows of every fill-in product that landed in row i of a
        non-near block, one product per (eliminated neighbour, block), plus
        the R_i rows of the fill-in carried up from the level below.  A
        rank-revealing (column-pivoted) QR of the concatenation, truncated
        once the Frobenius norm of the remaining part is <= tau_i =
        tau * sqrt(|cluster i| / n) (the construction's budget, so that the
        truncations of one level sum to at most tau in the 2-norm), gives t
        directions that join the skeleton: the
        redundant coordinates are rotated by W = [Q_perp | Q_t] (Q_t an
        orthonormal basis of the kept directions) and the last t of them
        become skeleton coordinates.  The redundant rows of the
        non-near blocks of row i are then dropped (the truncation).
  (ii)  pivot block P = S_ii^{RR}; its inertia is added to nu (Eq.
        blr2-diag-ldl; Sylvester's law, Sec. 2 and Sec. 4).  The oracle takes
        the plain definition: the number of negative eigenvalues of P.
  (iii) elimination (Eq. blr2-diag-elimination) and Schur complements (Eq.
        blr2-diag-schur) for every ordered pair (j,k) of near neighbours of i,
        with the rows of j restricted to its skeleton part once j is
        eliminated (including j = i): S_jk -= S_ji P^{-1} S_ik.  Pairs (j,k)
        that are not near receive fill-in.
After all clusters of a level: merge (Sec. 3.3): each parent's coordinates
are [new skeleton directions of child 1 | of child 2 | E^T (original
skeleton coordinates of both children)], where E = [E^R | E^S] is the
transfer matrix; new directions start in the parent's redundant part.  Near
parent blocks receive the children's skeleton blocks (near blocks, and
couplings plus fill-in of admissible child pairs); fill-in of non-near parent
pairs is carried up.  The root is reached with no skeleton part left.

Readings where the paper is silent are listed in the design notes: the
concatenated products (per eliminated neighbour and block), the truncation
rule (remaining Frobenius norm <= tau * sqrt(|cluster| / n), tau = eps*normA),
inherited-far fill-in carried to the
parent level, and the embedding of the transfer matrix after rank growth.
"""
from __future__ import annotations

import math

import numpy as np


def rrqr_directions(X: np.ndarray, tol: float):
    """Rank-revealing QR of the concatenation X (R_i x ncol), Sec. 3.4.

    Column-pivoted Householder QR of X^T: the pivots are coordinates of the
    redundant part, chosen by largest remaining norm (recomputed at every
    step, first index on ties), stopping when the Frobenius norm of the whole
    remaining block is <= tol.  With X^T P = Q R, X ~= P R^T Q^T, so the
    kept directions are the first t columns of P R^T, and X minus its
    projection on them has Frobenius norm <= tol.  Returns (t, P R^T[:, :t])."""
    A = np.array(X.T, dtype=np.float64, copy=True)     # ncol x R_i
    n, m = A.shape
    perm = np.arange(m)
    t = 0
    for k in range(min(n, m)):
        sq = np.sum(A[k:, k:] * A[k:, k:], axis=0)
        if not math.sqrt(float(np.sum(sq))) > tol:
            break
        j = int(np.argmax(sq))
        j += k
        if j != k:
            A[:, [k, j]] = A[:, [j, k]]
            perm[[k, j]] = perm[[j, k]]
        x = A[k:, k].copy()
        alpha = -np.copysign(np.linalg.norm(x), x[0] if x[0] != 0 else 1.0)
        v = x
        v[0] -= alpha
        vn = np.dot(v, v)
        if vn > 0:
            A[k:, k:] -= np.outer(v, (2.0 / vn) * (v @ A[k:, k:]))
        t = k + 1
    Rt = np.triu(A[:t, :]).T                           # m x t, rows in pivoted order
    At = np.zeros((m, t))
    At[perm, :] = Rt
    return t, At


def _rotate(i, W, R_i, S, F, nbS, nbF):
    """Rotate the first R_i coordinates of cluster i by W (R_i x R_i):
    rows of blocks (i, *) and columns of blocks (*, i)."""
    for store, nb in ((S, nbS), (F, nbF)):
        for q in nb:
            blk = store[(i, q)]
            blk[:R_i, :] = W.T @ blk[:R_i, :]
        for q in nb:
            blk = store[(q, i)]
            blk[:, :R_i] = blk[:, :R_i] @ W


def inertia(H, sigma: float, stats: dict | None = None, on_level=None) -> int:
    """nu(A~ - sigma I) = #{lambda(A~) < sigma} by the generalized H^2-LDL.

    on_level, if given, is called after the eliminations of every level l and
    before its merge as on_level(l, nu, S, F, m, R): the negative pivots
    counted so far and the blocks that hold the remaining (skeleton) system,
    for checks of the inertia bookkeeping; it must not modify them."""
    T, L = H.tree, H.tree.L
    m = list(H.m[L])
    r0 = list(H.r[L])
    R = [m[i] - r0[i] for i in range(1 << L)]
    S = {}
    for i in range(1 << L):
        for j in T.near[L][i]:
            S[(i, j)] = H.B[(i, j)].copy()
        S[(i, i)] -= sigma * np.eye(m[i])
    F = {}
    nu = 0
    if stats is not None:
        stats.setdefault("t", [])
        stats.setdefault("R", [])
        stats.setdefault("m", [])
    for l in range(L, -1, -1):
        N = 1 << l
        near = T.near_set[l]
        elim = [False] * N
        pending = [[] for _ in range(N)]
        for (i, q), blk in F.items():
            if R[i] > 0:
                pending[i].append(blk[:R[i], :].copy())
        tl = [0] * N
        fnb = [set() for _ in range(N)]        # non-near partners holding fill-in
        for (a, b) in F:
            fnb[a].add(b)
        for i in T.order[l]:
            # (i) recompression of row/column i
            Ri = R[i]
            if Ri > 0:
                if pending[i]:
                    Xc = np.concatenate(pending[i], axis=1)
                    t, At = rrqr_directions(Xc, H.cluster_tol(l, i))
                    if t > 0:
                        Qc, _ = np.linalg.qr(At, mode="complete")
                        W = np.concatenate([Qc[:, t:], Qc[:, :t]], axis=1)
                        _rotate(i, W, Ri, S, F, T.near[l][i], sorted(fnb[i]))
                        Ri -= t
                        R[i] = Ri
                        tl[i] = t
                for q in fnb[i]:
                    F[(i, q)][:Ri, :] = 0.0
                    F[(q, i)][:, :Ri] = 0.0
            # (ii) pivot block and its inertia
            if Ri > 0:
                P = S[(i, i)][:Ri, :Ri]
                nu += int(np.sum(np.linalg.eigvalsh(P) < 0.0))
                nb = T.near[l][i]
                rows = {}
                for k in nb:
                    rows[k] = slice(R[k], m[k]) if (k == i or elim[k]) else slice(0, m[k])
                Bk = {k: S[(k, i)][rows[k], :Ri] for k in nb}
                Zk = {k: np.linalg.solve(P, Bk[k].T).T for k in nb}
                # (iii) Schur complements and fill-in
                for j in nb:
                    for k in nb:
                        upd = Zk[j] @ Bk[k].T
                        if k in near[j]:
                            S[(j, k)][rows[j], rows[k]] -= upd
                        else:
                            if (j, k) not in F:
                                F[(j, k)] = np.zeros((m[j], m[k]))
                                fnb[j].add(k)
                            F[(j, k)][rows[j], rows[k]] -= upd
                            if not elim[j]:
                                pending[j].append(upd[:R[j], :].copy())
            elim[i] = True
        if stats is not None:
            stats["t"].append(tl)
            stats["R"].append(list(R))
            stats["m"].append(list(m))
        if on_level is not None:
            on_level(l, nu, S, F, list(m), list(R))
        if l == 0:
            break
        # ---- merge to level l-1
        s = [m[c] - R[c] for c in range(N)]
        t = [s[c] - r0[c] for c in range(N)]
        Pm, mp, r0p, Rp = [], [], [], []
        for p in range(N >> 1):
            c1, c2 = 2 * p, 2 * p + 1
            E = H.Q[l - 1][p]
            s1, s2, t1, t2 = s[c1], s[c2], t[c1], t[c2]
            Mp = np.zeros((s1 + s2, t1 + t2 + r0[c1] + r0[c2]))
            Mp[0:t1, 0:t1] = np.eye(t1)
            Mp[s1:s1 + t2, t1:t1 + t2] = np.eye(t2)
            old = np.concatenate([np.arange(t1, s1), np.arange(s1 + t2, s1 + s2)])
            Mp[old, t1 + t2:] = E
            Pm.append(Mp)
            mp.append(Mp.shape[1])
            r0p.append(H.r[l - 1][p])
            Rp.append(Mp.shape[1] - H.r[l - 1][p])

        def child_ss(c, d, with_coupling):
            if d in near[c]:
                return S[(c, d)][R[c]:, R[d]:]
            blk = np.zeros((s[c], s[d]))
            if (c, d) in F:
                blk += F[(c, d)][R[c]:, R[d]:]
            if with_coupling and (c, d) in H.C[l]:
                blk[t[c]:, t[d]:] += H.C[l][(c, d)]
            return blk

        def assemble(p, q, with_coupling):
            top = np.concatenate([child_ss(2 * p, 2 * q, with_coupling), child_ss(2 * p, 2 * q + 1, with_coupling)], axis=1)
            bot = np.concatenate([child_ss(2 * p + 1, 2 * q, with_coupling), child_ss(2 * p + 1, 2 * q + 1, with_coupling)], axis=1)
            return Pm[p].T @ np.concatenate([top, bot], axis=0) @ Pm[q]

        S_new, F_new = {}, {}
        for p in range(N >> 1):
            for q in T.near[l - 1][p]:
                S_new[(p, q)] = assemble(p, q, True)
        for (c, d) in F:
            p, q = c >> 1, d >> 1
            if q not in T.near_set[l - 1][p] and (p, q) not in F_new:
                F_new[(p, q)] = assemble(p, q, False)
        S, F = S_new, F_new
        m, r0, R = mp, r0p, Rp
    return nu


def inertia_many(H, sigmas) -> np.ndarray:
    return np.array([inertia(H, float(s)) for s in sigmas], dtype=np.int64)
