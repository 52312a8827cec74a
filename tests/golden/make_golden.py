"""Writes the stored expected values of the small cube workload (oracle only).

Workload: n = 2048 points uniform in the unit cube (seed 0), A_ij = 1/|x_i - x_j|
off the diagonal, A_ii = 1e3, leaf 128, eta = 1, eps = 1e-8; the k-th eigenvalue
for k = n/2 at absolute tolerance 1e-8 (Algorithm 1, Sec. 2).

Every value below comes from ``oracle/`` (the H^2 oracle and its dense
checkers): the inertia nu(sigma) on a grid of shifts together with the counts at
sigma -/+ w, w = 1e3 * eps * normA (the window inside which a truncation-level
difference may move an eigenvalue across sigma); lambda_{n/2} from the oracle's
Algorithm 1 with its step count; lambda_{n/2} of the dense matrix from LAPACK
(``numpy.linalg.eigvalsh``), which the H^2 result must approach within
tol/2 + 10 * eps * normA (Eq. error-bound plus the construction error); and a
scan of the oracle's nu at 17 shifts 1e-4 apart around lambda_{n/2}.

Run from the repository root:  python tests/golden/make_golden.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.bisect import bisect_kth, gershgorin  # noqa: E402
from oracle.build import H2  # noqa: E402
from oracle.factor import inertia  # noqa: E402
from oracle.kernels import Kernel  # noqa: E402
from paper_2311_08618_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cube_laplace_n2048.json")


def main():
    n, leaf, eta, eps, tol, k = 2048, 128, 1.0, 1e-8, 1e-8, 1024
    X = W.cube_points(n, 0)
    kern = Kernel(W.K_LAPLACE, 1e3)
    t0 = time.time()
    H = H2(X, kern, leaf, eta, eps)
    w = 1e3 * eps * H.normA
    shifts = [float(s) for s in np.linspace(820.0, 1240.0, 15)] + [985.0, 985.3, 985.38, 990.0, 1000.0]
    recs = []
    for s in shifts:
        recs.append({"sigma": s, "nu": int(inertia(H, s)), "nu_lo": int(inertia(H, s - w)),
                     "nu_hi": int(inertia(H, s + w))})
    ab = gershgorin(X, kern, 10.0 * eps * H.normA)
    lam, br, steps = bisect_kth(lambda mu: inertia(H, mu), k, ab[0], ab[1], tol)
    dense = np.linalg.eigvalsh(kern.dense(X))
    # a fine scan around lambda_k: steps of 1e-4 (about 2 tau); at these shifts
    # the oracle's count equals the dense one
    lam_d = float(dense[k - 1])
    scan = []
    for j in range(-8, 9):
        s = lam_d + j * 1e-4
        scan.append({"sigma": s, "nu": int(inertia(H, s)), "nu_dense": int(np.sum(dense < s))})
    data = {
        "workload": "cube-laplace n=2048 leaf=128 eta=1 eps=1e-8 A_ii=1e3 (points: cube_points(2048, seed 0))",
        "source": "oracle/ (H^2 oracle, Algorithm 1) and numpy.linalg.eigvalsh of the dense matrix",
        "n": n, "leaf": leaf, "eta": eta, "eps": eps, "tol": tol, "k": k,
        "normA": H.normA, "window": w,
        "tree_perm_head": [int(v) for v in H.tree.perm()[:64]],
        "inertia": recs,
        "gershgorin": list(ab),
        "lambda_oracle": lam, "bracket_oracle": list(br), "steps_oracle": steps,
        "lambda_dense": float(dense[k - 1]),
        "gap_below": float(dense[k - 1] - dense[k - 2]), "gap_above": float(dense[k] - dense[k - 1]),
        "scan_near_lambda": scan,
    }
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1)
    print("wrote %s in %.1f s: lambda_oracle %.10f lambda_dense %.10f steps %d" %
          (OUT, time.time() - t0, lam, dense[k - 1], steps))


if __name__ == "__main__":
    main()
