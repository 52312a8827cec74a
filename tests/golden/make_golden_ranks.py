"""Writes the stored rank statistics of the factorization at n = 8192 (oracle only).

Workloads: n = 8192 points uniform in the unit cube (seed 0), leaf 256, eta = 1:
  * A_ij = 1/|x_i - x_j|, A_ii = 1e3, eps = 1e-8;
  * A_ij = exp(-|x_i - x_j|)/|x_i - x_j|, A_ii = 1e3, eps = 1e-10.
For one shift in the bulk of each spectrum the oracle's generalized H^2-LDL
(Secs. 3.2-3.4) records, per level l = 0 .. L, the sum over the level's
clusters of the directions t added by fill-in recompression, the sum and the
maximum of the cluster dimensions m, and the sum of the pivot block sizes R;
together with the inertia nu(sigma) and nu(sigma -/+ w), w = 1e3 * eps * normA.
The construction ranks per level (sum and maximum) are stored too.

Run from the repository root:  python tests/golden/make_golden_ranks.py
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.build import H2  # noqa: E402
from oracle.factor import inertia  # noqa: E402
from oracle.kernels import Kernel  # noqa: E402
from paper_2311_08618_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rank_stats_n8192.json")

CASES = [
    ("cube-laplace", W.K_LAPLACE, 1e-8, 1000.0),
    ("cube-yukawa", W.K_YUKAWA, 1e-10, 1005.0),
]


def case(name, kind, eps, sigma, n=8192, leaf=256):
    t0 = time.time()
    X = W.cube_points(n, 0)
    H = H2(X, Kernel(kind, 1e3), leaf, 1.0, eps)
    tb = time.time() - t0
    w = 1e3 * eps * H.normA
    st = {}
    nu = int(inertia(H, sigma, st))
    L = H.tree.L
    levels = []
    # stats lists run from level L down to the last level reached
    for j, (tl, Rl, ml) in enumerate(zip(st["t"], st["R"], st["m"])):
        l = L - j
        levels.append({"level": l, "sum_t": int(sum(tl)), "sum_m": int(sum(ml)), "max_m": int(max(ml)),
                       "sum_R": int(sum(Rl))})
    rec = {
        "name": name, "n": n, "leaf": leaf, "eta": 1.0, "eps": eps, "kind": kind, "diag": 1e3,
        "normA": H.normA, "sigma": sigma, "window": w,
        "nu": nu, "nu_lo": int(inertia(H, sigma - w)), "nu_hi": int(inertia(H, sigma + w)),
        "levels": levels,
        "basis_ranks": [{"level": l, "sum": int(sum(H.r[l])), "max": int(max(H.r[l]))} for l in range(L + 1)],
        "build_s": round(tb, 1), "total_s": round(time.time() - t0, 1),
    }
    print("%s: nu %d [%d, %d], levels %s (%.0f s)" % (name, nu, rec["nu_lo"], rec["nu_hi"],
                                                     [(v["level"], v["sum_t"], v["max_m"]) for v in levels],
                                                     rec["total_s"]), flush=True)
    return rec


def main():
    data = {
        "workload": "cube_points(8192, seed 0), leaf 256, eta 1; Laplace eps 1e-8 and Yukawa eps 1e-10, A_ii = 1e3",
        "source": "oracle/ (H^2 construction and generalized H^2-LDL)",
        "cases": [case(*c) for c in CASES],
    }
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
