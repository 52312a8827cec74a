"""Autotuner of the batched MFMA GEMM's launch parameters on the device it runs on.

The dense contractions of the factorization (rotation, elimination, Schur
updates, fill-in Gram, merge) all run in one batched GEMM kernel per operand
layout and precision.  Its launch parameters are a table keyed by (layout,
precision, capacity bucket): the workgroups per shift (grid), the tile order
inside an item (group_m) and the output tile size (64 or 128).  Results do not
depend on them, only the speed.

For every candidate (grid, group_m, tile) the tuner writes it into every entry, runs
factorizations of a representative matrix (cube points, Laplace kernel; FP64
and FP32 contractions) with the profiler on, and charges each GEMM kernel's
HIP-event time at every level to the capacity bucket of that level (the
largest cluster dimension there).  Each entry then takes the candidate with
the least time, the minimum over repetitions.  The table is written as JSON to
tuning/gemm_tuning.json, which the binding applies at import.

    python -m paper_2311_08618_amd.autotune [--n 65536] [--reps 2] [--grids 256,512,...]
                                            [--groups 1,8] [--tiles 64,128] [--out PATH]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

from . import h2eig
from . import workloads as W

LAYOUTS = {"k_gemm<false, false>": 0, "k_gemm<false, true>": 1, "k_gemm<true, false>": 2, "k_gemm<true, true>": 3}
BUCKET_CAPS = [256, 512, 1024, 2048, None]
GRIDS = [256, 512, 1024, 2048]
GROUPS = [1, 8]
TILES = [64, 128]


def bucket_of(cap: int) -> int:
    for b, c in enumerate(BUCKET_CAPS):
        if c is None or cap <= c:
            return b
    return len(BUCKET_CAPS) - 1


def symbol(name: str):
    """(layout, f32) of a profiler GEMM entry 'kernel:k_gemm...<..>', else None
    (both tile sizes map to the same entry)."""
    if not name.startswith("kernel:"):
        return None
    s = name[len("kernel:"):].replace("k_gemm128", "k_gemm")
    f32 = s.startswith("k_gemm_f32")
    key = s.replace("k_gemm_f32", "k_gemm")
    return (LAYOUTS[key], int(f32)) if key in LAYOUTS else None


def measure(A, sig, f32: bool, reps: int):
    """{(layout, f32, bucket): ms} of one factorization, minimum over reps.
    Only the kernels of the precision under test count: an FP32 factorization
    also runs FP64 GEMMs (recompression, pivot LDL), which the FP64
    factorization measures in full."""
    best = {}
    for _ in range(reps):
        A.profile_enable(True)
        A.inertia(sig, f32=f32)
        lev = A.profile_levels()
        A.profile_enable(False)
        caps = A.level_dims()
        acc = {}
        for name, row in lev.items():
            sym = symbol(name)
            if sym is None or sym[1] != int(f32):
                continue
            for l, ms in enumerate(row[:len(caps)]):
                if ms > 0 and caps[l] > 0:
                    key = sym + (bucket_of(caps[l]),)
                    acc[key] = acc.get(key, 0.0) + ms
        for k, v in acc.items():
            best[k] = min(best.get(k, float("inf")), v)
    return best


def tune(n: int = 65536, reps: int = 2, grids=GRIDS, groups=GROUPS, tiles=TILES, log=print) -> dict:
    t0 = time.perf_counter()
    A = h2eig.H2Matrix(W.cube_points(n, 0), W.K_LAPLACE, 1e3, 256, 1.0, 1e-8, max_shifts=2)
    sig = W.shift_grid(900.0, 1100.0, 2, seed=0)
    A.inertia(sig)                      # warm-up: workspace, kernels loaded
    A.inertia(sig, f32=True)
    log("autotune: n=%d built and warmed up in %.1f s" % (n, time.perf_counter() - t0))
    saved = {(l, f, b): h2eig.get_gemm_tuning(l, f, b) for l in range(4) for f in (0, 1) for b in range(5)}
    times = {}
    try:
        for t in tiles:
            for g in grids:
                for gm in groups:
                    for key in saved:
                        h2eig.set_gemm_tuning(*key, g, gm, t)
                    for f32 in (False, True):
                        for key, ms in measure(A, sig, f32, reps).items():
                            times.setdefault(key, {})["%d/%d/%d" % (g, gm, t)] = ms
                    log("autotune: grid %d group_m %d tile %d done (%.0f s)" % (g, gm, t, time.perf_counter() - t0))
    finally:
        for key, val in saved.items():
            h2eig.set_gemm_tuning(*key, *val)
    entries = []
    for (layout, f32, bucket), cand in sorted(times.items()):
        win = min(cand, key=cand.get)
        g, gm, t = (int(x) for x in win.split("/"))
        entries.append({"layout": layout, "f32": f32, "bucket": bucket, "grid": g, "group_m": gm, "tile": t,
                        "ms": {k: round(v, 3) for k, v in sorted(cand.items())}})
    return {
        "kind": "gemm launch parameters (grid, group_m, tile) by layout (0 NN, 1 NT, 2 TN, 3 TT), f32, capacity "
                "bucket (largest block dimension <= 256, 512, 1024, 2048, larger); candidates grid/group_m/tile",
        "arch": os.environ.get("H2EIG_ARCH", "gfx950"),
        "workload": "cube-laplace n=%d leaf=256 eta=1 eps=1e-8 A_ii=1e3, 2 shifts in [900, 1100]; minimum of %d "
                    "factorizations per candidate and precision" % (n, reps),
        "candidates": ["%d/%d/%d" % (g, gm, t) for t in tiles for g in grids for gm in groups],
        "entries": entries,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--grids", default=",".join(map(str, GRIDS)))
    ap.add_argument("--groups", default=",".join(map(str, GROUPS)))
    ap.add_argument("--tiles", default=",".join(map(str, TILES)))
    ap.add_argument("--out", default=h2eig.TUNING_FILE)
    args = ap.parse_args()
    grids = [int(x) for x in args.grids.split(",")]
    groups = [int(x) for x in args.groups.split(",")]
    tiles = [int(x) for x in args.tiles.split(",")]
    table = tune(args.n, args.reps, grids, groups, tiles, log=lambda s: print(s, file=sys.stderr, flush=True))
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print("autotune: wrote %d entries to %s" % (len(table["entries"]), args.out), file=sys.stderr)


if __name__ == "__main__":
    main()
