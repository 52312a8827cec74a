"""Benchmark: H^2 LDL + inertia evaluations per second on one MI355X.

A step is one pass of the whole hot path over one batch of shifts: the
generalized H^2-LDL of A~ - sigma_s I for every shift of the batch (leaf
near-block load with the shift, fill-in recompression, basis rotation, pivot
LDL with negative-pivot count, elimination, Schur and fill-in updates, merge,
every level up to the root), ending in the inertia counts nu_s.

Workload (default): n = 2^18 points uniform in the unit cube (seed 0), Laplace
kernel 1/r off the diagonal, A_ii = 1e3, leaf 256, eta = 1, eps = 1e-8; the
shifts lie in the bulk of the spectrum (seeded, uniform in [900, 1100]).  The
H^2 matrix is built once before the timed region and stays resident in HBM.

Prints one JSON line with the metric, a "roofline" object for the dominant
kernel class (live HIP-event timing and the library's algorithmic flop
counters) and a "cpu_baseline" object (the CPU oracle timed on a bounded
sample of the same workload family).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 (matrix and vector)
HBM_PEAK_GBS = 8000.0
GEMM_CLASSES = {"recompress_w", "rotate", "elimination", "schur", "fillin_gram", "merge_fillin", "merge_transfer",
                "pivot_ldl_inverse", "recompress_pchol_update", "pivot_ldl_update"}


# step-bench workloads: (default n, points(n), kernel, A_ii, leaf, eps, p0, p1, shift range, default batch)
WORKLOADS = {
    # n points uniform in the unit cube (seed 0), 1/r: the headline configuration at n = 2^18
    "cube-laplace": (1 << 18, "cube", 0, 1e3, 256, 1e-8, 0.0, 0.0, (900.0, 1100.0), 0),
    # the same points at n = 131072, exp(-r)/r, eps 1e-10
    "cube-yukawa": (131072, "cube", 1, 1e3, 256, 1e-10, 0.0, 0.0, (900.0, 1100.0), 0),
    # 2^20 points on 16 parallel cylinders (seed 0), exp(-r^2/0.01)/(r+0.01), A_ii = 10, leaf 512
    "cylinders-gauss": (1 << 20, "cylinders", 2, 10.0, 512, 1e-8, 0.01, 0.01, (5.0, 15.0), 0),
}

KERNEL_SOURCE = os.path.join(ROOT, "paper_2311_08618_amd", "csrc", "kernels.hip")
# besides the GEMM section of KERNEL_SOURCE, what decides the GEMM's launches
GEMM_SOURCES = [os.path.join(ROOT, "paper_2311_08618_amd", "csrc", "desc.hpp"),
                os.path.join(ROOT, "paper_2311_08618_amd", "tuning", "gemm_tuning.json")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_gemm_nt_cube_laplace_n262144.md")


def gemm_source_hash(kernel_text=None, other_texts=None) -> str:
    """First 16 hex digits of the sha256 of the code that decides the batched
    GEMM's memory traffic: the GEMM section of kernels.hip (tile scan, k_gemm*
    kernels, the transposed copy-back) and its launchers, the descriptor header
    and the launch-parameter table.  Texts may be passed in (e.g. read from an
    older commit); ValueError when the section markers are missing."""
    if kernel_text is None:
        with open(KERNEL_SOURCE) as f:
            kernel_text = f.read()
    if other_texts is None:
        other_texts = []
        for p in GEMM_SOURCES:
            with open(p) as f:
                other_texts.append(f.read())

    def cut(a, b):
        i = kernel_text.index(a)
        return kernel_text[i:kernel_text.index(b, i)]

    h = hashlib.sha256()
    for t in [cut("GEMM (FP64 MFMA)", "matrix sums"), cut("void launch_variant(", "void launch_copyback(")] + other_texts:
        h.update(t.encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, n: int, S: int):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size), or None
    when it covers another kernel or workload, or the GEMM's code changed since
    the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    fields = dict(re.findall(r"^- (\w+): (.+)$", txt, flags=re.M))
    try:
        if (fields["kernel"].strip() != kernel or int(fields["n"]) != n or int(fields["shifts_per_step"]) != S
                or fields["gemm_source_sha256_16"].strip() != gemm_source_hash()):
            return None
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(nbytes: int, reps: int = 4):
    """A plain device-to-device copy of nbytes, reps times: the reference that
    scales the HBM byte counters (FETCH_SIZE reads nbytes, WRITE_SIZE writes
    nbytes per copy)."""
    import torch
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 8, "reps": reps}))


def serve_bench(args):
    """Serving loop: matrices resident in HBM, Poisson arrivals of k-th
    eigenvalue queries, continuous batching per matrix and admission by one
    shared device-memory budget (h2s_*).  For every offered rate of the sweep:
    arrivals for --serve-window seconds, then a drain until --serve-cap
    seconds after the first arrival.  Prints one JSON line: per rate the
    served and offered counts and rates, the latency percentiles of the
    finished queries, and the censored percentiles over every submitted query
    (an unfinished one counted at its age when the cap is reached)."""
    import numpy as np
    from paper_2311_08618_amd import workloads as W
    from paper_2311_08618_amd.h2eig import H2Matrix, H2Server

    sizes = [int(x) for x in args.serve_sizes.split(",")]
    rates = [float(x) for x in str(args.serve_rate).split(",")]
    seeds = {n: i for i, n in enumerate(sorted(sizes))}
    t0 = time.perf_counter()
    mats = [H2Matrix(W.cube_points(n, seeds[n]), W.K_LAPLACE, 1e3, 256, 1.0, 1e-8) for n in sizes]
    build_s = time.perf_counter() - t0
    print("serve: built %s in %.1f s" % (sizes, build_s), file=sys.stderr, flush=True)
    sweep = []
    for ri, rate in enumerate(rates):
        srv = H2Server(max_slots=args.serve_slots_max)
        t0 = time.perf_counter()
        ids = [srv.add(A) for A in mats]
        add_s = time.perf_counter() - t0
        print("serve: resident, workspace per shift measured in %.1f s" % add_s, file=sys.stderr, flush=True)
        rng = np.random.default_rng(args.serve_seed + ri)  # its own arrivals and queries per rate
        window = max(args.serve_window, 4.0 / rate)      # at least ~4 arrivals at low rates
        cap = window + args.serve_cap                    # drain after the last possible arrival
        arr = np.cumsum(rng.exponential(1.0 / rate, size=int(rate * window * 2) + 16))
        arr = arr[arr < window]
        which = rng.integers(0, len(sizes), len(arr))
        tols = np.where(rng.random(len(arr)) < 0.5, 1e-6, 1e-10)
        ks = [int(rng.integers(1, sizes[w] + 1)) for w in which]
        tickets = []
        t0 = time.perf_counter()
        for t_a, w, k, tol in zip(arr, which, ks, tols):
            dt = t0 + t_a - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            tickets.append(srv.submit(ids[w], k, float(tol)))
        print("serve: %d queries submitted over %.1f s at %g/s" % (len(tickets), window, rate),
              file=sys.stderr, flush=True)
        done = {}
        t_last = time.perf_counter()
        while len(done) < len(tickets) and time.perf_counter() - t0 < cap:
            for tk in tickets:
                if tk not in done:
                    lam = srv.poll(tk)
                    if lam is not None:
                        done[tk] = lam
            if time.perf_counter() - t_last > 10.0:
                t_last = time.perf_counter()
                print("serve: %d/%d served after %.0f s" % (len(done), len(tickets), t_last - t0),
                      file=sys.stderr, flush=True)
            time.sleep(0.05)
        elapsed = time.perf_counter() - t0
        st = srv.stats()
        cen = srv.latency()
        per = {}
        for n in sizes:
            idx = [j for j, w in enumerate(which) if sizes[w] == n]
            per[str(n)] = {"offered": len(idx), "served": sum(1 for j in idx if tickets[j] in done)}
        srv.close()
        sweep.append({
            "rate": rate, "window_s": window, "cap_s": cap,
            "offered_rate": len(tickets) / window, "offered": len(tickets), "served": st["served"],
            "served_rate": st["served"] / elapsed, "elapsed_s": round(elapsed, 1),
            "p50_ms_finished": st["p50_ms"], "p99_ms_finished": st["p99_ms"],
            "p50_ms_censored": cen["p50_ms"], "p99_ms_censored": cen["p99_ms"],
            "unfinished_at_cap": cen["unfinished"], "budget_gb": cen["budget_bytes"] / 1e9,
            "per_matrix": per,
        })
        print("serve: rate %g done: %s" % (rate, json.dumps(sweep[-1])), file=sys.stderr, flush=True)
    best = max(sweep, key=lambda r: r["served_rate"])
    line = {
        "metric": "k-th eigenvalue queries served/s (serving loop, continuous batching)",
        "value": best["served_rate"],
        "unit": "queries/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f64",
        "data": "synthetic",
        "p50_ms_censored": best["p50_ms_censored"],
        "p99_ms_censored": best["p99_ms_censored"],
        "sweep": sweep,
        "config": {"workload": "cube-laplace resident n=%s leaf=256 eta=1 eps=1e-8 A_ii=1e3; Poisson arrivals "
                               "(seed %d + index of the rate) at %s/s for max(%g s, 4/rate), k uniform in [1,n], tol 1e-6 or 1e-10 "
                               "(p=0.5); drain %g s after the arrival window; admission by one shared HBM budget "
                               "(85%% of free memory)" % (sizes, args.serve_seed, rates, args.serve_window, args.serve_cap),
                   "max_slots": args.serve_slots_max, "build_s": round(build_s, 1)},
    }
    print(json.dumps(line))


QUERY_FORMS = {"plain_f64_1shift": (1, 0.0), "batched_f64": (0, 0.0), "batched_mixed": (0, 1e-4)}


def queries_bench(args):
    """k-th eigenvalue queries, measured, in three forms on fresh handles (no
    records shared between forms): one shift per factorization in FP64
    (plain), every open bracket in one batched factorization per step in FP64,
    and batched with FP32 contractions while a bracket is at least 1e-4 normA
    wide.  For the tolerance ladder --tol t1,t2,... each form runs Algorithm 1
    to t1, then continues on the same handle to t2 and so on: the later calls
    start from the brackets the record cache holds, which are the brackets the
    uninterrupted bisection to t2 has once it passes t1, so the cumulative time
    at each tolerance is that of a run straight to it.  Prints one JSON line
    with the cumulative seconds and eigenvalues per second of every form at
    every tolerance, the eigenvalues, and their largest difference from the
    plain form when it ran."""
    import numpy as np
    from paper_2311_08618_amd import workloads as W
    from paper_2311_08618_amd.h2eig import H2Matrix

    n = args.n or 262144
    tols = [float(t) for t in str(args.tol).split(",")]
    ks = [int(k) for k in args.ks.split(",")] if args.ks else [max(1, j * n // args.nq) for j in range(args.nq)]
    forms = args.forms.split(",") if args.forms else list(QUERY_FORMS)
    os.environ["H2EIG_PROGRESS"] = "1"       # one stderr line per bisection step
    X = W.cube_points(n, 0)
    out, norm, interval = {}, None, None
    for name in forms:
        maxs, mixed = QUERY_FORMS[name]
        t0 = time.perf_counter()
        A = H2Matrix(X, W.K_LAPLACE, 1e3, 256, 1.0, 1e-8)
        print("queries: %s: built in %.1f s" % (name, time.perf_counter() - t0), file=sys.stderr, flush=True)
        if maxs:
            A.set_max_shifts(maxs)
        A.set_mixed(mixed)
        interval = A.interval()           # the starting interval, outside the timed region
        norm = A.norm()
        rec, total = {}, 0.0
        for tol in tols:
            t0 = time.perf_counter()
            lam, br = A.kth_eig(ks, tol)
            total += time.perf_counter() - t0
            st = A.stats()
            rec["tol=%g" % tol] = {"seconds": total, "eigvals_per_s": len(ks) / total, "lambda": lam.tolist(),
                                   "max_bracket": float(np.max(br[:, 1] - br[:, 0])),
                                   "evals_f64": st["evals_f64"], "evals_f32": st["evals_f32"]}
            print("queries: %s at tol %g after %.1f s (%d FP64 + %d FP32 shifts)"
                  % (name, tol, total, st["evals_f64"], st["evals_f32"]), file=sys.stderr, flush=True)
        out[name] = rec
        A.close()
    line = {
        "metric": "k-th eigenvalues/sec at n=%d: plain one-shift FP64, batched FP64, batched + FP32 early steps" % n,
        "value": None, "unit": "eigvals/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f64 (FP32 contractions in early steps for batched_mixed)", "data": "synthetic",
        "forms": out,
        "config": {"workload": "cube-laplace n=%d leaf=256 eta=1 eps=1e-8 A_ii=1e3" % n, "n": n, "ks": ks,
                   "tols": tols, "normA": norm, "interval": list(interval)},
    }
    summarize_queries(line)
    print(json.dumps(line))


def summarize_queries(line):
    """Fills value (the best form at the finest tolerance), the speedups over the
    plain form and |delta lambda| against it, per tolerance, where the plain
    form is present."""
    import numpy as np
    forms = line["forms"]
    tols = line["config"]["tols"]
    key = "tol=%g" % tols[-1]
    line["value"] = max(f[key]["eigvals_per_s"] for f in forms.values() if key in f)
    if "plain_f64_1shift" not in forms:
        return
    ref = forms["plain_f64_1shift"]
    line["speedup_vs_plain"], line["max_abs_dlambda_vs_plain"] = {}, {}
    for tol in tols:
        k = "tol=%g" % tol
        for name, f in forms.items():
            if k not in f or k not in ref:
                continue
            line["speedup_vs_plain"].setdefault(name, {})[k] = f[k]["eigvals_per_s"] / ref[k]["eigvals_per_s"]
            d = np.abs(np.array(f[k]["lambda"]) - np.array(ref[k]["lambda"]))
            line["max_abs_dlambda_vs_plain"].setdefault(name, {})[k] = float(np.max(d))


def merge_queries(paths):
    """One query record from the JSON lines of separate --queries runs on the
    same workload and tolerances (forms, or groups of k of one form, run in
    separate processes).  Groups of k of one form add their seconds: the form
    then answered all of them in that time, without the records the groups
    could have shared."""
    lines = [json.loads(open(p).read().strip().splitlines()[-1]) for p in paths]
    base = lines[0]
    tols = base["config"]["tols"]
    ks_all = sorted({k for ln in lines for k in ln["config"]["ks"]})
    forms = {}
    for ln in lines:
        if ln["config"]["tols"] != tols or ln["config"]["n"] != base["config"]["n"]:
            raise ValueError("query records of different workloads or tolerances")
        for name, rec in ln["forms"].items():
            dst = forms.setdefault(name, {})
            for k, r in rec.items():
                d = dst.setdefault(k, {"seconds": 0.0, "lam": {}, "evals_f64": 0, "evals_f32": 0, "max_bracket": 0.0})
                d["seconds"] += r["seconds"]
                d["evals_f64"] += r["evals_f64"]
                d["evals_f32"] += r["evals_f32"]
                d["max_bracket"] = max(d["max_bracket"], r["max_bracket"])
                d["lam"].update(dict(zip(ln["config"]["ks"], r["lambda"])))
    for name, rec in forms.items():
        for k, d in rec.items():
            if sorted(d["lam"]) != ks_all:
                raise ValueError("form %s at %s does not cover every k" % (name, k))
            d["lambda"] = [d["lam"][q] for q in ks_all]
            del d["lam"]
            d["eigvals_per_s"] = len(ks_all) / d["seconds"]
    line = dict(base)
    line["forms"] = forms
    line["config"] = dict(base["config"], ks=ks_all, merged_from=[os.path.basename(p) for p in paths])
    summarize_queries(line)
    print(json.dumps(line))


def cpu_baseline(n_sample: int = 4096, shifts: int = 4, n_target: int = 262144) -> dict:
    """The oracle as it stands, on the GPU host's cores, on a bounded sample."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from paper_2311_08618_amd import workloads as W
    from oracle.build import H2
    from oracle.factor import inertia
    from oracle.kernels import Kernel

    X = W.cube_points(n_sample, 0)
    H = H2(X, Kernel(W.K_LAPLACE, 1e3), 256, 1.0, 1e-8)
    sig = W.shift_grid(900.0, 1100.0, shifts, seed=1)
    t0 = time.perf_counter()
    for s in sig:
        inertia(H, float(s))
    dt = (time.perf_counter() - t0) / shifts
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    # the host's FP64 matrix-multiply rate through the same BLAS (best of 3,
    # 2048^3): context for the oracle's rate, whose block work runs on it
    M = np.random.default_rng(0).standard_normal((2048, 2048))
    best = math.inf
    for _ in range(3):
        t1 = time.perf_counter()
        M @ M
        best = min(best, time.perf_counter() - t1)
    return {
        "value": (1.0 / dt) * (n_sample / n_target),
        "unit": "evals/s",
        "cores": int(threads),
        "nproc": os.cpu_count(),
        "cpu_model": cpu_model,
        "host_dgemm_gflops": round(2.0 * 2048 ** 3 / best / 1e9, 1),
        "kind": "oracle",
        "sample": ("%d shifts of the oracle at n=%d (same kernel, leaf 256, eta 1, eps 1e-8), %.2f s per "
                   "shift, scaled linearly by n=%d/%d (the paper's O(n) per factorization; measured cost grows "
                   "faster than n here, so this favours the CPU)" % (shifts, n_sample, dt, n_sample, n_target)),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube-laplace", choices=sorted(WORKLOADS))
    ap.add_argument("--n", type=int, default=0, help="points (0 = the workload's size)")
    ap.add_argument("--batch", type=int, default=0, help="shifts per step (0 = the workload's default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--queries", action="store_true",
                    help="k-th eigenvalue queries: plain one-shift FP64 vs batched vs batched+mixed (uses --n)")
    ap.add_argument("--nq", type=int, default=4, help="eigenvalues for --queries (k = j n / nq)")
    ap.add_argument("--ks", default="", help="explicit comma list of k for --queries")
    ap.add_argument("--forms", default="", help="comma list of query forms (default: all): " + ",".join(QUERY_FORMS))
    ap.add_argument("--tol", default="1e-6,1e-10", help="comma list of absolute tolerances for --queries")
    ap.add_argument("--queries-merge", nargs="+", metavar="JSON", help="merge the lines of separate --queries runs")
    ap.add_argument("--serve", action="store_true", help="serving-loop measurement instead of the step bench")
    ap.add_argument("--serve-sizes", default="262144,131072,65536,16384")
    ap.add_argument("--serve-slots-max", type=int, default=16, help="most in-flight queries per matrix")
    ap.add_argument("--serve-rate", default="200", help="Poisson arrivals per second (comma list: a sweep)")
    ap.add_argument("--serve-window", type=float, default=1.0, help="seconds of arrivals")
    ap.add_argument("--serve-seed", type=int, default=7, help="seed of the arrivals of the first rate")
    ap.add_argument("--serve-cap", type=float, default=120.0,
                    help="seconds of drain after the arrival window until the measurement stops")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only (the batch of shifts is one GPU's share); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calib:
        copy_calibration(args.copy_calib)
        return
    if args.serve:
        serve_bench(args)
        return
    if args.queries_merge:
        merge_queries(args.queries_merge)
        return
    os.environ["H2EIG_PROGRESS"] = "1"       # h2_build reports each level (large constructions run for minutes)
    if args.queries:
        queries_bench(args)
        return

    from paper_2311_08618_amd import workloads as W
    from paper_2311_08618_amd.h2eig import H2Matrix

    n0, geom, kind, diag, leaf, eps, p0, p1, srange, S0 = WORKLOADS[args.workload]
    n, S = args.n or n0, args.batch or S0
    X = W.cube_points(n, 0) if geom == "cube" else W.cylinder_points(n, 0)
    t0 = time.perf_counter()
    A = H2Matrix(X, kind, diag, leaf, 1.0, eps, p0=p0, p1=p1, max_shifts=max(S, 1))
    build_s = time.perf_counter() - t0
    print("bench: built n=%d in %.1f s" % (n, build_s), file=sys.stderr, flush=True)
    if S == 0:
        # as many shifts per step as the device holds: one shift measures the
        # workspace of a shift, then the handle's capacity sets the batch
        A.inertia(W.shift_grid(srange[0], srange[1], 1, seed=0))
        A.set_max_shifts(0)
        S = A.capacity()
        A.set_max_shifts(S)
        print("bench: %d shift(s) per step" % S, file=sys.stderr, flush=True)
    sig = W.shift_grid(srange[0], srange[1], S, seed=0)
    for w in range(args.warmup):
        A.inertia(sig)
        print("bench: warmup %d done" % w, file=sys.stderr, flush=True)
    # timed steps: HIP events around the GEMM launches only (the dominant
    # kernel's live timing), so that instrumentation costs little
    A.profile_enable(2)
    t0 = time.perf_counter()
    for k in range(args.steps):
        nu = A.inertia(sig)          # returns after the device work is complete
        print("bench: step %d done" % k, file=sys.stderr, flush=True)
    dt = time.perf_counter() - t0
    prof = A.profile_read()
    A.profile_enable(False)
    st = A.stats()
    # one more step, outside the timed region, with every launch bracketed:
    # the time of each role of the factorization
    A.profile_enable(True)
    A.inertia(sig)
    roles_prof = A.profile_read()
    A.profile_enable(False)
    # the same shifts with the contractions in FP32 (h2_inertia_f32), outside
    # the timed region of `value`: its rate and whether its counts agree
    t1 = time.perf_counter()
    nu32 = A.inertia(sig, f32=True)
    dt32 = time.perf_counter() - t1
    print("bench: FP32 step done", file=sys.stderr, flush=True)

    evals = S * args.steps
    value = evals / dt
    # dominant kernel: the GEMM instantiation (operand layout) with the most live
    # HIP-event time; its algorithmic flops over that time
    kern = {k[len("kernel:"):]: v for k, v in prof.items() if k.startswith("kernel:")}
    roles = {k: v for k, v in roles_prof.items() if not k.startswith("kernel:")}
    kname, krec = max(kern.items(), key=lambda kv: kv[1]["ms"])
    achieved = krec["flops"] / (krec["ms"] * 1e-3) / 1e12 if krec["ms"] > 0 else 0.0
    cname, crec = max(roles.items(), key=lambda kv: kv[1]["ms"])
    roofline = {
        "bound": "mfma",
        "kernel": "h2::" + kname,
        "achieved": achieved,
        "peak": PEAK_FP64_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP64_TFLOPS,
        "traffic": measured_traffic("h2::" + kname, n, S),
        # the bytes its products must move at least (operands once, weights,
        # outputs read and written), per launch, from the device counters
        "algorithmic_bytes": krec.get("bytes", 0.0) / max(1, krec["launches"]),
        "launches": krec["launches"],
        "avg_launch_ms": krec["ms"] / max(1, krec["launches"]),
        "share_of_step": krec["ms"] / (dt * 1e3),
        "largest_role": {"name": cname, "ms": round(crec["ms"], 1),
                         "bound": "mfma" if cname in GEMM_CLASSES else "latency"},
    }
    if roofline["traffic"] and roofline["algorithmic_bytes"] > 0:
        roofline["traffic_over_algorithmic"] = roofline["traffic"] / roofline["algorithmic_bytes"]
    # algorithmic flops of the timed steps (the device counters run in both modes)
    total_flops = sum(v["flops"] for k, v in prof.items() if not k.startswith("kernel:"))
    # k-th eigenvalues per second implied by this rate: one query takes
    # ceil(log2((b - a) / tol)) bisection steps from the starting interval
    a0, b0 = A.interval()
    steps_q = {tol: math.ceil(math.log2((b0 - a0) / tol)) for tol in (1e-6, 1e-10)}
    line = {
        "metric": "H2 LDL+inertia evals/sec at n=2^18" if (args.workload, n) == ("cube-laplace", 1 << 18)
                  else "H2 LDL+inertia evals/sec",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s n=%d leaf=%d eta=1 eps=%g A_ii=%g%s, %d shift(s) per step in [%g, %g]"
                               % (args.workload, n, leaf, eps, diag, " p0=%g p1=%g" % (p0, p1) if p0 or p1 else "",
                                  S, srange[0], srange[1]),
                   "n": n, "shifts_per_step": S, "build_s": round(build_s, 2),
                   "resident_gb": round(st["resident_bytes"] / 1e9, 1)},
        "roofline": roofline,
        "path_tflops": total_flops / dt / 1e12,
        "kth_eigvals_per_s_derived": {"tol=%g" % t: value / s for t, s in steps_q.items()},
        "steps_per_query": {"tol=%g" % t: s for t, s in steps_q.items()},
        "max_cluster_dim": st["last_rank_max"],
        "workspace_gb": st["last_work_bytes"] / 1e9,
        "nu": [int(x) for x in nu],
        "f32_step": {"evals_per_s": S / dt32, "ms_per_step": dt32 * 1e3, "nu": [int(x) for x in nu32],
                     "counts_equal_f64": bool(list(nu32) == list(nu)),
                     "note": "rotation, elimination, Schur and merge contractions in FP32; recompression and "
                             "pivot LDL in FP64"},
        "classes_ms": {k: round(v["ms"], 1) for k, v in roles.items()},
        "classes_tflops": {k: round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 2) for k, v in roles.items()
                           if v["ms"] > 0 and v["flops"] > 0},
        "gemm_kernels_ms": {k: round(v["ms"], 1) for k, v in kern.items()},
    }
    if not args.no_cpu_baseline and args.workload == "cube-laplace":
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
