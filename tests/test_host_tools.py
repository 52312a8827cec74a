"""Host-side logic (no device work): the autotuner's mapping of profiler
symbols and capacities to table entries, the bench's use of a committed counter
record only while it matches the GEMM's code and the workload, the merge of
separate query runs, and the library's own host code against the oracle (the
inertia-record cache, the cluster tree, the norm and kernel entries, the static
schedule), also under sanitizers."""
import math
import os
import re

import numpy as np
import pytest


@pytest.fixture(scope="module")
def autotune():
    from paper_2311_08618_amd import autotune
    return autotune


def test_symbol_mapping(autotune):
    assert autotune.symbol("kernel:k_gemm<false, false>") == (0, 0)
    assert autotune.symbol("kernel:k_gemm<false, true>") == (1, 0)
    assert autotune.symbol("kernel:k_gemm<true, false>") == (2, 0)
    assert autotune.symbol("kernel:k_gemm_f32<false, true>") == (1, 1)
    assert autotune.symbol("kernel:k_gemm128<true, false>") == (2, 0)
    assert autotune.symbol("kernel:k_gemm128_f32<true, true>") == (3, 1)
    assert autotune.symbol("schur") is None
    assert autotune.symbol("kernel:k_other<false, true>") is None


def test_bucket_boundaries(autotune):
    from paper_2311_08618_amd import h2eig
    for cap, b in [(8, 0), (256, 0), (257, 1), (512, 1), (1024, 2), (1025, 3), (2048, 3), (2049, 4), (5000, 4)]:
        assert autotune.bucket_of(cap) == b, cap
    # the library's table has an entry for every (layout, precision, bucket)
    for layout in range(4):
        for f32 in (0, 1):
            for b in range(5):
                g, gm, t = h2eig.get_gemm_tuning(layout, f32, b)
                assert g % 8 == 0 and gm >= 1 and t in (64, 128)


def test_traffic_record_validity(tmp_path, monkeypatch):
    import bench
    src = tmp_path / "kernels.hip"
    src.write_text("// head\n// GEMM (FP64 MFMA)\ngemm kernels\n// matrix sums\nother kernels\n"
                   "void launch_variant(gemm launchers)\nvoid launch_copyback(other launchers)\n")
    desc, tune = tmp_path / "desc.hpp", tmp_path / "tuning.json"
    desc.write_text("struct GItem;\n")
    tune.write_text("{}\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    monkeypatch.setattr(bench, "GEMM_SOURCES", [str(desc), str(tune)])
    h = bench.gemm_source_hash()
    rec = tmp_path / "traffic.md"
    rec.write_text("# counters\n\n- kernel: h2::k_gemm<false, true>\n- n: 262144\n- shifts_per_step: 2\n"
                   "- gemm_source_sha256_16: %s\n- hbm_bytes_per_launch: 1.5e+09\n" % h)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(rec))
    assert bench.measured_traffic("h2::k_gemm<false, true>", 262144, 2) == 1.5e9
    assert bench.measured_traffic("h2::k_gemm<true, false>", 262144, 2) is None
    assert bench.measured_traffic("h2::k_gemm<false, true>", 131072, 2) is None
    assert bench.measured_traffic("h2::k_gemm<false, true>", 262144, 1) is None
    # a change outside the GEMM section keeps the record; inside it, in its
    # launchers, the descriptors or the table, drops it
    src.write_text(src.read_text().replace("other kernels", "changed recompression kernels"))
    assert bench.measured_traffic("h2::k_gemm<false, true>", 262144, 2) == 1.5e9
    for path, a, b in [(src, "gemm kernels", "gemm kernels changed"), (src, "gemm launchers", "new launchers"),
                       (desc, "GItem", "GItem2"), (tune, "{}", "{\"a\": 1}")]:
        old = path.read_text()
        path.write_text(old.replace(a, b))
        assert bench.measured_traffic("h2::k_gemm<false, true>", 262144, 2) is None, (path, a)
        path.write_text(old)
    assert bench.measured_traffic("h2::k_gemm<false, true>", 262144, 2) == 1.5e9
    src.write_text("// no markers\n")
    assert bench.measured_traffic("h2::k_gemm<false, true>", 262144, 2) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic("h2::k_gemm<false, true>", 262144, 2) is None


def test_committed_traffic_record_matches_committed_kernels():
    """The committed counter record is used only while it was taken on the
    committed GEMM code (otherwise the bench reports traffic as null)."""
    import bench
    if not os.path.exists(bench.TRAFFIC_FILE):
        pytest.skip("no counter record")
    txt = open(bench.TRAFFIC_FILE).read()
    if bench.gemm_source_hash() not in txt:
        pytest.skip("counter record predates the current GEMM code: traffic is reported as null")
    fields = dict(re.findall(r"^- (\w+): (.+)$", txt, flags=re.M))
    kernel, n, S = fields["kernel"].strip(), int(fields["n"]), int(fields["shifts_per_step"])
    assert kernel.startswith("h2::k_gemm")
    got = bench.measured_traffic(kernel, n, S)
    assert got is not None and got > 0
    # the stored total is the two scaled counters
    want = 1024.0 * (float(fields["fetch_kib_per_dispatch"]) * float(fields["fetch_scale"])
                     + float(fields["write_kib_per_dispatch"]) * float(fields["write_scale"]))
    assert abs(got - want) <= 1e-3 * want
    assert bench.measured_traffic(kernel, n + 1, S) is None and bench.measured_traffic(kernel, n, S + 1) is None


def _query_line(forms, ks, tols=(1e-6, 1e-10)):
    return {"metric": "q", "value": None, "forms": forms,
            "config": {"n": 1000, "ks": list(ks), "tols": list(tols), "normA": 1.0, "interval": [0.0, 1.0]}}


def _rec(seconds, lam, f64=10, f32=0):
    return {"seconds": seconds, "eigvals_per_s": len(lam) / seconds, "lambda": list(lam), "max_bracket": 1e-12,
            "evals_f64": f64, "evals_f32": f32}


def test_query_merge_adds_groups_and_orders_by_k(tmp_path, capsys):
    """Groups of k of one form run in separate processes add their seconds and
    their eigenvalues land at their k; the largest |delta lambda| and the
    speedups are taken against the plain form at every tolerance."""
    import json
    import bench
    a = _query_line({"plain_f64_1shift": {"tol=1e-06": _rec(10.0, [1.0, 3.0]), "tol=1e-10": _rec(14.0, [1.0, 3.0])}},
                    [1, 500])
    b = _query_line({"plain_f64_1shift": {"tol=1e-06": _rec(20.0, [2.0, 4.0]), "tol=1e-10": _rec(26.0, [2.0, 4.0])}},
                    [250, 750])
    c = _query_line({"batched_f64": {"tol=1e-06": _rec(15.0, [1.0, 2.0, 3.0, 4.5]),
                                     "tol=1e-10": _rec(20.0, [1.0, 2.0, 3.0, 4.0])}}, [1, 250, 500, 750])
    paths = []
    for name, ln in (("a", a), ("b", b), ("c", c)):
        p = tmp_path / (name + ".json")
        p.write_text(json.dumps(ln) + "\n")
        paths.append(str(p))
    bench.merge_queries(paths)
    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert out["config"]["ks"] == [1, 250, 500, 750]
    plain = out["forms"]["plain_f64_1shift"]
    assert plain["tol=1e-06"]["seconds"] == 30.0 and plain["tol=1e-10"]["seconds"] == 40.0
    assert plain["tol=1e-06"]["lambda"] == [1.0, 2.0, 3.0, 4.0]
    assert plain["tol=1e-06"]["evals_f64"] == 20
    d = out["max_abs_dlambda_vs_plain"]["batched_f64"]
    assert d["tol=1e-06"] == 0.5 and d["tol=1e-10"] == 0.0
    sp = out["speedup_vs_plain"]["batched_f64"]
    assert abs(sp["tol=1e-06"] - 2.0) < 1e-12 and abs(sp["tol=1e-10"] - 2.0) < 1e-12
    assert out["value"] == 4 / 20.0


def test_query_merge_rejects_mixed_workloads(tmp_path):
    import json
    import bench
    a = _query_line({"batched_f64": {"tol=1e-06": _rec(1.0, [1.0])}}, [1], tols=(1e-6,))
    b = _query_line({"batched_f64": {"tol=1e-06": _rec(1.0, [1.0])}}, [2], tols=(1e-8,))
    pa, pb = tmp_path / "a.json", tmp_path / "b.json"
    pa.write_text(json.dumps(a))
    pb.write_text(json.dumps(b))
    with pytest.raises(ValueError):
        bench.merge_queries([str(pa), str(pb)])


def test_inertia_record_cache(tmp_path):
    """The record cache shared by h2_kth_eig and the serving loop
    (csrc/records.hpp): a C++ harness compares brackets from the compacted list
    with brackets from every record ever inserted (Sec. 4.2's inertia reuse)."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    here = os.path.dirname(os.path.abspath(__file__))
    exe = str(tmp_path / "records_check")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror", "-o", exe,
                    os.path.join(here, "records_check.cpp")], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr


def _tree_cases():
    """(name, points, leaf, eta, kernel (kind, diag, p0, p1))"""
    from paper_2311_08618_amd import workloads as W
    rng = np.random.default_rng(11)
    grid = np.array([[x, y] for x in range(12) for y in range(9)], dtype=np.float64) * 0.5
    return [
        ("cube-300-leaf32", W.cube_points(300, 1), 32, 1.0, (W.K_LAPLACE, 1e3, 0.0, 0.0)),
        ("cube-2000-leaf64-eta0.7", W.cube_points(2000, 0), 64, 0.7, (W.K_YUKAWA, 1e3, 0.0, 0.0)),
        ("circle-512-leaf32", W.circle_points(512), 32, 1.0, (W.K_REG_LAPLACE, 1e3, 1e-3, 0.0)),
        ("line-700-leaf64", W.line_points(700), 64, 1.0, (W.K_TRIDIAG_1D, 2.0, 1.0, 0.0)),
        ("cylinders-1024-leaf64", W.cylinder_points(1024, 0), 64, 1.0, (W.K_GAUSS_DAMPED, 10.0, 0.01, 0.01)),
        ("cube-1000-weak", W.cube_points(1000, 2), 64, math.inf, (W.K_LAPLACE, 1e3, 0.0, 0.0)),
        ("grid-ties-108-leaf4", grid, 4, 1.0, (W.K_YUKAWA, 5.0, 0.0, 0.0)),
        ("duplicates-96-leaf8", np.repeat(rng.random((24, 3)), 4, axis=0), 8, 1.0, (W.K_REG_LAPLACE, 50.0, 0.1, 0.0)),
        ("single-point", np.zeros((1, 3)), 2, 1.0, (W.K_LAPLACE, 1e3, 0.0, 0.0)),
        ("ragged-37-leaf5", rng.random((37, 2)), 5, 1.0, (W.K_GAUSS_DAMPED, 3.0, 0.5, 0.1)),
    ]


@pytest.fixture(scope="module")
def tree_exe(tmp_path_factory):
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    lib = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2311_08618_amd",
                       "libh2eig.so")
    if gxx is None:
        pytest.skip("g++ not found")
    assert os.path.exists(lib), "libh2eig.so is not built (run __graft_entry__.build())"
    here = os.path.dirname(os.path.abspath(__file__))
    exe = str(tmp_path_factory.mktemp("tree") / "tree_check")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", "-o", exe, os.path.join(here, "tree_check.cpp"),
                    "-L" + os.path.dirname(lib), "-l:libh2eig.so", "-Wl,-rpath," + os.path.dirname(lib)],
                   check=True)
    return exe


@pytest.mark.parametrize("case", _tree_cases(), ids=lambda c: c[0])
def test_library_tree_equals_oracle(tree_exe, case):
    """The library's host code, without a GPU, against the oracle: its cluster
    tree, block tree and colouring equal the oracle's index for index (median
    split of the longest axis, strong admissibility, near and interaction
    lists, greedy colouring; Secs. 3.1 and 3.4) with the leaf-order
    permutation; its normA (the scale of every truncation tolerance) equals the
    oracle's to summation order; its kernel entries to a few ulps."""
    import subprocess
    from oracle.build import estimate_norm
    from oracle.kernels import Kernel
    from oracle.tree import Tree
    name, X, leaf, eta, (kind, diag, p0, p1) = case
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X.reshape(-1, 1)
    n, dim = X.shape
    inp = ("%d %d %d %r %d %r %r %r\n" % (n, dim, leaf, eta, kind, diag, p0, p1)
           + " ".join("%.17g" % v for v in X.ravel()) + "\n")
    out = subprocess.run([tree_exe], input=inp, capture_output=True, text=True, timeout=120, check=True).stdout
    T = Tree(X, leaf, eta)
    got, kb = {}, []
    for line in out.splitlines():
        tok = line.split()
        if tok[0] == "L":
            got["L"] = int(tok[1])
        elif tok[0] == "norm":
            got["norm"] = float(tok[1])
        elif tok[0] == "kblock":
            kb.append([float(v) for v in tok[2:]])
        else:
            got[(tok[0], int(tok[1]), int(tok[2]))] = [int(v) for v in tok[3:]]
    assert got["L"] == T.L
    for l in range(T.L + 1):
        assert got[("colour", l, -1)] == list(T.colour[l]), (name, l)
        for i in range(1 << l):
            assert got[("idx", l, i)] == [int(v) for v in T.idx[l][i]], (name, l, i)
            assert got[("near", l, i)] == list(T.near[l][i]), (name, l, i)
            assert got[("far", l, i)] == list(T.far[l][i]), (name, l, i)
    assert got[("perm", -1, -1)] == [int(v) for v in T.perm()]
    k = Kernel(kind, diag, p0, p1)
    assert abs(got["norm"] - estimate_norm(X, k)) <= 1e-12 * abs(estimate_norm(X, k)), (got["norm"],)
    m = min(n, 24)
    ids = np.arange(m)
    want = k.block(X, ids, ids)
    # a few ulps, times the kernel's condition number |d log f / d log r| at
    # that distance (the two sides may round r differently by an ulp)
    d = X[:m, None, :] - X[None, :m, :]
    r = np.sqrt(np.sum(d * d, axis=2))
    h = 1e-6
    with np.errstate(divide="ignore", invalid="ignore"):
        cond = np.abs((k.f(r * (1 + h)) - k.f(r * (1 - h))) / (2 * h * k.f(r)))
    cond = np.where(np.isfinite(cond), cond, 0.0)
    tol = 8e-16 * (2.0 + cond) * np.abs(want)
    got_kb = np.array(kb)
    assert got_kb.shape == want.shape and np.all(np.abs(got_kb - want) <= tol), name


def test_host_code_under_sanitizers(tree_exe, plan_exe, matvec_exe, tmp_path):
    """The host code shared by the harnesses, built with the address and
    undefined-behaviour sanitizers (any report is fatal) and, separately, with
    the thread sanitizer: the record cache, the library's host.cpp (tree,
    threaded norm estimate, kernel entries, threaded H^2 matvec) and plan.cpp
    (the static schedule) run clean and print what the plain build prints.  Host code only; no device
    code is built here."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    here = os.path.dirname(os.path.abspath(__file__))
    libdir = os.path.join(os.path.dirname(here), "paper_2311_08618_amd")
    common = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
    link = ["-L" + libdir, "-l:libh2eig.so", "-Wl,-rpath," + libdir, "-pthread"]
    san = {"asan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
           "tsan": ["-fsanitize=thread"]}
    from paper_2311_08618_amd import workloads as W
    X = W.cube_points(2000, 1)
    inp = "2000 3 64 0.7 %d 1000.0 0.0 0.0\n" % W.K_YUKAWA + " ".join("%.17g" % v for v in X.ravel()) + "\n"
    plain = subprocess.run([tree_exe], input=inp, capture_output=True, text=True, timeout=120, check=True).stdout
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", TSAN_OPTIONS="halt_on_error=1")
    plan_inp = inp.split("\n", 1)
    plan_inp = " ".join(plan_inp[0].split()[:4]) + "\n" + plan_inp[1]
    plain_plan = subprocess.run([plan_exe], input=plan_inp, capture_output=True, text=True, timeout=120,
                                check=True).stdout
    # the library sources as instrumented objects, compiled side by side; plan.cpp
    # runs on one thread, so the thread sanitizer covers the tree harness only
    objs = {("host.cpp", "asan"), ("plan.cpp", "asan"), ("host.cpp", "tsan")}
    procs = {}
    for src, name in objs:
        obj = str(tmp_path / ("%s_%s.o" % (src[:-4], name)))
        procs[(src, name)] = (obj, subprocess.Popen([gxx] + common + san[name] + ["-c", "-o", obj,
                                                                                   os.path.join(libdir, "csrc", src)]))
    for key, (obj, pr) in procs.items():
        assert pr.wait(timeout=600) == 0, key
    mv_inp = _matvec_input(300, 32, W.K_LAPLACE, 1e-6, 2)[0]
    plain_mv = subprocess.run([matvec_exe], input=mv_inp, capture_output=True, text=True, timeout=120,
                              check=True).stdout
    runs = [("tree", "asan", ["host.cpp"], inp, plain), ("plan", "asan", ["plan.cpp", "host.cpp"], plan_inp, plain_plan),
            ("matvec", "asan", ["host.cpp"], mv_inp, plain_mv), ("tree", "tsan", ["host.cpp"], inp, plain),
            ("matvec", "tsan", ["host.cpp"], mv_inp, plain_mv)]
    for harness, name, srcs, text, want in runs:
        exe = str(tmp_path / (harness + "_" + name))
        subprocess.run([gxx] + common + san[name] + ["-o", exe, os.path.join(here, harness + "_check.cpp")]
                       + [procs[(f, name)][0] for f in srcs] + link, check=True)
        out = subprocess.run([exe], input=text, capture_output=True, text=True, timeout=300, env=env)
        assert out.returncode == 0 and "Sanitizer" not in out.stderr, (name, harness, out.stderr[-2000:])
        assert out.stdout == want, (name, harness)
    exe = str(tmp_path / "records_asan")
    subprocess.run([gxx] + common + san["asan"] + ["-o", exe, os.path.join(here, "records_check.cpp")], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr[-2000:]


@pytest.fixture(scope="module")
def plan_exe(tree_exe, tmp_path_factory):
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    here = os.path.dirname(os.path.abspath(__file__))
    libdir = os.path.join(os.path.dirname(here), "paper_2311_08618_amd")
    exe = str(tmp_path_factory.mktemp("plan") / "plan_check")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", "-o", exe, os.path.join(here, "plan_check.cpp"),
                    "-L" + libdir, "-l:libh2eig.so", "-Wl,-rpath," + libdir], check=True)
    return exe


@pytest.mark.parametrize("n,leaf,eta,seed", [(2048, 128, 1.0, 0), (1000, 64, 1.5, 3)])
def test_library_schedule_carries_the_oracles_fill_in(plan_exe, n, leaf, eta, seed):
    """The library's static schedule (host code, no GPU) against the oracle's
    factorization (Secs. 3.3-3.4): the near-pair rows are the tree's near lists,
    the colour classes partition each level into pairwise non-near clusters in
    the oracle's colouring, and the fill-in blocks the schedule carries into
    each level are exactly the pairs on which the oracle's elimination of the
    level below left fill-in that its merge carries up (parents not near)."""
    import subprocess
    from oracle import factor as OF
    from oracle.build import H2
    from oracle.kernels import Kernel
    from paper_2311_08618_amd import workloads as W
    X = W.cube_points(n, seed)
    inp = "%d 3 %d %r\n" % (n, leaf, eta) + " ".join("%.17g" % v for v in X.ravel()) + "\n"
    out = subprocess.run([plan_exe], input=inp, capture_output=True, text=True, timeout=120, check=True).stdout
    got = {}
    for line in out.splitlines():
        tok = line.split()
        if tok[0] != "L":
            got[(tok[0], int(tok[1]), int(tok[2]))] = [int(v) for v in tok[3:]]
    H = H2(X, Kernel(W.K_LAPLACE, 1e3), leaf, eta, 1e-6)
    T = H.tree
    fkeys, allR = {}, {}

    def hook(l, nu, S, F, m, R):
        fkeys[l] = set(F.keys())
        allR[l] = list(R)

    OF.inertia(H, 1000.0, on_level=hook)
    for l in range(T.L + 1):
        N = 1 << l
        for i in range(N):
            assert got[("near", l, i)] == list(T.near[l][i]), (l, i)
        classes = [got[("class", l, c)] for c in range(max(T.colour[l]) + 1)]
        assert sorted(i for cl in classes for i in cl) == list(range(N))
        for c, cl in enumerate(classes):
            assert cl == [i for i in range(N) if T.colour[l][i] == c], (l, c)
            assert all(b not in T.near_set[l][a] for a in cl for b in cl if a != b), (l, c)
        if l == T.L:
            assert all(got[("carried", l, i)] == [] for i in range(N))
            continue
        # the oracle creates fill-in only behind clusters with a pivot block
        # (R > 0); the schedule lays it out for every cluster
        carried = {(min(c >> 1, d >> 1), max(c >> 1, d >> 1)) for (c, d) in fkeys[l + 1]
                   if (d >> 1) not in T.near_set[l][c >> 1]}
        sched = {(i, j) for i in range(N) for j in got[("carried", l, i)]}
        if all(r > 0 for r in allR[l + 1]):
            assert sched == carried, (l, sorted(sched ^ carried)[:10])
        else:
            assert carried <= sched, l
    assert any(got[("carried", l, i)] for l in range(T.L) for i in range(1 << l))   # fill-in is carried somewhere


def test_host_sources_compile_without_warnings():
    """The library's host C++ (tree and bases, schedule, level engine and C ABI,
    serving loop) is clean under g++ -Wall -Wextra."""
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    csrc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2311_08618_amd", "csrc")
    procs = [(f, subprocess.Popen([gxx, "-std=c++17", "-fsyntax-only", "-Wall", "-Wextra", "-Werror",
                                   "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", os.path.join(csrc, f)],
                                  stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
             for f in ("host.cpp", "plan.cpp", "engine.cpp", "server.cpp")]
    for f, pr in procs:
        out, err = pr.communicate(timeout=300)
        assert pr.returncode == 0, (f, err[-3000:])


def _matvec_input(n, leaf, kind, eps, seed):
    """Input of tests/matvec_check.cpp for the oracle's H^2 matrix of n cube
    points: (text, oracle H2, kernel, points, x)."""
    from oracle.build import H2
    from oracle.kernels import Kernel
    from paper_2311_08618_amd import workloads as W
    X = W.cube_points(n, seed)
    k = Kernel(kind, 1e3)
    H = H2(X, k, leaf, 1.0, eps)
    L = H.tree.L
    parts = ["%d 3 %d %r %d %r 0 0\n" % (n, leaf, 1.0, kind, 1e3), " ".join("%.17g" % v for v in X.ravel()), "\n"]
    for l in range(1, L + 1):
        for i in range(1 << l):
            Q = np.asarray(H.Q[l][i])
            m, r = H.m[l][i], H.r[l][i]
            assert Q.shape == (m, m)
            parts.append("%d %d\n" % (m, r))
            parts.append(" ".join("%.17g" % v for v in Q.ravel(order="F")) + "\n")
            cpl = [(j, np.asarray(H.C[l][(i, j)])) for j in H.tree.far[l][i]]
            parts.append("%d\n" % len(cpl))
            for j, C in cpl:
                parts.append("%d %d " % (j, H.r[l][j]) + " ".join("%.17g" % v for v in C.ravel(order="F")) + "\n")
    x = np.random.default_rng(seed + 1).standard_normal(n)
    parts.append(" ".join("%.17g" % v for v in x) + "\n")
    return "".join(parts), H, k, X, x


@pytest.fixture(scope="module")
def matvec_exe(tree_exe, tmp_path_factory):
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    here = os.path.dirname(os.path.abspath(__file__))
    libdir = os.path.join(os.path.dirname(here), "paper_2311_08618_amd")
    exe = str(tmp_path_factory.mktemp("matvec") / "matvec_check")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", "-o", exe, os.path.join(here, "matvec_check.cpp"),
                    "-L" + libdir, "-l:libh2eig.so", "-Wl,-rpath," + libdir], check=True)
    return exe


@pytest.mark.parametrize("n,leaf,kind,eps,seed", [(1024, 64, 0, 1e-6, 0), (700, 32, 1, 1e-9, 4)])
def test_library_host_matvec_equals_oracle_dense(matvec_exe, n, leaf, kind, eps, seed):
    """The library's host H^2 matvec (the diagnostic behind h2_matvec, with
    which the GPU tests measure ||A - A~||) applied to the oracle's bases,
    transfer matrices and couplings equals the oracle's densely assembled A~
    times x to rounding: both read the nested bases of Sec. 3.1 the same way
    (skeleton columns last, transfer matrices on the children's skeletons,
    couplings between skeletons), and the library adds the exact near field."""
    import subprocess
    text, H, k, X, x = _matvec_input(n, leaf, kind, eps, seed)
    out = subprocess.run([matvec_exe], input=text, capture_output=True, text=True, timeout=300, check=True).stdout
    y = np.array([float(v) for v in out.split()])
    want = H.dense() @ x
    assert y.shape == want.shape
    assert np.linalg.norm(y - want) <= 1e-13 * np.linalg.norm(want), np.linalg.norm(y - want) / np.linalg.norm(want)
    # and it is the H^2 matrix, not the exact one: the difference is the construction error
    exact = k.dense(X) @ x
    assert 0.0 < np.linalg.norm(y - exact) <= 10 * eps * H.normA * np.linalg.norm(x)
