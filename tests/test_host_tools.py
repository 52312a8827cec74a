"""Host-side logic of the measurement and tuning tools (no device work):
the autotuner's mapping of profiler symbols and capacities to table entries,
and the bench's use of a committed counter record only while it matches the
kernel, the workload and the kernel source."""
import hashlib
import os
import re

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
    src.write_text("// kernel source\n")
    h = hashlib.sha256(src.read_bytes()).hexdigest()[:16]
    rec = tmp_path / "traffic.md"
    rec.write_text("# counters\n\n- kernel: h2::k_gemm<false, true>\n- n: 262144\n- shifts_per_step: 2\n"
                   "- kernels_hip_sha256_16: %s\n- hbm_bytes_per_launch: 1.5e+09\n" % h)
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(rec))
    assert bench.measured_traffic("h2::k_gemm<false, true>", 262144, 2) == 1.5e9
    assert bench.measured_traffic("h2::k_gemm<true, false>", 262144, 2) is None
    assert bench.measured_traffic("h2::k_gemm<false, true>", 131072, 2) is None
    assert bench.measured_traffic("h2::k_gemm<false, true>", 262144, 1) is None
    src.write_text("// changed kernel source\n")
    assert bench.measured_traffic("h2::k_gemm<false, true>", 262144, 2) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic("h2::k_gemm<false, true>", 262144, 2) is None


def test_committed_traffic_record_matches_committed_kernels():
    """The committed counter record is used only while it was taken on the
    committed kernel source (otherwise the bench reports traffic as null)."""
    import bench
    if not os.path.exists(bench.TRAFFIC_FILE):
        pytest.skip("no counter record")
    txt = open(bench.TRAFFIC_FILE).read()
    h = hashlib.sha256(open(bench.KERNEL_SOURCE, "rb").read()).hexdigest()[:16]
    if h not in txt:
        pytest.skip("counter record predates the current kernels.hip: traffic is reported as null")
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
