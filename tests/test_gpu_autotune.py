"""The GEMM tuning table and its autotuner on the GPU: the launch parameters
change only the speed, never a count, and a short tuning run produces a table
of valid entries that the binding can load."""
import json

import numpy as np
import pytest

from paper_2311_08618_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2311_08618_amd import h2eig
    return h2eig


def test_counts_do_not_depend_on_tuning(lib):
    print("case tuning-independence cube n=4096", flush=True)
    A = lib.H2Matrix(W.cube_points(4096, 2), W.K_LAPLACE, 1e3, 128, 1.0, 1e-8)
    sig = np.array([850.0, 990.0, 1000.0, 1010.0, 1300.0])
    ref = A.inertia(sig)
    ref32 = A.inertia(sig, f32=True)
    saved = {(l, f, b): lib.get_gemm_tuning(l, f, b) for l in range(4) for f in (0, 1) for b in range(5)}
    try:
        for g, gm, t in [(8, 1, 64), (512, 8, 64), (4096, 3, 64), (256, 1, 128), (1024, 8, 128)]:
            for key in saved:
                lib.set_gemm_tuning(*key, g, gm, t)
            assert np.array_equal(A.inertia(sig), ref), (g, gm, t)
            assert np.array_equal(A.inertia(sig, f32=True), ref32), (g, gm, t)
    finally:
        for key, val in saved.items():
            lib.set_gemm_tuning(*key, *val)


def test_short_autotune_writes_a_loadable_table(lib, tmp_path):
    print("case autotune n=4096", flush=True)
    from paper_2311_08618_amd import autotune
    saved = {(l, f, b): lib.get_gemm_tuning(l, f, b) for l in range(4) for f in (0, 1) for b in range(5)}
    table = autotune.tune(n=4096, reps=1, grids=[1024, 2048], groups=[1], tiles=[64, 128], log=lambda s: None)
    assert table["entries"]
    for e in table["entries"]:
        assert e["grid"] in (1024, 2048) and e["group_m"] == 1 and e["tile"] in (64, 128)
        assert 0 <= e["layout"] <= 3 and e["f32"] in (0, 1) and 0 <= e["bucket"] <= 4
    # the tuner leaves the table as it found it
    assert {k: lib.get_gemm_tuning(*k) for k in saved} == saved
    p = tmp_path / "t.json"
    p.write_text(json.dumps(table))
    try:
        assert lib.apply_tuning(str(p)) == len(table["entries"])
        e = table["entries"][0]
        assert lib.get_gemm_tuning(e["layout"], e["f32"], e["bucket"]) == (e["grid"], e["group_m"], e["tile"])
    finally:
        for key, val in saved.items():
            lib.set_gemm_tuning(*key, *val)
