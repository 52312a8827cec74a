"""The C-ABI boundary without a GPU: the library loads, exports every symbol
that include/h2eig.h declares, and rejects invalid arguments with H2_EINVAL
(and H2_EDEVICE when no GPU is present) before any device work."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "h2eig.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:h2_status|int32_t|const char\*|void)\s+(h2s?_\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def mod():
    from paper_2311_08618_amd import h2eig
    return h2eig


def test_header_symbols_exported(mod):
    names = _declared()
    assert len(names) >= 10
    for nm in names:
        assert hasattr(mod._lib, nm), nm          # dlsym succeeds
    assert sorted(mod.EXPORTED) == names


def _build(mod, pts, n, dim, kind=0, diag=1e3, leaf=8, eta=1.0, eps=1e-8, p0=0.0, p1=0.0):
    kern = mod._Kernel(kind, diag, p0, p1)
    h = C.c_void_p()
    arr = np.ascontiguousarray(pts, dtype=np.float64)
    ptr = arr.ctypes.data_as(C.POINTER(C.c_double)) if arr.size else None
    return mod._lib.h2_build(ptr, n, dim, kern, leaf, eta, eps, None, C.byref(h)), h


@pytest.mark.parametrize("case", ["n0", "dim0", "dim4", "leaf1", "eps0", "eta_neg", "kind7", "nan_point",
                                  "inf_diag", "gauss_p0", "tridiag_p0"])
def test_build_rejects_invalid(mod, case):
    X = np.random.default_rng(0).random((16, 3))
    args = dict(pts=X, n=16, dim=3)
    kw = {}
    if case == "n0":
        args["n"] = 0
    elif case == "dim0":
        args["dim"] = 0
    elif case == "dim4":
        args["dim"] = 4
    elif case == "leaf1":
        kw["leaf"] = 1
    elif case == "eps0":
        kw["eps"] = 0.0
    elif case == "eta_neg":
        kw["eta"] = -1.0
    elif case == "kind7":
        kw["kind"] = 7
    elif case == "nan_point":
        X = X.copy()
        X[3, 1] = math.nan
        args["pts"] = X
    elif case == "inf_diag":
        kw["diag"] = math.inf
    elif case == "gauss_p0":
        kw.update(kind=2, p0=0.0, p1=0.01)
    elif case == "tridiag_p0":
        kw.update(kind=4, p0=0.0)
    st, h = _build(mod, args["pts"], args["n"], args["dim"], **kw)
    assert st == mod.H2_EINVAL, (case, st)
    assert not h.value
    assert len(mod._lib.h2_last_error()) > 0


def test_null_handles(mod):
    L = mod._lib
    nu = (C.c_int64 * 1)()
    sig = (C.c_double * 1)(1.0)
    assert L.h2_inertia(None, sig, 1, nu, None) == mod.H2_EINVAL
    assert L.h2_inertia_f32(None, sig, 1, nu, None) == mod.H2_EINVAL
    assert L.h2_set_mixed(None, 1e-4) == mod.H2_EINVAL
    assert L.h2_level_dims(None, 1, None) == mod.H2_EINVAL
    k = (C.c_int64 * 1)(1)
    lam = (C.c_double * 1)()
    assert L.h2_kth_eig(None, k, 1, 1e-8, None, lam, None) == mod.H2_EINVAL
    x = C.c_double()
    assert L.h2_norm(None, C.byref(x)) == mod.H2_EINVAL
    assert L.h2_tree_perm(None, None) == mod.H2_EINVAL
    assert L.h2_profile_enable(None, 1) == mod.H2_EINVAL
    assert L.h2_profile_bytes(None, 0, C.byref(x)) == mod.H2_EINVAL
    assert L.h2_profile_read(None, 0, None, None, None) == mod.H2_EINVAL
    assert L.h2_release_workspace(None) == mod.H2_EINVAL
    L.h2_free(None)   # no-op


def test_profile_class_names(mod):
    L = mod._lib
    n = L.h2_profile_classes()
    names = [L.h2_profile_class_name(c).decode() for c in range(n)]
    assert all(names) and len(set(names)) == n
    assert any(s.startswith("kernel:k_gemm") for s in names)
    assert L.h2_profile_class_name(-1).decode() == "" and L.h2_profile_class_name(n).decode() == ""


def test_build_without_gpu_is_edevice(mod):
    X = np.random.default_rng(0).random((64, 3))
    st, h = _build(mod, X, 64, 3)
    if st == mod.H2_OK:   # a GPU is present: nothing to check here
        mod._lib.h2_free(h)
        pytest.skip("a GPU is present")
    assert st == mod.H2_EDEVICE, st


def test_server_argument_errors(mod):
    """The serving loop's calls reject bad arguments before any device work;
    a server with no matrices starts and stops cleanly."""
    L = mod._lib
    h = C.c_void_p()
    assert L.h2s_create(0, -1, C.byref(h)) == mod.H2_EINVAL
    assert L.h2s_create(-5, 0, C.byref(h)) == mod.H2_EINVAL
    assert L.h2s_create(0, 0, None) == mod.H2_EINVAL
    assert L.h2s_create(1 << 30, 4, C.byref(h)) == mod.H2_OK and h.value   # explicit budget: no device query
    i = C.c_int32()
    t = C.c_int64()
    lam = C.c_double()
    done = C.c_int32()
    assert L.h2s_add(h, None, 0, C.byref(i)) == mod.H2_EINVAL
    assert L.h2s_add(None, None, 0, C.byref(i)) == mod.H2_EINVAL
    assert L.h2_set_max_shifts(None, 1) == mod.H2_EINVAL
    assert L.h2_interval(None, None) == mod.H2_EINVAL
    assert L.h2_capacity(None, None) == mod.H2_EINVAL
    assert L.h2s_submit(h, 0, 1, 1e-8, C.byref(t)) == mod.H2_EINVAL       # no matrix 0
    assert L.h2s_submit(h, 0, 1, 0.0, C.byref(t)) == mod.H2_EINVAL
    assert L.h2s_poll(h, 1, C.byref(lam), C.byref(done)) == mod.H2_EINVAL  # unknown ticket
    assert L.h2s_wait(h, 7, C.byref(lam)) == mod.H2_EINVAL
    p50, p99 = C.c_double(-1), C.c_double(-1)
    served, sub = C.c_int64(-1), C.c_int64(-1)
    assert L.h2s_stats(h, C.byref(p50), C.byref(p99), C.byref(served), C.byref(sub)) == mod.H2_OK
    assert (p50.value, p99.value, served.value, sub.value) == (0.0, 0.0, 0, 0)
    open_, budget, used = C.c_int64(-1), C.c_int64(-1), C.c_int64(-1)
    assert L.h2s_latency(None, None, None, None, None, None) == mod.H2_EINVAL
    assert L.h2s_latency(h, C.byref(p50), C.byref(p99), C.byref(open_), C.byref(budget), C.byref(used)) == mod.H2_OK
    assert (open_.value, budget.value, used.value) == (0, 1 << 30, 0)
    assert L.h2_release_workspace(None) == mod.H2_EINVAL
    L.h2s_destroy(h)
    L.h2s_destroy(None)   # no-op


def test_gemm_tuning_table(mod):
    """The tuning table validates its arguments and round-trips an entry
    (host only: no device work)."""
    L = mod._lib
    g0, gm0, t0 = mod.get_gemm_tuning(1, 0, 3)
    assert g0 % 8 == 0 and g0 >= 8 and gm0 >= 1 and t0 in (64, 128)
    for bad in [(4, 0, 0, 1024, 1, 64), (0, 2, 0, 1024, 1, 64), (0, 0, 5, 1024, 1, 64), (0, 0, 0, 1001, 1, 64),
                (0, 0, 0, 4, 1, 64), (0, 0, 0, 1024, 65, 64), (-1, 0, 0, 1024, 1, 64), (0, 0, 0, 1024, 1, 96)]:
        assert L.h2_set_gemm_tuning(*bad) == mod.H2_EINVAL, bad
    try:
        mod.set_gemm_tuning(1, 0, 3, 512, 8, 128)
        assert mod.get_gemm_tuning(1, 0, 3) == (512, 8, 128)
    finally:
        mod.set_gemm_tuning(1, 0, 3, g0, gm0, t0)
    assert mod.get_gemm_tuning(1, 0, 3) == (g0, gm0, t0)


def test_allocator_hook_arguments(mod):
    """h2_set_allocator: both callbacks or neither (no device work is done)."""
    L = mod._lib
    rel = mod.RELEASE_FN(lambda p, ctx: None)
    al = mod.ALLOC_FN(lambda n, ctx: 0)
    assert L.h2_set_allocator(mod.ALLOC_FN(), rel, None) == mod.H2_EINVAL
    assert L.h2_set_allocator(al, mod.RELEASE_FN(), None) == mod.H2_EINVAL
    assert L.h2_set_allocator(al, rel, None) == mod.H2_OK
    assert L.h2_set_allocator(mod.ALLOC_FN(), mod.RELEASE_FN(), None) == mod.H2_OK
    with pytest.raises(ValueError):
        mod.set_allocator(lambda n: 0, None)
    mod.set_allocator(lambda n: 0, lambda p: None)
    mod.set_allocator()
