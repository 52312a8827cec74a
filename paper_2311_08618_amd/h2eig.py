"""Thin ctypes binding of the C ABI in include/h2eig.h (argument marshalling only).

Every computation runs inside libh2eig.so on the GPU; if the library is not
built this module raises at import, and calls fail with H2EigError when no GPU
is present.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libh2eig.so")
TUNING_FILE = os.path.join(_HERE, "tuning", "gemm_tuning.json")

H2_OK, H2_EINVAL, H2_ENOMEM, H2_EDEVICE, H2_ENUMERIC, H2_EBUSY = 0, -1, -2, -3, -4, -5

K_LAPLACE, K_YUKAWA, K_GAUSS_DAMPED, K_REG_LAPLACE, K_TRIDIAG_1D = 0, 1, 2, 3, 4


class H2EigError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("h2eig status %d: %s" % (status, msg))
        self.status = status


class _Kernel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("diag", C.c_double), ("p0", C.c_double), ("p1", C.c_double)]


class _Opts(C.Structure):
    _fields_ = [("reserved0", C.c_int32), ("reserved1", C.c_int32), ("max_shifts", C.c_int32),
                ("reserved", C.c_int32 * 5)]


class _Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("levels", C.c_int32), ("leaf_max", C.c_int32), ("rank_max", C.c_int32),
                ("near_max", C.c_int32), ("near_blocks", C.c_int64), ("resident_bytes", C.c_int64),
                ("last_work_bytes", C.c_int64), ("last_flops", C.c_double), ("last_bytes", C.c_double),
                ("build_seconds", C.c_double), ("last_rank_max", C.c_int32), ("evals_f64", C.c_int32),
                ("evals_f32", C.c_int32), ("reserved", C.c_int32 * 3)]


# device allocator hook of h2_set_allocator: alloc(bytes, ctx) -> address, release(address, ctx)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError("libh2eig.so is not built (run __graft_entry__.build())")
    lib = C.CDLL(path)
    P = C.POINTER
    lib.h2_build.restype = C.c_int
    lib.h2_build.argtypes = [P(C.c_double), C.c_int64, C.c_int32, _Kernel, C.c_int32, C.c_double, C.c_double,
                             P(_Opts), P(C.c_void_p)]
    lib.h2_inertia.restype = C.c_int
    lib.h2_inertia.argtypes = [C.c_void_p, P(C.c_double), C.c_int64, P(C.c_int64), P(C.c_int32)]
    lib.h2_kth_eig.restype = C.c_int
    lib.h2_kth_eig.argtypes = [C.c_void_p, P(C.c_int64), C.c_int64, C.c_double, P(C.c_double), P(C.c_double),
                               P(C.c_double)]
    lib.h2_norm.restype = C.c_int
    lib.h2_norm.argtypes = [C.c_void_p, P(C.c_double)]
    lib.h2_stats.restype = C.c_int
    lib.h2_stats.argtypes = [C.c_void_p, P(_Stats)]
    lib.h2_set_stream.restype = C.c_int
    lib.h2_set_stream.argtypes = [C.c_void_p, C.c_void_p]
    lib.h2_tree_perm.restype = C.c_int
    lib.h2_tree_perm.argtypes = [C.c_void_p, P(C.c_int64)]
    lib.h2_count.restype = C.c_int
    lib.h2_count.argtypes = [C.c_void_p, C.c_double, C.c_double, P(C.c_int64)]
    lib.h2_eigs_in.restype = C.c_int
    lib.h2_eigs_in.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_int64, P(C.c_double),
                               P(C.c_int64)]
    lib.h2_gap.restype = C.c_int
    lib.h2_gap.argtypes = [C.c_void_p, C.c_int64, C.c_double, P(C.c_double), P(C.c_double)]
    lib.h2_level_stats.restype = C.c_int
    lib.h2_level_stats.argtypes = [C.c_void_p, C.c_int32, C.c_int32, P(C.c_int64)]
    lib.h2_basis_ranks.restype = C.c_int
    lib.h2_basis_ranks.argtypes = [C.c_void_p, C.c_int32, P(C.c_int32)]
    lib.h2_matvec.restype = C.c_int
    lib.h2_matvec.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
    lib.h2_kernel_matvec.restype = C.c_int
    lib.h2_kernel_matvec.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
    lib.h2_kernel_matvec_noalloc.restype = C.c_int
    lib.h2_kernel_matvec_noalloc.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
    lib.h2_profile_enable.restype = C.c_int
    lib.h2_profile_enable.argtypes = [C.c_void_p, C.c_int32]
    lib.h2_profile_classes.restype = C.c_int32
    lib.h2_profile_classes.argtypes = []
    lib.h2_profile_class_name.restype = C.c_char_p
    lib.h2_profile_class_name.argtypes = [C.c_int32]
    lib.h2_profile_read.restype = C.c_int
    lib.h2_profile_read.argtypes = [C.c_void_p, C.c_int32, P(C.c_int64), P(C.c_double), P(C.c_double)]
    lib.h2_profile_bytes.restype = C.c_int
    lib.h2_profile_bytes.argtypes = [C.c_void_p, C.c_int32, P(C.c_double)]
    lib.h2_profile_level_ms.restype = C.c_int
    lib.h2_profile_level_ms.argtypes = [C.c_void_p, C.c_int32, C.c_int32, P(C.c_double)]
    lib.h2_inertia_f32.restype = C.c_int
    lib.h2_inertia_f32.argtypes = [C.c_void_p, P(C.c_double), C.c_int64, P(C.c_int64), P(C.c_int32)]
    lib.h2_set_mixed.restype = C.c_int
    lib.h2_set_mixed.argtypes = [C.c_void_p, C.c_double]
    lib.h2_interval.restype = C.c_int
    lib.h2_interval.argtypes = [C.c_void_p, P(C.c_double)]
    lib.h2_capacity.restype = C.c_int
    lib.h2_capacity.argtypes = [C.c_void_p, P(C.c_int32)]
    lib.h2_level_dims.restype = C.c_int
    lib.h2_level_dims.argtypes = [C.c_void_p, C.c_int32, P(C.c_int32)]
    lib.h2_set_gemm_tuning.restype = C.c_int
    lib.h2_set_gemm_tuning.argtypes = [C.c_int32] * 6
    lib.h2_get_gemm_tuning.restype = C.c_int
    lib.h2_get_gemm_tuning.argtypes = [C.c_int32, C.c_int32, C.c_int32, P(C.c_int32), P(C.c_int32), P(C.c_int32)]
    lib.h2_set_max_shifts.restype = C.c_int
    lib.h2_set_max_shifts.argtypes = [C.c_void_p, C.c_int32]
    lib.h2_set_allocator.restype = C.c_int
    lib.h2_set_allocator.argtypes = [ALLOC_FN, RELEASE_FN, C.c_void_p]
    lib.h2_free.restype = None
    lib.h2_free.argtypes = [C.c_void_p]
    lib.h2s_create.restype = C.c_int
    lib.h2s_create.argtypes = [C.c_int64, C.c_int32, P(C.c_void_p)]
    lib.h2s_latency.restype = C.c_int
    lib.h2s_latency.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double), P(C.c_int64), P(C.c_int64),
                                P(C.c_int64)]
    lib.h2_release_workspace.restype = C.c_int
    lib.h2_release_workspace.argtypes = [C.c_void_p]
    lib.h2s_add.restype = C.c_int
    lib.h2s_add.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, P(C.c_int32)]
    lib.h2s_submit.restype = C.c_int
    lib.h2s_submit.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_double, P(C.c_int64)]
    lib.h2s_poll.restype = C.c_int
    lib.h2s_poll.argtypes = [C.c_void_p, C.c_int64, P(C.c_double), P(C.c_int32)]
    lib.h2s_wait.restype = C.c_int
    lib.h2s_wait.argtypes = [C.c_void_p, C.c_int64, P(C.c_double)]
    lib.h2s_stats.restype = C.c_int
    lib.h2s_stats.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double), P(C.c_int64), P(C.c_int64)]
    lib.h2s_destroy.restype = None
    lib.h2s_destroy.argtypes = [C.c_void_p]
    lib.h2_last_error.restype = C.c_char_p
    lib.h2_last_error.argtypes = []
    return lib


_lib = load_library()

EXPORTED = ["h2_build", "h2_inertia", "h2_inertia_f32", "h2_set_mixed", "h2_kth_eig", "h2_norm", "h2_stats", "h2_set_stream", "h2_tree_perm",
            "h2_basis_ranks", "h2_level_stats", "h2_count", "h2_eigs_in", "h2_gap", "h2_matvec", "h2_kernel_matvec", "h2_kernel_matvec_noalloc",
            "h2_profile_enable", "h2_profile_classes", "h2_profile_class_name", "h2_profile_read", "h2_profile_bytes",
            "h2_profile_level_ms", "h2_interval", "h2_capacity", "h2_set_max_shifts", "h2_set_allocator", "h2_level_dims",
            "h2_set_gemm_tuning", "h2_get_gemm_tuning", "h2_free", "h2_last_error",
            "h2s_create", "h2s_latency", "h2_release_workspace", "h2s_add", "h2s_submit", "h2s_poll", "h2s_wait", "h2s_stats", "h2s_destroy"]


def _check(st: int):
    if st != H2_OK:
        raise H2EigError(st, _lib.h2_last_error().decode())


# every pair of callbacks ever installed: a block keeps the allocator that made
# it, so the wrappers must outlive the hook
_allocators = []


def set_allocator(alloc=None, release=None):
    """Route the library's device allocations made from now on through
    alloc(nbytes) -> device address (int; 0 or an exception: out of memory) and
    release(address) (h2_set_allocator); both None restores hipMalloc/hipFree."""
    if (alloc is None) != (release is None):
        raise ValueError("alloc and release must both be given or both be None")
    if alloc is None:
        _check(_lib.h2_set_allocator(ALLOC_FN(), RELEASE_FN(), None))
        return

    def _alloc(nbytes, ctx):
        try:
            return int(alloc(int(nbytes)) or 0)
        except Exception:
            return 0

    def _release(ptr, ctx):
        release(int(ptr))

    pair = (ALLOC_FN(_alloc), RELEASE_FN(_release))
    _allocators.append(pair)
    _check(_lib.h2_set_allocator(pair[0], pair[1], None))


def set_gemm_tuning(layout: int, f32: int, bucket: int, grid: int, group_m: int, tile: int = 0):
    _check(_lib.h2_set_gemm_tuning(int(layout), int(f32), int(bucket), int(grid), int(group_m), int(tile)))


def get_gemm_tuning(layout: int, f32: int, bucket: int):
    """(grid, group_m, tile) of one entry."""
    g, gm, t = C.c_int32(), C.c_int32(), C.c_int32()
    _check(_lib.h2_get_gemm_tuning(int(layout), int(f32), int(bucket), C.byref(g), C.byref(gm), C.byref(t)))
    return g.value, gm.value, t.value


def apply_tuning(path: str = TUNING_FILE) -> int:
    """Load the autotuner's table (JSON written by autotune.py) into the
    library; returns the number of entries applied."""
    with open(path) as f:
        table = json.load(f)
    n = 0
    for e in table["entries"]:
        set_gemm_tuning(e["layout"], e["f32"], e["bucket"], e["grid"], e["group_m"], e.get("tile", 64))
        n += 1
    return n


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


if os.path.exists(TUNING_FILE):
    apply_tuning(TUNING_FILE)


class H2Matrix:
    """A built H^2 matrix resident on the GPU (h2_build)."""

    def __init__(self, points, kind: int, diag: float, leaf: int, eta: float, eps: float,
                 p0: float = 0.0, p1: float = 0.0, max_shifts: int = 0):
        X = np.ascontiguousarray(points, dtype=np.float64)
        if X.ndim == 1:
            X = X.reshape(-1, 1)
        n, dim = X.shape
        opts = _Opts(0, 0, int(max_shifts), (C.c_int32 * 5)())
        h = C.c_void_p()
        _check(_lib.h2_build(_dptr(X), n, dim, _Kernel(int(kind), float(diag), float(p0), float(p1)), int(leaf),
                             float(eta), float(eps), C.byref(opts), C.byref(h)))
        self._h = h
        self.n = n

    def close(self):
        if getattr(self, "_h", None):
            _lib.h2_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def inertia(self, sigma, return_status: bool = False, f32: bool = False):
        """nu(sigma_s) = #{eigenvalues < sigma_s}; f32 = h2_inertia_f32."""
        s = np.ascontiguousarray(np.atleast_1d(sigma), dtype=np.float64)
        nu = np.zeros(len(s), dtype=np.int64)
        st = np.zeros(len(s), dtype=np.int32)
        fn = _lib.h2_inertia_f32 if f32 else _lib.h2_inertia
        r = fn(self._h, _dptr(s), len(s), nu.ctypes.data_as(C.POINTER(C.c_int64)),
               st.ctypes.data_as(C.POINTER(C.c_int32)))
        if r != H2_OK and not (return_status and r == H2_ENUMERIC):
            _check(r)
        return (nu, st) if return_status else nu

    def kth_eig(self, ks, tol: float, ab=None):
        k = np.ascontiguousarray(np.atleast_1d(ks), dtype=np.int64)
        lam = np.zeros(len(k))
        br = np.zeros(2 * len(k))
        abp = None
        if ab is not None:
            abv = np.ascontiguousarray(ab, dtype=np.float64)
            abp = _dptr(abv)
        _check(_lib.h2_kth_eig(self._h, k.ctypes.data_as(C.POINTER(C.c_int64)), len(k), float(tol), abp,
                               _dptr(lam), _dptr(br)))
        return lam, br.reshape(-1, 2)

    def norm(self) -> float:
        v = C.c_double()
        _check(_lib.h2_norm(self._h, C.byref(v)))
        return v.value

    def stats(self) -> dict:
        s = _Stats()
        _check(_lib.h2_stats(self._h, C.byref(s)))
        return {f[0]: getattr(s, f[0]) for f in _Stats._fields_ if f[0] != "reserved"}

    def tree_perm(self) -> np.ndarray:
        p = np.zeros(self.n, dtype=np.int64)
        _check(_lib.h2_tree_perm(self._h, p.ctypes.data_as(C.POINTER(C.c_int64))))
        return p

    def count(self, a: float, b: float) -> int:
        """Number of eigenvalues of A~ in [a, b)."""
        c = C.c_int64()
        _check(_lib.h2_count(self._h, float(a), float(b), C.byref(c)))
        return int(c.value)

    def eigs_in(self, a: float, b: float, tol: float, cap: int = 1 << 20) -> np.ndarray:
        """Every eigenvalue of A~ in [a, b), each to absolute tolerance tol."""
        c = C.c_int64()
        st = _lib.h2_count(self._h, float(a), float(b), C.byref(c))
        _check(st)
        lam = np.zeros(max(1, min(int(cap), int(c.value))))
        _check(_lib.h2_eigs_in(self._h, float(a), float(b), float(tol), len(lam), _dptr(lam), C.byref(c)))
        return lam[:int(c.value)]

    def gap(self, k: int, tol: float):
        """(lambda_k, lambda_{k+1}, lambda_{k+1} - lambda_k), each eigenvalue to tolerance tol."""
        lam = np.zeros(2)
        g = C.c_double()
        _check(_lib.h2_gap(self._h, int(k), float(tol), _dptr(lam), C.byref(g)))
        return float(lam[0]), float(lam[1]), float(g.value)

    def release_workspace(self):
        """Free the factorization workspace (the next inertia call allocates it again)."""
        _check(_lib.h2_release_workspace(self._h))

    def level_stats(self, shift: int = 0) -> np.ndarray:
        """Per level of the last factorization: (sum t, sum m, max m, sum R) for one shift of its batch."""
        nlev = self.stats()["levels"] + 1
        out = np.zeros((nlev, 4), dtype=np.int64)
        _check(_lib.h2_level_stats(self._h, int(shift), nlev, out.ctypes.data_as(C.POINTER(C.c_int64))))
        return out

    def basis_ranks(self, level: int) -> np.ndarray:
        r = np.zeros(1 << int(level), dtype=np.int32)
        _check(_lib.h2_basis_ranks(self._h, int(level), r.ctypes.data_as(C.POINTER(C.c_int32))))
        return r

    def matvec(self, x) -> np.ndarray:
        """y = A~ x with the built H^2 matrix (original point order)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.n)
        _check(_lib.h2_matvec(self._h, _dptr(x), _dptr(y)))
        return y

    def kernel_matvec(self, x) -> np.ndarray:
        """y = A x with the exact kernel matrix, on the GPU."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.n)
        _check(_lib.h2_kernel_matvec(self._h, _dptr(x), _dptr(y)))
        return y

    def kernel_matvec_noalloc(self, x) -> np.ndarray:
        """y = A x as kernel_matvec, staged through the library's static device scratch (no allocation)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.n)
        _check(_lib.h2_kernel_matvec_noalloc(self._h, _dptr(x), _dptr(y)))
        return y

    def profile_enable(self, on=True):
        """True/1: every launch timed; 2: GEMM launches only; False/0: off."""
        _check(_lib.h2_profile_enable(self._h, int(on)))

    def profile_read(self) -> dict:
        out = {}
        for c in range(_lib.h2_profile_classes()):
            n = C.c_int64()
            ms = C.c_double()
            fl = C.c_double()
            _check(_lib.h2_profile_read(self._h, c, C.byref(n), C.byref(ms), C.byref(fl)))
            by = C.c_double()
            _check(_lib.h2_profile_bytes(self._h, c, C.byref(by)))
            out[_lib.h2_profile_class_name(c).decode()] = {"launches": n.value, "ms": ms.value, "flops": fl.value,
                                                           "bytes": by.value}
        return out

    def profile_levels(self, levels: int = 32) -> dict:
        """{class name: [ms at level 0, 1, ...]} since profiling was enabled."""
        out = {}
        for c in range(_lib.h2_profile_classes()):
            row = []
            for lev in range(levels):
                ms = C.c_double()
                _check(_lib.h2_profile_level_ms(self._h, c, lev, C.byref(ms)))
                row.append(ms.value)
            out[_lib.h2_profile_class_name(c).decode()] = row
        return out

    def set_stream(self, stream_ptr: int):
        _check(_lib.h2_set_stream(self._h, C.c_void_p(stream_ptr)))

    def set_mixed(self, switch_rel: float):
        """h2_kth_eig bisects in FP32 while a bracket is >= switch_rel * normA wide (0 = FP64 only)."""
        _check(_lib.h2_set_mixed(self._h, float(switch_rel)))

    def interval(self):
        ab = np.zeros(2)
        _check(_lib.h2_interval(self._h, _dptr(ab)))
        return float(ab[0]), float(ab[1])

    def level_dims(self) -> list:
        """Block capacity of every level in the last factorization (0 = not reached)."""
        nlev = self.stats()["levels"] + 1
        cap = (C.c_int32 * nlev)()
        _check(_lib.h2_level_dims(self._h, nlev, cap))
        return list(cap)

    def set_max_shifts(self, max_shifts: int):
        _check(_lib.h2_set_max_shifts(self._h, int(max_shifts)))

    def capacity(self) -> int:
        v = C.c_int32()
        _check(_lib.h2_capacity(self._h, C.byref(v)))
        return v.value


class H2Server:
    """Serving loop over resident matrices (h2s_*): continuous batching of
    k-th eigenvalue queries, one worker per matrix.  Holds references to the
    added matrices until close()."""

    def __init__(self, max_slots: int = 0, budget_bytes: int = 0):
        h = C.c_void_p()
        _check(_lib.h2s_create(int(budget_bytes), int(max_slots), C.byref(h)))
        self._h = h
        self._mats = []

    def add(self, A: H2Matrix, slots: int = 0) -> int:
        i = C.c_int32()
        _check(_lib.h2s_add(self._h, A._h, int(slots), C.byref(i)))
        self._mats.append(A)
        return i.value

    def submit(self, mat: int, k: int, tol: float) -> int:
        t = C.c_int64()
        _check(_lib.h2s_submit(self._h, int(mat), int(k), float(tol), C.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """lambda once finished, else None."""
        lam = C.c_double()
        done = C.c_int32()
        _check(_lib.h2s_poll(self._h, int(ticket), C.byref(lam), C.byref(done)))
        return lam.value if done.value else None

    def wait(self, ticket: int) -> float:
        lam = C.c_double()
        _check(_lib.h2s_wait(self._h, int(ticket), C.byref(lam)))
        return lam.value

    def stats(self) -> dict:
        p50, p99 = C.c_double(), C.c_double()
        served, submitted = C.c_int64(), C.c_int64()
        _check(_lib.h2s_stats(self._h, C.byref(p50), C.byref(p99), C.byref(served), C.byref(submitted)))
        return {"p50_ms": p50.value, "p99_ms": p99.value, "served": served.value, "submitted": submitted.value}

    def latency(self) -> dict:
        """Censored latency over every submitted query (unfinished ones at their age)."""
        p50, p99 = C.c_double(), C.c_double()
        open_, budget, used = C.c_int64(), C.c_int64(), C.c_int64()
        _check(_lib.h2s_latency(self._h, C.byref(p50), C.byref(p99), C.byref(open_), C.byref(budget),
                                C.byref(used)))
        return {"p50_ms": p50.value, "p99_ms": p99.value, "unfinished": open_.value,
                "budget_bytes": budget.value, "used_bytes": used.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.h2s_destroy(self._h)
            self._h = None
            self._mats = []

    def __del__(self):
        self.close()
