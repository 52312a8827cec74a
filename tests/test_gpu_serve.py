"""The serving loop (h2s_*) on the GPU: k-th eigenvalue queries for two resident
matrices, submitted interleaved and batched by the workers (Algorithm 1 with
inertia reuse, Secs. 2 and 4.2).  Every answer is checked against what fixes it
independently of the path: the closed-form spectrum 2 - 2cos(j pi/(n+1)) of the
second-difference matrix, LAPACK on the dense cube matrix, and a standalone
h2_kth_eig on the same handle before it was made resident.
"""
import time

import numpy as np
import pytest

from oracle.dense import tridiag_eigs
from oracle.kernels import Kernel
from paper_2311_08618_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2311_08618_amd import h2eig
    return h2eig


def test_serve_two_matrices_interleaved(lib):
    print("case serve cube n=2048 + tridiag n=4096, slots 3", flush=True)
    n1, n2, tol = 2048, 4096, 1e-8
    X = W.cube_points(n1, 0)
    A = lib.H2Matrix(X, W.K_LAPLACE, 1e3, 128, 1.0, 1e-8)
    T = lib.H2Matrix(W.line_points(n2), W.K_TRIDIAG_1D, 2.0, 64, 1.0, 1e-12, p0=1.0)
    dense = np.linalg.eigvalsh(Kernel(W.K_LAPLACE, 1e3).dense(X))
    exact_t = tridiag_eigs(n2)
    rng = np.random.default_rng(5)
    ks_a = [int(k) for k in rng.integers(1, n1 + 1, 5)] + [n1 // 2, n1 // 2]   # a repeated query
    ks_t = [1, n2] + [int(k) for k in rng.integers(1, n2 + 1, 4)]
    alone_a, _ = A.kth_eig(ks_a, tol)
    bound_a = tol / 2 + 10 * 1e-8 * A.norm()
    bound_t = tol / 2 + 10 * 1e-12 * T.norm()
    # the first midpoint of the Gershgorin interval [0, 4] is 2, where the
    # leaf pivot blocks of odd order are exactly singular: bisection must
    # split elsewhere and still converge
    assert T.inertia(np.array([2.0]), return_status=True)[1][0] == lib.H2_ENUMERIC
    alone_t, _ = T.kth_eig([n2 // 2, n2 // 2 + 1], tol)
    assert np.all(np.abs(alone_t - exact_t[[n2 // 2 - 1, n2 // 2]]) <= bound_t), alone_t

    S = lib.H2Server(max_slots=3)
    try:
        ia, it = S.add(A), S.add(T)
        assert (ia, it) == (0, 1)
        tickets = []
        for j in range(max(len(ks_a), len(ks_t))):
            if j < len(ks_a):
                tickets.append(("a", ks_a[j], j, S.submit(ia, ks_a[j], tol)))
            if j < len(ks_t):
                tickets.append(("t", ks_t[j], j, S.submit(it, ks_t[j], tol)))
        for which, k, j, tk in tickets:
            lam = S.wait(tk)
            with pytest.raises(lib.H2EigError):      # a finished ticket is read once
                S.poll(tk)
            if which == "a":
                assert abs(lam - dense[k - 1]) <= bound_a, (k, lam, dense[k - 1])
                assert abs(lam - alone_a[j]) <= tol + 10 * 1e-8 * A.norm(), (k, lam, alone_a[j])
            else:
                assert abs(lam - exact_t[k - 1]) <= bound_t, (k, lam, exact_t[k - 1])
        st = S.stats()
        assert st["served"] == st["submitted"] == len(ks_a) + len(ks_t)
        assert 0.0 < st["p50_ms"] <= st["p99_ms"]
    finally:
        S.close()
    # the handles are the caller's again once the server is gone
    nu = T.inertia(np.array([2.5]))
    assert nu[0] == int(np.sum(exact_t < 2.5))


def test_serve_one_slot_queue(lib):
    """One slot: queries wait in the queue and are admitted one at a time."""
    print("case serve tridiag n=1024, slots 1", flush=True)
    n, tol = 1024, 1e-9
    T = lib.H2Matrix(W.line_points(n), W.K_TRIDIAG_1D, 2.0, 32, 1.0, 1e-12, p0=1.0)
    exact = tridiag_eigs(n)
    S = lib.H2Server(max_slots=1)
    try:
        m = S.add(T)
        ks = [3, 500, 1024, 77, 3]
        tk = [S.submit(m, k, tol) for k in ks]
        for k, t in zip(ks, tk):
            lam = S.wait(t)
            assert abs(lam - exact[k - 1]) <= tol / 2 + 10 * 1e-12 * T.norm(), (k, lam)
        with pytest.raises(lib.H2EigError):
            S.submit(m, n + 1, tol)
        with pytest.raises(lib.H2EigError):
            S.submit(5, 1, tol)
        assert S.stats()["served"] == len(ks)
    finally:
        S.close()


def test_serve_shared_memory_budget(lib):
    """Admission by memory: with a budget of one shift of the larger matrix,
    the two matrices never hold more than the budget together, queries of the
    other matrix wait until the share is returned, and every answer is still
    exact (closed-form spectrum)."""
    print("case serve budget: two tridiag matrices, budget of one shift", flush=True)
    n1, n2, tol = 2048, 1024, 1e-9
    T1 = lib.H2Matrix(W.line_points(n1), W.K_TRIDIAG_1D, 2.0, 64, 1.0, 1e-12, p0=1.0)
    T2 = lib.H2Matrix(W.line_points(n2), W.K_TRIDIAG_1D, 2.0, 32, 1.0, 1e-12, p0=1.0)
    T1.inertia(np.array([1.37]))
    per1 = T1.stats()["last_work_bytes"]
    T1.release_workspace()
    budget = int(1.5 * per1)
    S = lib.H2Server(max_slots=4, budget_bytes=budget)
    try:
        i1, i2 = S.add(T1), S.add(T2)
        ks1, ks2 = [1, 700, n1], [5, 512]
        tk = [(n1, k, S.submit(i1, k, tol)) for k in ks1] + [(n2, k, S.submit(i2, k, tol)) for k in ks2]
        peak = 0
        for n, k, t in tk:
            while True:
                lat = S.latency()
                peak = max(peak, lat["used_bytes"])
                lam = S.poll(t)
                if lam is not None:
                    break
                time.sleep(0.002)
            exact = tridiag_eigs(n)
            assert abs(lam - exact[k - 1]) <= tol / 2 + 10 * 1e-12 * 4.0, (n, k, lam)
        assert lat["budget_bytes"] == budget
        assert 0 < peak <= budget
        assert S.stats()["served"] == len(tk)
        assert S.latency()["unfinished"] == 0
    finally:
        S.close()


def test_serve_two_readers_of_one_ticket(lib):
    """h2s_wait in a thread and h2s_poll in the caller on the same ticket:
    exactly one of them reports the eigenvalue (closed form), the other finds
    the ticket already read (H2_EINVAL), and neither blocks."""
    import threading
    print("case serve two readers of one ticket, tridiag n=1024", flush=True)
    n, tol = 1024, 1e-9
    T = lib.H2Matrix(W.line_points(n), W.K_TRIDIAG_1D, 2.0, 32, 1.0, 1e-12, p0=1.0)
    exact = tridiag_eigs(n)
    S = lib.H2Server(max_slots=2)
    try:
        m = S.add(T)
        for k in (1, 300, n):
            t = S.submit(m, k, tol)
            got = []

            def reader(t=t, got=got):
                try:
                    got.append(("wait", S.wait(t)))
                except lib.H2EigError:
                    got.append(("wait", None))

            th = threading.Thread(target=reader)
            th.start()
            t0 = time.time()
            while True:
                try:
                    lam = S.poll(t)
                except lib.H2EigError:
                    got.append(("poll", None))
                    break
                if lam is not None:
                    got.append(("poll", lam))
                    break
                assert time.time() - t0 < 60
                time.sleep(0.001)
            th.join(60)
            assert not th.is_alive()
            vals = [v for _, v in got if v is not None]
            assert len(got) == 2 and len(vals) == 1, got
            assert abs(vals[0] - exact[k - 1]) <= tol / 2 + 10 * 1e-12 * T.norm(), (k, vals)
    finally:
        S.close()


def _free_device_bytes():
    """hipMemGetInfo of the current device, through the HIP runtime the library
    already initialised in this process."""
    import ctypes
    try:
        hip = ctypes.CDLL("libamdhip64.so.7")       # the runtime libh2eig.so loaded
    except OSError:
        hip = ctypes.CDLL("/opt/rocm/lib/libamdhip64.so")
    free, total = ctypes.c_size_t(), ctypes.c_size_t()
    assert hip.hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)) == 0
    return free.value


def test_serve_destroy_frees_workspace(lib):
    """A server destroyed while its queries are in flight frees the
    factorization workspace of its matrices: the device memory held before the
    server existed is all that remains held."""
    print("case serve destroy: cube n=16384 with queries in flight", flush=True)
    A = lib.H2Matrix(W.cube_points(16384, 3), W.K_LAPLACE, 1e3, 256, 1.0, 1e-8)
    A.interval()
    free0 = _free_device_bytes()
    S = lib.H2Server(max_slots=4)
    try:
        i = S.add(A)
        for k in (1, 4000, 8000, 16000):
            S.submit(i, k, 1e-12)
        t0 = time.time()
        while S.latency()["used_bytes"] == 0 and time.time() - t0 < 60:
            time.sleep(0.01)
        assert S.latency()["used_bytes"] > 0
        time.sleep(1.0)                     # the first batched factorization has its arenas
        assert S.latency()["unfinished"] > 0
    finally:
        S.close()
    free1 = _free_device_bytes()
    assert free1 >= free0 - (64 << 20), (free0, free1)
    A.close()
