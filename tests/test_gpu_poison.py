"""Initialisation of the device workspace: with H2EIG_POISON=1 every workspace
byte is 0xFF (a NaN in every double) at allocation and before every
factorization, so a kernel that reads memory the call did not write gives a
different count (or a failed shift).  The counts must equal those of the clean
workspace, shift for shift, for batches of several sizes (arenas grow and are
reused), and the tridiagonal counts must equal the closed form.
"""
import json
import os

import numpy as np
import pytest

from oracle.dense import tridiag_eigs
from paper_2311_08618_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cube_laplace_n2048.json")


@pytest.fixture(scope="module")
def lib():
    from paper_2311_08618_amd import h2eig
    return h2eig


@pytest.fixture
def poison():
    old = os.environ.get("H2EIG_POISON")
    os.environ["H2EIG_POISON"] = "1"
    yield
    if old is None:
        os.environ.pop("H2EIG_POISON", None)
    else:
        os.environ["H2EIG_POISON"] = old


def _batches(A, sig):
    out = []
    for bs in (1, 3, 7, len(sig)):
        nu = np.concatenate([A.inertia(sig[i:i + bs]) for i in range(0, len(sig), bs)])
        out.append(nu)
    return out


def test_cube_counts_with_poisoned_workspace(lib, poison):
    print("case poison cube n=2048", flush=True)
    g = json.load(open(GOLDEN))
    A = lib.H2Matrix(W.cube_points(g["n"], 0), W.K_LAPLACE, 1e3, g["leaf"], g["eta"], g["eps"])
    sig = np.array([r["sigma"] for r in g["inertia"]])
    dirty = _batches(A, sig)
    os.environ.pop("H2EIG_POISON")
    B = lib.H2Matrix(W.cube_points(g["n"], 0), W.K_LAPLACE, 1e3, g["leaf"], g["eta"], g["eps"])
    clean = B.inertia(sig)
    for nu in dirty:
        assert np.array_equal(nu, clean), (nu - clean)
    for r, v in zip(g["inertia"], clean):
        assert r["nu_lo"] <= v <= r["nu_hi"], (r, v)


def test_tridiag_counts_with_poisoned_workspace(lib, poison):
    print("case poison tridiag n=4100", flush=True)
    n = 4100   # ragged: leaves of 64 and 65 points
    T = lib.H2Matrix(W.line_points(n), W.K_TRIDIAG_1D, 2.0, 64, 1.0, 1e-12, p0=1.0)
    lam = tridiag_eigs(n)
    sig = np.concatenate([np.linspace(-0.2, 4.2, 11) + 1e-3 * np.sqrt(2.0), lam[[0, 1, n // 2, n - 1]] + 1e-9])
    want = np.array([int(np.sum(lam < s)) for s in sig])
    for nu in _batches(T, sig):
        assert np.array_equal(nu, want), (nu - want)
