"""The allocation-free exact-kernel matvec (h2_kernel_matvec_noalloc) against
h2_kernel_matvec: the same kernel and summation order, so the same bits, on two
calls in a row, the second with a smaller input."""
import numpy as np
import pytest

from paper_2311_08618_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_noalloc_matvec_matches_allocating_one():
    from paper_2311_08618_amd import h2eig
    rng = np.random.default_rng(11)
    for n, leaf, kind in ((20000, 256, W.K_YUKAWA), (3001, 64, W.K_LAPLACE)):
        print("case noalloc n=%d kind=%d" % (n, kind), flush=True)
        A = h2eig.H2Matrix(W.cube_points(n, 5), kind, 1e3, leaf, 1.0, 1e-6)
        x = rng.standard_normal(n)
        want = A.kernel_matvec(x)
        got = A.kernel_matvec_noalloc(x)
        assert np.array_equal(got, want)
        A.close()
