"""Seeded synthetic inputs shared by the tests, the bench and the oracle's callers.

This module only draws numbers: point clouds, shift grids, eigenvalue indices
and request arrival times.  It holds none of the method's arithmetic (no kernel
evaluation, no tree, no factorization), so that the HIP path and the CPU oracle
can be fed identical inputs without sharing any computation.

Workloads (all synthetic; the paper's ELSES fullerene matrices are private):
  * ``cube``: points uniform in the unit cube, NumPy PCG64 ``default_rng(seed)``.
  * ``circle``: equispaced points on the unit circle (the paper's synthetic
    Laplace test, Sec. 5.1, read as equispaced).
  * ``line``: x_i = i on a line (the 1-D second-difference matrix test).
  * ``cylinders``: points on the surfaces of parallel cylinders with Gaussian
    jitter (nanotube-like layout).
"""
from __future__ import annotations

import numpy as np

# kernel kinds; the numeric codes are part of the C ABI (include/h2eig.h)
K_LAPLACE = 0        # 1/r
K_YUKAWA = 1         # exp(-r)/r
K_GAUSS_DAMPED = 2   # exp(-r^2/p0)/(r+p1)
K_REG_LAPLACE = 3    # 1/(r+p0)
K_TRIDIAG_1D = 4     # -1 if |r-p0| < 1e-9*p0 else 0


def cube_points(n: int, seed: int = 0) -> np.ndarray:
    """n points uniform in [0,1]^3 (row-major float64, shape (n, 3))."""
    return np.random.default_rng(seed).random((n, 3))


def circle_points(n: int) -> np.ndarray:
    """n equispaced points on the unit circle, shape (n, 2)."""
    th = 2.0 * np.pi * np.arange(n) / n
    return np.ascontiguousarray(np.stack([np.cos(th), np.sin(th)], axis=1))


def line_points(n: int) -> np.ndarray:
    """x_i = i, shape (n, 1)."""
    return np.arange(n, dtype=np.float64).reshape(n, 1)


def cylinder_points(n: int, seed: int = 0, ncyl: int = 16, radius: float = 0.05,
                    length: float = 1.0, spacing: float = 0.25,
                    jitter: float = 1e-3) -> np.ndarray:
    """Points on the surfaces of ``ncyl`` z-parallel cylinders on a square grid.

    Points are uniform in angle and height, then jittered by N(0, jitter^2)
    per coordinate.  ``n`` must be divisible by ``ncyl``.
    """
    assert n % ncyl == 0
    g = int(round(np.sqrt(ncyl)))
    rng = np.random.default_rng(seed)
    per = n // ncyl
    out = []
    for c in range(ncyl):
        cx, cy = (c % g) * spacing, (c // g) * spacing
        th = rng.random(per) * 2.0 * np.pi
        z = rng.random(per) * length
        p = np.stack([cx + radius * np.cos(th), cy + radius * np.sin(th), z], axis=1)
        out.append(p)
    pts = np.concatenate(out, axis=0)
    pts += rng.normal(0.0, jitter, size=pts.shape)
    return np.ascontiguousarray(pts)


def shift_grid(lo: float, hi: float, count: int, seed: int = 0) -> np.ndarray:
    """``count`` shifts uniform in [lo, hi), sorted, seeded."""
    return np.sort(np.random.default_rng(seed).uniform(lo, hi, count))


def k_spread(n: int, count: int) -> np.ndarray:
    """Eigenvalue indices {1, n/count, 2n/count, ...} (1-based)."""
    ks = [max(1, (j * n) // count) for j in range(count)]
    return np.asarray(ks, dtype=np.int64)


def k_uniform(n: int, count: int, seed: int = 1) -> np.ndarray:
    """``count`` 1-based indices uniform in [1, n], seeded."""
    return np.random.default_rng(seed).integers(1, n + 1, count).astype(np.int64)


def poisson_arrivals(rate: float, duration: float, seed: int = 7) -> np.ndarray:
    """Arrival times of a Poisson stream with the given rate over ``duration`` s."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        out.append(t)
    return np.asarray(out)
