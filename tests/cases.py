"""Small seeded H^2 inputs shared by the CPU checks and the GPU parity tests."""
import functools

import numpy as np

from h2inputs import configs, points
from h2inputs.build import (HelmholtzKernel, LaplaceKernel, chebyshev_h2,
                            random_h2)
from h2inputs.structure import BlockTree, ClusterTree


@functools.lru_cache(maxsize=None)
def cube1k():
    return configs.cube1k().build()


@functools.lru_cache(maxsize=None)
def plates(n, leaf=32, order=3):
    return configs.plates_n(n, leaf=leaf, order=order).build()


@functools.lru_cache(maxsize=None)
def cube(n, leaf=32, order=3, seed=0):
    return configs.cube_n(n, seed=seed, leaf=leaf, order=order).build()


@functools.lru_cache(maxsize=None)
def random_pair(n, leaf, kr, kc, seed, complex_=False, geometry="plates"):
    """Two different random H^2 matrices (distinct row and column sides) on
    one partition; kr/kc are the ranks per level (constant)."""
    if geometry == "plates":
        pts = points.plates_random(n, 0.1, 1e-3, seed)
    else:
        pts = points.cube(n, seed)
    t = ClusterTree(pts, leaf)
    b = BlockTree(t, 1.0)
    L = t.L
    A = random_h2(t, b, [kr] * (L + 1), [kc] * (L + 1), seed + 1, complex_)
    B = random_h2(t, b, [kc] * (L + 1), [kr] * (L + 1), seed + 2, complex_)
    return A, B


@functools.lru_cache(maxsize=None)
def ragged_plates(n, leaf, order=2, seed=7):
    """Random plate points with N not a power of two: leaves of unequal size."""
    pts = points.plates_random(n, 0.1, 1e-3, seed)
    t = ClusterTree(pts, leaf)
    b = BlockTree(t, 1.0)
    return chebyshev_h2(t, b, LaplaceKernel(1.0), order)


@functools.lru_cache(maxsize=None)
def helmholtz_sphere(n, leaf, order, kappa):
    pts = points.fibonacci_sphere(n)
    t = ClusterTree(pts, leaf)
    b = BlockTree(t, 1.0)
    rho = 2.0 / np.sqrt(n)
    A = chebyshev_h2(t, b, HelmholtzKernel(kappa, 1 / (2 * np.pi * rho) - 1j * kappa / (4 * np.pi)), order)
    B = chebyshev_h2(t, b, HelmholtzKernel(kappa / 2, 1 / (2 * np.pi * rho) - 1j * kappa / (8 * np.pi)), order)
    return A, B
