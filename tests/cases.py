"""Small seeded H^2 inputs shared by the CPU checks and the GPU parity tests."""
import functools

import numpy as np

from h2inputs import configs, points
from h2inputs.build import (HelmholtzKernel, LaplaceKernel, chebyshev_h2,
                            random_h2)
from h2inputs.h2data import H2Matrix
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


def transpose_h2(M):
    """M^T in the same (symmetric) partition: row and column sides swapped,
    couplings and dense blocks transposed."""
    L = M.L
    S, Fd = [], []
    for lev in range(L + 1):
        pos = {(int(i), int(j)): q for q, (i, j) in
               enumerate(zip(M.blocks.rows[lev], M.blocks.cols[lev]))}
        out = [None] * len(M.blocks.rows[lev])
        for (i, j), q in pos.items():
            s = M.S[lev][q]
            out[pos[(j, i)]] = None if s is None else np.ascontiguousarray(s.T)
        S.append(out)
        if lev == L:
            Fd = [None] * len(M.blocks.rows[lev])
            for (i, j), q in pos.items():
                f = M.F[q]
                Fd[pos[(j, i)]] = None if f is None else np.ascontiguousarray(f.T)
    return H2Matrix(M.tree, M.blocks, M.W, M.Ec, M.V, M.Er, S, Fd)


def scaled_h2(M, alpha):
    """alpha M: couplings and dense blocks scaled, bases unchanged."""
    S = [[None if s is None else alpha * s for s in sl] for sl in M.S]
    Fd = [None if f is None else alpha * f for f in M.F]
    return H2Matrix(M.tree, M.blocks, M.V, M.Er, M.W, M.Ec, S, Fd)


@functools.lru_cache(maxsize=None)
def plates_two_orders(n):
    """Two different real symmetric matrices of one kernel on one partition
    (Chebyshev orders 3 and 2): A B != B A and the row and column sides of
    C = A B come from inputs of different rank."""
    w = configs.plates_n(n)
    t = w.tree()
    b = BlockTree(t, w.eta)
    return chebyshev_h2(t, b, w.kernel, 3), chebyshev_h2(t, b, w.kernel, 2)
