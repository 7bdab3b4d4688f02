"""Approximate inverse of an H^2 matrix by repeated H^2 matrix-matrix
products (the use Section I names for the product: inverse-based fast
solvers).  Newton-Schulz iteration

    X_0 = alpha I,   X_{j+1} = X_j (2 I - A X_j),

started at X_1 = 2 alpha I - alpha^2 A (exact, in A's partition and bases),
then each step two products of `oracle.mmp.h2_mmp` at eps and one shift of
the dense diagonal blocks (2 I - Y keeps Y's partition and bases: the
identity lives in the dense diagonal leaf blocks only).  For A with eigenvalues in
(0, 1/alpha] (symmetric positive definite A, alpha <= 1/lambda_max) the
residual I - A X_j squares every step until the truncation at eps limits it.
Plain FP64 NumPy over the oracle's product.

Part of the CPU checker: test infrastructure only.
"""
import numpy as np

from h2inputs.h2data import H2Matrix
from . import h2ops
from .mmp import ACCURACY, h2_mmp


def scale_shift(M, a, b):
    """a M + b I (same partition and bases)."""
    L = M.L
    S = [[None if s is None else a * s for s in sl] for sl in M.S]
    Fd = []
    for t, s, f in zip(M.blocks.rows[L], M.blocks.cols[L], M.F):
        if f is None:
            Fd.append(None)
            continue
        g = a * f
        if t == s:
            g = g + b * np.eye(f.shape[0], dtype=g.dtype)
        Fd.append(g)
    return H2Matrix(M.tree, M.blocks, M.V, M.Er, M.W, M.Ec, S, Fd)


def newton_schulz(A, eps, alpha, steps, mode=ACCURACY, probes=None):
    """X_steps (steps >= 1) and the residuals ||x - A X_j x|| / ||x|| after
    every step j = 1 .. steps for the probe columns `probes` (n x p), when
    given."""
    res = []
    X = None
    for j in range(steps):
        if j == 0:
            X = scale_shift(A, -alpha * alpha, 2.0 * alpha)
        else:
            Y, _ = h2_mmp(A, X, eps, mode=mode)
            X, _ = h2_mmp(X, scale_shift(Y, -1.0, 2.0), eps, mode=mode)
        if probes is not None:
            r = probes - h2ops.matvec(A, h2ops.matvec(X, probes))
            res.append(float(np.linalg.norm(r) / np.linalg.norm(probes)))
    return X, res
