"""Construction of the input H^2 matrices.

The paper builds its inputs with a method it cites but does not describe
(Section VI); these inputs stand in for them.  Two families:

  * `chebyshev_h2`: kernel matrices with nested tensor Chebyshev
    interpolation bases.  Each cluster gets first-kind Chebyshev nodes of
    order p per axis on its tight bounding box (degenerate extents padded to
    1e-9 times the root diameter, or 1e-9 when all points coincide); the leaf
    basis is the tensor Lagrange basis evaluated at the cluster's points, the
    transfer matrix of a child is
    the parent's Lagrange basis evaluated at the child's nodes (exact, since
    the interpolant of a degree p-1 polynomial at p nodes is itself), a
    coupling matrix is the kernel at the two clusters' node sets, and a dense
    block is the kernel at the points with a configured self-term on
    coincident points.
  * `random_h2`: seeded Gaussian bases, transfers, couplings and dense
    blocks with prescribed ranks per level and distinct row/column sides,
    used to exercise non-symmetric and complex products.
"""
import math

import numpy as np

from .h2data import H2Matrix
from .structure import R, F


# ----------------------------------------------------------------- kernels
class LaplaceKernel:
    """1/(4 pi r), with `self_value` where r = 0."""

    dtype = np.dtype(np.float64)

    def __init__(self, self_value):
        self.self_value = float(self_value)

    def __call__(self, X, Y):
        d = np.sqrt(((X[:, None, :] - Y[None, :, :]) ** 2).sum(axis=2))
        with np.errstate(divide="ignore"):
            K = 1.0 / (4.0 * math.pi * d)
        K[d == 0.0] = self.self_value
        return K


class HelmholtzKernel:
    """exp(-j kappa r)/(4 pi r), with `self_value` where r = 0."""

    dtype = np.dtype(np.complex128)

    def __init__(self, kappa, self_value):
        self.kappa = float(kappa)
        self.self_value = complex(self_value)

    def __call__(self, X, Y):
        d = np.sqrt(((X[:, None, :] - Y[None, :, :]) ** 2).sum(axis=2))
        with np.errstate(divide="ignore", invalid="ignore"):
            K = np.exp(-1j * self.kappa * d) / (4.0 * math.pi * d)
        K[d == 0.0] = self.self_value
        return K


def panel_self_term(a, b):
    """Mean of 1/(4 pi r) over an a-by-b rectangle about its centre."""
    return (2 * a * math.asinh(b / a) + 2 * b * math.asinh(a / b)) / (4 * math.pi * a * b)


# --------------------------------------------------------------- chebyshev
def _cheb_1d(p):
    return np.cos((2.0 * np.arange(p) + 1.0) * math.pi / (2.0 * p))


def _lagrange_1d(xi, x):
    p = xi.shape[0]
    out = np.ones((x.shape[0], p))
    for m in range(p):
        for q in range(p):
            if q != m:
                out[:, m] *= (x - xi[q]) / (xi[m] - xi[q])
    return out


class _BoxNodes:
    def __init__(self, lo, hi, p, pad):
        c = 0.5 * (lo + hi)
        h = np.maximum(0.5 * (hi - lo), 0.5 * pad)
        t = _cheb_1d(p)
        self.axes = [c[a] + h[a] * t for a in range(3)]
        self.p = p

    def lagrange(self, X):
        """(n, p^3) tensor Lagrange basis at points X; column (m0*p+m1)*p+m2."""
        l0 = _lagrange_1d(self.axes[0], X[:, 0])
        l1 = _lagrange_1d(self.axes[1], X[:, 1])
        l2 = _lagrange_1d(self.axes[2], X[:, 2])
        return np.einsum("na,nb,nc->nabc", l0, l1, l2).reshape(X.shape[0], -1)

    def points(self):
        g = np.meshgrid(*self.axes, indexing="ij")
        return np.stack([a.ravel() for a in g], axis=1)


def chebyshev_h2(tree, blocks, kernel, order):
    L = tree.L
    pts = tree.points
    root_diam = float(np.linalg.norm(tree.hi[0][0] - tree.lo[0][0]))
    pad = 1e-9 * (root_diam if root_diam > 0.0 else 1.0)  # a single point: absolute pad
    nodes = [[_BoxNodes(tree.lo[lev][c], tree.hi[lev][c], order, pad)
              for c in range(1 << lev)] for lev in range(L + 1)]
    cdt = kernel.dtype
    V = []
    for c in range(1 << L):
        X = pts[tree.indices(L, c)]
        V.append(nodes[L][c].lagrange(X).astype(cdt))
    Er = [[None]]
    for lev in range(1, L + 1):
        Er.append([nodes[lev - 1][c // 2].lagrange(nodes[lev][c].points()).astype(cdt)
                   for c in range(1 << lev)])
    S = []
    for lev in range(L + 1):
        sl = []
        for t, s, typ in zip(blocks.rows[lev], blocks.cols[lev], blocks.types[lev]):
            if typ == R:
                sl.append(kernel(nodes[lev][t].points(), nodes[lev][s].points()).astype(cdt))
            else:
                sl.append(None)
        S.append(sl)
    Fd = []
    for t, s, typ in zip(blocks.rows[L], blocks.cols[L], blocks.types[L]):
        if typ == F:
            Fd.append(kernel(pts[tree.indices(L, t)], pts[tree.indices(L, s)]).astype(cdt))
        else:
            Fd.append(None)
    return H2Matrix(tree, blocks, V, Er, V, Er, S, Fd)


# ------------------------------------------------------------------ random
def random_h2(tree, blocks, krow, kcol, seed, complex_=False, dense_scale=1.0):
    """Random H^2 matrix; krow[l] / kcol[l] are the ranks at level l."""
    rng = np.random.default_rng(seed)
    L = tree.L

    def g(*shape):
        x = rng.standard_normal(shape)
        if complex_:
            x = x + 1j * rng.standard_normal(shape)
        return x

    V = [g(tree.size(L, c), krow[L]) / math.sqrt(max(1, tree.size(L, c)))
         for c in range(1 << L)]
    W = [g(tree.size(L, c), kcol[L]) / math.sqrt(max(1, tree.size(L, c)))
         for c in range(1 << L)]
    Er, Ec = [[None]], [[None]]
    for lev in range(1, L + 1):
        Er.append([g(krow[lev], krow[lev - 1]) / math.sqrt(krow[lev]) for _ in range(1 << lev)])
        Ec.append([g(kcol[lev], kcol[lev - 1]) / math.sqrt(kcol[lev]) for _ in range(1 << lev)])
    S = []
    for lev in range(L + 1):
        S.append([g(krow[lev], kcol[lev]) if typ == R else None
                  for typ in blocks.types[lev]])
    Fd = []
    for t, s, typ in zip(blocks.rows[L], blocks.cols[L], blocks.types[L]):
        if typ == F:
            Fd.append(dense_scale * g(tree.size(L, t), tree.size(L, s)))
        else:
            Fd.append(None)
    return H2Matrix(tree, blocks, V, Er, W, Ec, S, Fd)


def identity_h2(like):
    """The identity in the partition of `like`: dense diagonal blocks equal to
    I, every other dense block and every coupling zero; bases copied."""
    L = like.L
    cdt = like.dtype
    S = [[None if s is None else np.zeros_like(s) for s in sl] for sl in like.S]
    Fd = []
    for t, s, f in zip(like.blocks.rows[L], like.blocks.cols[L], like.F):
        if f is None:
            Fd.append(None)
        elif t == s:
            Fd.append(np.eye(f.shape[0], dtype=cdt))
        else:
            Fd.append(np.zeros_like(f))
    return H2Matrix(like.tree, like.blocks, like.V, like.Er, like.W, like.Ec, S, Fd)
