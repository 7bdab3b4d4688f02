"""Degenerate inputs of the product on the GPU, through the C-ABI, against
the CPU checker or the dense product: a single point, a single leaf, a
partition with no admissible block (every leaf block dense: the product is
exact at any eps), the zero matrix (empty Gram sums: no non-finite value,
C = 0), and an eps so large that one vector per cluster is kept."""
import numpy as np
import pytest

import paper_1908_05218_amd as h2
from h2inputs import points
from h2inputs.build import LaplaceKernel, chebyshev_h2
from h2inputs.h2data import H2Matrix
from h2inputs.structure import BlockTree, ClusterTree
from oracle import h2ops, mmp as omp
from tests import cases

pytestmark = pytest.mark.gpu


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


@pytest.fixture(scope="module")
def ctx():
    c = h2.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n", [1, 2, 3, 31])
def test_single_leaf_products(ctx, n):
    print(f"case single leaf n={n}", flush=True)
    pts = points.cube(n, 11)
    t = ClusterTree(pts, 32)
    A = chebyshev_h2(t, BlockTree(t, 1.0), LaplaceKernel(1.0), 2)
    dA = h2.load(ctx, A.to_flat())
    ref = h2ops.to_dense(A) @ h2ops.to_dense(A)
    for eps in (0.0, 1e-4):
        C = h2.mmp(ctx, dA, dA, eps)
        assert rel(h2.to_dense(ctx, C, n), ref) < 1e-12


def test_no_admissible_block(ctx):
    """eta so small that no block is admissible: C = A A exactly, at any eps."""
    print("case all-dense partition", flush=True)
    pts = points.plates_random(600, 0.1, 1e-3, 4)
    t = ClusterTree(pts, 16)
    b = BlockTree(t, 1e-6)
    assert b.count(1) == (1 << t.L) ** 2  # every leaf block dense
    A = chebyshev_h2(t, b, LaplaceKernel(1.0), 2)
    dA = h2.load(ctx, A.to_flat())
    C = h2.mmp(ctx, dA, dA, 1e-2)
    assert rel(h2.to_dense(ctx, C, A.n), h2ops.to_dense(A) @ h2ops.to_dense(A)) < 1e-12


def test_zero_matrix(ctx):
    print("case zero matrix", flush=True)
    A = cases.plates(1024, leaf=16, order=2)
    Z = H2Matrix(A.tree, A.blocks, A.V, A.Er, A.W, A.Ec,
                 [[None if s is None else np.zeros_like(s) for s in sl] for sl in A.S],
                 [None if f is None else np.zeros_like(f) for f in A.F])
    dZ = h2.load(ctx, Z.to_flat())
    C = h2.mmp(ctx, dZ, dZ, 1e-4)
    D = h2.to_dense(ctx, C, A.n)
    assert np.all(np.isfinite(D)) and np.abs(D).max() == 0.0
    x = np.random.default_rng(1).standard_normal(A.n)
    assert np.abs(h2.matvec(ctx, C, x)).max() == 0.0


def test_eps_large_keeps_one_vector(ctx):
    """PAPER mode at eps = 1: the threshold lambda_1 keeps exactly one vector
    per cluster; ACCURACY mode at eps = 1 keeps the checker's ranks."""
    print("case eps = 1", flush=True)
    A = cases.plates(2048)
    dA = h2.load(ctx, A.to_flat())
    for mode, om in (("paper", omp.PAPER), ("accuracy", omp.ACCURACY)):
        C = h2.mmp(ctx, dA, dA, 1.0, mode=mode)
        exp = h2.export(C)
        _, info = omp.h2_mmp(A, A, 1.0, mode=om)
        lmin = info["lmin"]
        for key, r in (("krow", "ranks_row"), ("kcol", "ranks_col")):
            got = np.asarray(exp[key])
            for lev in range(lmin, A.L + 1):
                ref = np.asarray(info[r][lev])
                g = got[(1 << lev) - 1:(2 << lev) - 1]
                assert np.array_equal(g, ref), (mode, key, lev)
                if mode == "paper":
                    assert g.max() == 1
