"""Pins of the checker's recompression (oracle/recompress.py) against facts
that do not go through its weight recursion: the dense matrix, singular
value decompositions of each cluster's far field taken from it (the
Eckart-Young optimum), orthonormality, an exactly low-rank kernel, and
planted mistakes that these pins must catch."""
import numpy as np
import pytest

from h2inputs.build import chebyshev_h2
from h2inputs.structure import BlockTree, ClusterTree, R
from h2inputs import points
from oracle import h2ops
from oracle import recompress as rc
from oracle.mmp import ACCURACY, threshold, truncated_levels
from tests import cases


def _cases():
    A, _ = cases.random_pair(1024, 32, 10, 7, 11)
    Z, _ = cases.random_pair(1024, 32, 8, 6, 13, complex_=True)
    H, _ = cases.helmholtz_sphere(1024, 32, 3, 12.0)
    return {"cube1k": cases.cube1k(), "plates2048": cases.plates(2048),
            "random_nonsym": A, "random_complex": Z, "helmholtz1k": H}


CASES = _cases()


def _far_columns(M, lev, t):
    """Columns (tree order) of the admissible blocks of t and its ancestors."""
    T, cols = M.tree, []
    for up in range(lev, -1, -1):
        a = t >> (lev - up)
        for r, s, typ in zip(M.blocks.rows[up], M.blocks.cols[up], M.blocks.types[up]):
            if int(r) == a and typ == R:
                cols.extend(range(T.start(up, int(s)), T.stop(up, int(s))))
    return np.array(sorted(cols), dtype=np.int64)


def _check_side(M, M2, D, tau, side):
    """Every cluster's new basis against the SVD of its far field (leaves) or
    of the far field projected onto the children's new bases (above)."""
    L, lmin, T = M.L, M.blocks.min_admissible_level(), M.tree
    Dside = D if side == 0 else D.T
    expand = h2ops.expanded_row_basis if side == 0 else h2ops.expanded_col_basis
    E2 = M2.Er if side == 0 else M2.Ec
    kold = M.krow if side == 0 else M.kcol
    checked = 0
    for lev in range(L, lmin - 1, -1):
        for t in range(1 << lev):
            far = _far_columns(M, lev, t) if side == 0 else None
            if side == 1:
                # column side: far field of the transpose, the blocks (t', s)
                # with s = t or an ancestor
                cols = []
                for up in range(lev, -1, -1):
                    a = t >> (lev - up)
                    for r, s, typ in zip(M.blocks.rows[up], M.blocks.cols[up],
                                         M.blocks.types[up]):
                        if int(s) == a and typ == R:
                            cols.extend(range(T.start(up, int(r)), T.stop(up, int(r))))
                far = np.array(sorted(cols), dtype=np.int64)
            if far.size == 0:
                continue
            Y = Dside[T.start(lev, t):T.stop(lev, t)][:, far]
            if lev == L:
                Un = M2.V[t] if side == 0 else M2.W[t]
            else:
                Q1, Q2 = expand(M2, lev + 1, 2 * t), expand(M2, lev + 1, 2 * t + 1)
                Q = np.zeros((Q1.shape[0] + Q2.shape[0], Q1.shape[1] + Q2.shape[1]), dtype=Y.dtype)
                Q[:Q1.shape[0], :Q1.shape[1]] = Q1
                Q[Q1.shape[0]:, Q1.shape[1]:] = Q2
                Y = Q.conj().T @ Y
                Un = np.vstack([E2[lev + 1][2 * t], E2[lev + 1][2 * t + 1]])
            sig = np.linalg.svd(Y, compute_uv=False)
            k = Un.shape[1]
            res = np.linalg.norm(Y - Un @ (Un.conj().T @ Y)) ** 2
            opt = float(np.sum(sig[k:] ** 2))
            assert res <= opt * (1 + 1e-6) + 1e-12 * sig[0] ** 2, (side, lev, t, res, opt)
            lam = sig ** 2
            near = np.abs(lam / (tau * lam[0]) - 1.0) < 1e-3
            if not near.any():
                want = max(1, min(int(np.count_nonzero(lam > tau * lam[0])), kold(lev, t)))
                assert k == want, (side, lev, t, k, want)
            checked += 1
    assert checked > 0


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("eps", [1e-3, 1e-6])
def test_bases_are_the_far_field_svd(name, eps):
    M = CASES[name]
    M2, info = rc.recompress(M, eps)
    D = h2ops.to_dense_tree_order(M)
    tau = threshold(eps, ACCURACY, levels=truncated_levels(M.L, info["lmin"]))
    _check_side(M, M2, D, tau, 0)
    _check_side(M, M2, D, tau, 1)


@pytest.mark.parametrize("name", sorted(CASES))
def test_error_within_eps_and_ranks_shrink(name):
    M = CASES[name]
    D = h2ops.to_dense(M)
    nD = np.linalg.norm(D)
    prev = None
    for eps in (1e-7, 1e-5, 1e-3):
        M2, info = rc.recompress(M, eps)
        err = np.linalg.norm(h2ops.to_dense(M2) - D) / nD
        assert err <= eps, (eps, err)
        # the mat-vec of the recompressed matrix agrees with its dense form
        x = np.random.default_rng(1).standard_normal(M.n)
        assert np.linalg.norm(h2ops.matvec(M2, x) - h2ops.to_dense(M2) @ x) <= 1e-12 * nD * np.linalg.norm(x)
        L = M.L
        for lev in range(info["lmin"], L + 1):
            for c in range(1 << lev):
                assert M2.krow(lev, c) <= M.krow(lev, c)
                assert M2.kcol(lev, c) <= M.kcol(lev, c)
        tot = sum(sum(r) for r in info["ranks_row"]) + sum(sum(r) for r in info["ranks_col"])
        if prev is not None:
            assert tot <= prev
        prev = tot


@pytest.mark.parametrize("name", ["plates2048", "helmholtz1k"])
def test_bases_orthonormal(name):
    M2, info = rc.recompress(CASES[name], 1e-5)
    for X in M2.V + M2.W:
        assert np.allclose(X.conj().T @ X, np.eye(X.shape[1]), atol=1e-12)
    for E in (M2.Er, M2.Ec):
        for lev in range(info["lmin"] + 1, M2.L + 1):
            for p in range(1 << (lev - 1)):
                T = np.vstack([E[lev][2 * p], E[lev][2 * p + 1]])
                assert np.allclose(T.conj().T @ T, np.eye(T.shape[1]), atol=1e-12)


class _Bilinear:
    """1 + x.y: separable of rank 4 in three dimensions."""
    dtype = np.dtype(np.float64)

    def __call__(self, X, Y):
        return 1.0 + X @ Y.T


def test_rank_four_kernel_recompresses_to_rank_four():
    pts = points.cube(1024, 5)
    t = ClusterTree(pts, 32)
    b = BlockTree(t, 1.0)
    M = chebyshev_h2(t, b, _Bilinear(), 3)
    M2, info = rc.recompress(M, 1e-6)
    D = h2ops.to_dense(M)
    assert np.linalg.norm(h2ops.to_dense(M2) - D) <= 1e-12 * np.linalg.norm(D)
    # rank 4 wherever there is a far field (symmetric partition: the row and
    # column far fields of a cluster are both empty or both not); one
    # vector where there is none
    for lev in range(info["lmin"], M.L + 1):
        for c in range(1 << lev):
            want = 4 if _far_columns(M, lev, c).size else 1
            assert M2.krow(lev, c) == want and M2.kcol(lev, c) == want, (lev, c)


def test_eps_floor():
    with pytest.raises(ValueError):
        rc.recompress(CASES["cube1k"], 1e-9)


def test_planted_missing_ancestor_weight_is_caught(monkeypatch):
    """Dropping the parent's far field from K_t (a plausible mistake) must
    fail the far-field SVD pin."""
    orig = rc.far_field_weights

    def planted(E, *a, **k):
        return orig([[None if e is None else np.zeros_like(e) for e in lev] for lev in E], *a, **k)
    monkeypatch.setattr(rc, "far_field_weights", planted)
    M = CASES["plates2048"]
    M2, info = rc.recompress(M, 1e-3)
    D = h2ops.to_dense_tree_order(M)
    tau = threshold(1e-3, ACCURACY, levels=truncated_levels(M.L, info["lmin"]))
    with pytest.raises(AssertionError):
        _check_side(M, M2, D, tau, 0)


def test_planted_unconjugated_basis_gram_is_caught(monkeypatch):
    """X^T X in place of X^T X^* (complex bases; the Chebyshev bases of the
    Helmholtz input are real) must fail the pins."""
    def planted(X, E, L):
        G = [None] * (L + 1)
        G[L] = [x.T @ x for x in X]
        for lev in range(L - 1, -1, -1):
            G[lev] = [E[lev + 1][2 * c].T @ G[lev + 1][2 * c] @ E[lev + 1][2 * c]
                      + E[lev + 1][2 * c + 1].T @ G[lev + 1][2 * c + 1] @ E[lev + 1][2 * c + 1]
                      for c in range(1 << lev)]
        return G
    monkeypatch.setattr(rc, "basis_grams", planted)
    M = CASES["random_complex"]
    M2, info = rc.recompress(M, 1e-3)
    D = h2ops.to_dense_tree_order(M)
    tau = threshold(1e-3, ACCURACY, levels=truncated_levels(M.L, info["lmin"]))
    with pytest.raises(AssertionError):
        _check_side(M, M2, D, tau, 0)
        _check_side(M, M2, D, tau, 1)
