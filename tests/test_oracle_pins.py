"""Pins of the CPU checker against facts the paper and the mathematics fix,
independent of the checker's own formulas.

  * structure: node counts of the synthetic unit-cube cases recomputed from
    the admissibility condition (equation admCond) by an independent probe;
  * the nested property of Section II (V_parent = diag(V_children) T);
  * the exact H^2 mat-vec equals the dense expansion (non-symmetric, complex);
  * EXACT mode (no truncation) reproduces the brute-force dense product A B
    to rounding, for real symmetric, real non-symmetric and complex inputs
    (Section V: every operation of the method is exact or eps-controlled);
  * ACCURACY mode meets ||C - AB||_F <= eps ||AB||_F on tiny N;
  * PAPER mode's error scales like sqrt(eps) (Tables I, II, IV);
  * C keeps the block partition of A and B (Section III);
  * the new bases are orthonormal; B = I gives C = A; A symmetric gives C
    symmetric; smaller eps gives smaller error and larger ranks;
  * scale invariance of the truncation (the normalisation of Section III-C
    makes each Gram component independent of the scale of its blocks):
    C(alpha A, B) = alpha C(A, B) with identical ranks;
  * the column side mirrors the row side: C(B^T, A^T) = C(A, B)^T with the
    row ranks of one equal to the column ranks of the other, for a real
    non-symmetric product and a complex one (which decides the conjugations
    of the column Grams, Section III-C and Section IV).
"""
import numpy as np
import pytest

from h2inputs.build import identity_h2
from oracle import h2ops, mmp
from tests import cases


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ------------------------------------------------------------ structure
def test_structure_counts_cube():
    # node counts of the same rules from an independent probe
    A = cases.cube1k()
    assert A.L == 5 and A.blocks.count(1) == 978 and A.blocks.count(0) == 46
    A = cases.cube(4096)
    assert A.L == 7 and A.blocks.count(1) == 7684 and A.blocks.count(0) == 4470
    assert A.blocks.min_admissible_level() == 5


def test_block_partition_covers_matrix_once():
    A = cases.plates(2048)
    cover = np.zeros((A.n, A.n), dtype=np.int32)
    t = A.tree
    for lev in range(A.L + 1):
        for i, j, typ in zip(A.blocks.rows[lev], A.blocks.cols[lev], A.blocks.types[lev]):
            if typ != 2:
                cover[t.start(lev, i):t.stop(lev, i), t.start(lev, j):t.stop(lev, j)] += 1
    assert (cover == 1).all()


def test_admissible_blocks_satisfy_condition():
    A = cases.plates(2048)
    t = A.tree
    for lev in range(A.L + 1):
        for i, j, typ in zip(A.blocks.rows[lev], A.blocks.cols[lev], A.blocks.types[lev]):
            if typ == 0:
                pi = t.points[t.indices(lev, i)]
                pj = t.points[t.indices(lev, j)]
                d = np.sqrt(((pi[:, None] - pj[None]) ** 2).sum(-1)).min()
                diam = max(np.linalg.norm(pi.max(0) - pi.min(0)), np.linalg.norm(pj.max(0) - pj.min(0)))
                assert diam <= d + 1e-12  # box gap <= point gap, eta = 1


# ------------------------------------------------------------ inputs
def test_chebyshev_nested_property():
    A = cases.plates(1024)
    from h2inputs.build import _BoxNodes
    t = A.tree
    root_diam = float(np.linalg.norm(t.hi[0][0] - t.lo[0][0]))
    for lev in (2, 4):
        for c in range(0, 1 << lev, 3):
            nodes = _BoxNodes(t.lo[lev][c], t.hi[lev][c], 3, 1e-9 * root_diam)
            direct = nodes.lagrange(t.points[t.indices(lev, c)])
            assert rel(h2ops.expanded_row_basis(A, lev, c), direct) < 1e-12


def test_chebyshev_approximates_kernel():
    A = cases.plates(1024)
    D = h2ops.to_dense(A)
    p = A.tree.points
    d = np.sqrt(((p[:, None] - p[None]) ** 2).sum(-1))
    with np.errstate(divide="ignore"):
        K = 1 / (4 * np.pi * d)
    np.fill_diagonal(K, np.diag(D))
    assert rel(D, K) < 5e-3


def test_matvec_matches_dense_nonsymmetric_complex():
    A, _ = cases.random_pair(512, 16, 6, 5, 3, complex_=True)
    D = h2ops.to_dense(A)
    x = np.random.default_rng(0).standard_normal((A.n, 3))
    assert rel(h2ops.matvec(A, x), D @ x) < 1e-13
    assert not np.allclose(D, D.T)


def test_identity_h2_is_identity():
    A = cases.plates(1024)
    assert np.array_equal(h2ops.to_dense(identity_h2(A)), np.eye(A.n))


# ------------------------------------------------------------ exact mode
@pytest.mark.parametrize("which", ["cube1k", "plates1024", "plates_leaf16", "ragged"])
def test_exact_mode_reproduces_dense_product_real(which):
    if which == "cube1k":
        A = B = cases.cube1k()
    elif which == "plates1024":
        A = B = cases.plates(1024)
    elif which == "plates_leaf16":
        A = B = cases.plates(1024, leaf=16, order=2)
    else:
        A = B = cases.ragged_plates(777, 12)
    C, info = mmp.h2_mmp(A, B, 0.0)
    DA = h2ops.to_dense(A)
    assert rel(h2ops.to_dense(C), DA @ DA) < 1e-13
    assert C.blocks.same_as(A.blocks)


def test_exact_mode_nonsymmetric_distinct_sides():
    A, B = cases.random_pair(512, 16, 6, 5, 11)
    C, _ = mmp.h2_mmp(A, B, 0.0)
    assert rel(h2ops.to_dense(C), h2ops.to_dense(A) @ h2ops.to_dense(B)) < 1e-12


def test_exact_mode_complex():
    A, B = cases.random_pair(512, 16, 5, 6, 21, complex_=True)
    C, _ = mmp.h2_mmp(A, B, 0.0)
    assert rel(h2ops.to_dense(C), h2ops.to_dense(A) @ h2ops.to_dense(B)) < 1e-12


def test_exact_mode_helmholtz_two_wavenumbers():
    A, B = cases.helmholtz_sphere(1024, 32, 2, 20.0)
    C, _ = mmp.h2_mmp(A, B, 0.0)
    assert rel(h2ops.to_dense(C), h2ops.to_dense(A) @ h2ops.to_dense(B)) < 1e-12


# ------------------------------------------------------------ accuracy mode
@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-6])
def test_accuracy_mode_meets_eps(eps):
    for A, B in [(cases.plates(2048),) * 2, cases.random_pair(512, 16, 6, 5, 4)]:
        C, info = mmp.h2_mmp(A, B, eps)
        ref = h2ops.to_dense(A) @ h2ops.to_dense(B)
        assert rel(h2ops.to_dense(C), ref) <= eps


def test_accuracy_complex_meets_eps():
    A, B = cases.helmholtz_sphere(1024, 32, 2, 20.0)
    C, _ = mmp.h2_mmp(A, B, 1e-4)
    assert rel(h2ops.to_dense(C), h2ops.to_dense(A) @ h2ops.to_dense(B)) <= 1e-4


def test_monotone_in_eps():
    A = cases.plates(2048)
    ref = h2ops.to_dense(A) @ h2ops.to_dense(A)
    errs, ranks = [], []
    for eps in (1e-2, 1e-4, 1e-6):
        C, info = mmp.h2_mmp(A, A, eps)
        errs.append(rel(h2ops.to_dense(C), ref))
        ranks.append(sum(sum(r) for r in info["ranks_row"]))
    assert errs[0] > errs[1] > errs[2]
    assert ranks[0] < ranks[1] < ranks[2]


def test_paper_mode_error_scales_like_sqrt_eps():
    A = cases.plates(2048)
    x = np.random.default_rng(2).standard_normal(A.n)
    for eps in (1e-2, 1e-4):
        C, _ = mmp.h2_mmp(A, A, eps, mode=mmp.PAPER)
        e = h2ops.relative_error(C, A, A, x)
        assert 1e-3 * np.sqrt(eps) < e < np.sqrt(eps)


# ------------------------------------------------------------ invariants
def _orthonormality_defects(C):
    L = C.L
    out = [np.abs(v.conj().T @ v - np.eye(v.shape[1])).max() for v in C.V + C.W]
    lmin = C.blocks.min_admissible_level()
    for lev in range(lmin, L):
        for c in range(1 << lev):
            for E in (C.Er, C.Ec):
                T = np.vstack([E[lev + 1][2 * c], E[lev + 1][2 * c + 1]])
                out.append(np.abs(T.conj().T @ T - np.eye(T.shape[1])).max())
    return max(out)


def test_new_bases_orthonormal():
    A = cases.plates(2048)
    C, _ = mmp.h2_mmp(A, A, 1e-4)
    assert _orthonormality_defects(C) < 1e-13


def test_times_identity_returns_a():
    A = cases.plates(2048)
    C, _ = mmp.h2_mmp(A, identity_h2(A), 1e-6)
    DA = h2ops.to_dense(A)
    assert rel(h2ops.to_dense(C), DA) <= 1e-6


def test_symmetric_square_is_symmetric():
    A = cases.plates(2048)
    C, info = mmp.h2_mmp(A, A, 1e-4)
    D = h2ops.to_dense(C)
    assert np.linalg.norm(D - D.T) <= 1e-4 * np.linalg.norm(D)
    assert info["ranks_row"] == info["ranks_col"]


def test_relative_error_criterion_small_when_exact():
    A = cases.plates(1024)
    C, _ = mmp.h2_mmp(A, A, 0.0)
    x = np.random.default_rng(9).standard_normal(A.n)
    assert h2ops.relative_error(C, A, A, x) < 1e-13


# ------------------------------------------------------------ planted mistakes
def _exact_error(A, B):
    C, _ = mmp.h2_mmp(A, B, 0.0)
    return rel(h2ops.to_dense(C), h2ops.to_dense(A) @ h2ops.to_dense(B))


def test_planted_dropped_term_is_caught(monkeypatch):
    """Dropping the admissible-admissible products must break the exact pin."""
    A, B = cases.random_pair(512, 16, 6, 5, 11)
    assert _exact_error(A, B) < 1e-12
    orig = mmp.Symbolic.triples
    monkeypatch.setattr(mmp.Symbolic, "triples",
                        lambda self, lev: [t for t in orig(self, lev) if not (t[5] == 0 and t[6] == 0)])
    assert _exact_error(A, B) > 1e-6


def test_planted_swapped_children_is_caught(monkeypatch):
    """Swapping the two children in the block-diagonal projections (a wrong
    index) must break the exact pin."""
    A, B = cases.random_pair(512, 16, 6, 6, 12)
    orig = mmp._blockdiag
    monkeypatch.setattr(mmp, "_blockdiag", lambda a, b: orig(b, a))
    assert _exact_error(A, B) > 1e-6


# ------------------------------------------------------------ scale and mirror
def _flat(info, key):
    return [r for lev, rr in enumerate(info[key]) if lev >= info["lmin"] for r in rr]


@pytest.mark.parametrize("alpha", [2.0 ** 10, 2.0 ** -10])
def test_scale_invariance(alpha):
    """Powers of two scale every floating-point step exactly, so the kept
    ranks must be identical and C must scale exactly."""
    A = cases.plates(2048)
    C, info = mmp.h2_mmp(A, A, 1e-4)
    Cs, infos = mmp.h2_mmp(cases.scaled_h2(A, alpha), A, 1e-4)
    assert infos["ranks_row"] == info["ranks_row"] and infos["ranks_col"] == info["ranks_col"]
    assert rel(h2ops.to_dense(Cs), alpha * h2ops.to_dense(C)) < 1e-14


def test_planted_missing_normalisation_is_caught(monkeypatch):
    """Summing the Gram components without dividing by their traces must
    break scale invariance."""
    orig = mmp.truncated_basis
    monkeypatch.setattr(mmp, "truncated_basis",
                        lambda comps, tau: orig([(g, 1.0 if tr > 0 else 0.0) for g, tr in comps], tau))
    A = cases.plates(2048)
    _, info = mmp.h2_mmp(A, A, 1e-4)
    _, infos = mmp.h2_mmp(cases.scaled_h2(A, 2.0 ** 10), A, 1e-4)
    assert infos["ranks_row"] != info["ranks_row"]


def _mirror(A, B, eps):
    C, info = mmp.h2_mmp(A, B, eps)
    Ct, infot = mmp.h2_mmp(cases.transpose_h2(B), cases.transpose_h2(A), eps)
    D, Dt = h2ops.to_dense(C), h2ops.to_dense(Ct)
    return rel(Dt, D.T), info, infot, D


def test_transpose_mirror_real_nonsymmetric():
    A, B = cases.plates_two_orders(2048)
    err, info, infot, D = _mirror(A, B, 1e-4)
    assert err < 1e-12
    assert _flat(infot, "ranks_row") == _flat(info, "ranks_col")
    assert _flat(infot, "ranks_col") == _flat(info, "ranks_row")
    # the product really is non-symmetric, so the check is not vacuous
    assert np.linalg.norm(D - D.T) > 1e3 * err * np.linalg.norm(D)
    assert _flat(info, "ranks_row") != _flat(info, "ranks_col")


def test_transpose_mirror_complex():
    A, B = cases.helmholtz_sphere(1024, 32, 2, 20.0)
    err, info, infot, D = _mirror(A, B, 1e-3)
    assert err < 1e-12
    assert _flat(infot, "ranks_row") == _flat(info, "ranks_col")
    assert _flat(infot, "ranks_col") == _flat(info, "ranks_row")
    assert np.linalg.norm(D - D.T) > 1e3 * err * np.linalg.norm(D)


def test_planted_unconjugated_column_gram_is_caught(monkeypatch):
    """A column Gram formed as Z^T Z (no conjugate) must break the complex
    mirror."""
    monkeypatch.setattr(mmp._Gram, "add_col",
                        lambda self, Z: (self.G.__iadd__(Z.T @ Z),
                                         setattr(self, "tr", self.tr + float(np.vdot(Z, Z).real))))
    A, B = cases.helmholtz_sphere(1024, 32, 2, 20.0)
    err, _, _, _ = _mirror(A, B, 1e-3)
    assert err > 1e-8


# ------------------------------------------------------------ fixed-basis mode
def test_fixed_basis_times_identity_is_a():
    """A I in fixed-basis mode: every contribution already lies in A's bases,
    so the projections are exact."""
    A = cases.plates(2048)
    C, _ = mmp.h2_mmp(A, identity_h2(A), 0.0, mode=mmp.FIXED)
    DA = h2ops.to_dense(A)
    assert rel(h2ops.to_dense(C), DA) < 1e-11


def test_fixed_basis_keeps_the_input_spans():
    """The new row bases of C span A's row bases and the column bases span
    B's, on every level from the leaves to l_min (nested bases expanded)."""
    A, B = cases.plates_two_orders(2048)
    C, info = mmp.h2_mmp(A, B, 0.0, mode=mmp.FIXED)
    for lev in range(info["lmin"], A.L + 1):
        for c in range(0, 1 << lev, max(1, (1 << lev) // 8)):
            for exp, M, N in ((h2ops.expanded_row_basis, C, A), (h2ops.expanded_col_basis, C, B)):
                Q, X = exp(M, lev, c), exp(N, lev, c)
                assert Q.shape[1] == X.shape[1]
                assert np.linalg.norm(X - Q @ (Q.conj().T @ X)) <= 1e-11 * np.linalg.norm(X)


def test_fixed_basis_error_well_above_proposed():
    """Table IV's claim on synthetic data: the fixed-basis product's error
    is far above the proposed product's at eps = 1e-4."""
    for A in (cases.plates(2048), cases.cube(2048)):
        ref = h2ops.to_dense(A) @ h2ops.to_dense(A)
        Cf, _ = mmp.h2_mmp(A, A, 0.0, mode=mmp.FIXED)
        Ca, _ = mmp.h2_mmp(A, A, 1e-4)
        ef, ea = rel(h2ops.to_dense(Cf), ref), rel(h2ops.to_dense(Ca), ref)
        assert ef > 10 * ea and ea <= 1e-4, (ef, ea)


# ------------------------------------------------------------ Newton-Schulz inverse
def _ns_dense(D, alpha, steps):
    X = alpha * np.eye(D.shape[0])
    for _ in range(steps):
        X = X @ (2.0 * np.eye(D.shape[0]) - D @ X)
    return X


def test_newton_schulz_exact_mode_equals_dense_iteration():
    """With exact products every iterate equals the dense Newton-Schulz
    iterate, in both a symmetric and a non-symmetric (complex) case."""
    from oracle import inverse
    A = cases.plates(1024, leaf=16, order=2)
    D = h2ops.to_dense(A)
    alpha = 1.0 / np.linalg.eigvalsh(D).max()
    for steps in (1, 4):
        X, _ = inverse.newton_schulz(A, 0.0, alpha, steps)
        ref = _ns_dense(D, alpha, steps)
        assert rel(h2ops.to_dense(X), ref) < 1e-12
    Ac, _ = cases.random_pair(512, 16, 6, 5, 11, complex_=True)
    Dc = h2ops.to_dense(Ac)
    a = 0.5 / np.linalg.norm(Dc, 2) ** 2
    # for a general matrix the iteration runs on A^H-scaled starts; here only
    # the algebra of the first steps is compared
    X, _ = inverse.newton_schulz(Ac, 0.0, a, 3)
    assert rel(h2ops.to_dense(X), _ns_dense(Dc, a, 3)) < 1e-12


def test_newton_schulz_converges_to_the_inverse():
    """Symmetric positive definite A, alpha = 1/lambda_max: the residual
    falls quadratically once below 1/2 and the limit is the inverse of the
    dense matrix within the product's accuracy."""
    from oracle import inverse
    from h2inputs import vectors
    A = cases.plates(1024)
    D = h2ops.to_dense(A)
    w = np.linalg.eigvalsh(D)
    X, res = inverse.newton_schulz(A, 1e-6, 1.0 / w.max(), 12, probes=vectors.probes(A.n, 2, 7))
    # I - A X_{j+1} = (I - A X_j)^2: the probe residual falls about quadratically
    for a, b in zip(res, res[1:]):
        if 1e-8 < a < 0.1:
            assert b < 10 * a * a + 1e-10
    assert res[-1] < 1e-8
    Ainv = np.linalg.inv(D)
    assert rel(h2ops.to_dense(X), Ainv) < 1e-8
