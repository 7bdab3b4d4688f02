"""GPU parity for complex128 H^2 matrices (the Helmholtz-type inputs of
Section VI's scattering examples): the HIP library through the C-ABI against
the CPU checker on the same seeded inputs.  Tolerances as for real data:
mat-vec and dense expansion 1e-13 relative, EXACT products 1e-12 relative to
the dense product, ACCURACY products within eps of AB and of the checker's
C, kept ranks equal on >= 99 % of clusters (|difference| <= 2 elsewhere),
new bases orthonormal in the Hermitian sense."""
import numpy as np
import pytest

import paper_1908_05218_amd as h2
from h2inputs.h2data import H2Matrix
from oracle import h2ops, mmp as omp
from tests import cases

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def ctx():
    c = h2.Context(0)
    yield c
    c.close()


CASES = {
    "random_complex": lambda: cases.random_pair(512, 16, 5, 6, 21, complex_=True),
    "helmholtz_sphere1k": lambda: cases.helmholtz_sphere(1024, 32, 2, 20.0),
}


def _load(ctx, A, B):
    return h2.load(ctx, A.to_flat()), h2.load(ctx, B.to_flat())


@pytest.mark.parametrize("name", list(CASES))
def test_complex_matvec_dense_export(ctx, name):
    print(f"case complex matvec {name}", flush=True)
    A, B = CASES[name]()
    dA, _ = _load(ctx, A, B)
    x = np.random.default_rng(4).standard_normal((A.n, 2)) + 1j * np.random.default_rng(5).standard_normal((A.n, 2))
    ref = h2ops.to_dense(A) @ x
    assert rel(h2.matvec(ctx, dA, x), ref) < 1e-13
    assert rel(h2.to_dense(ctx, dA, A.n), h2ops.to_dense(A)) < 1e-13
    d = h2.export(dA)
    f = A.to_flat()
    assert d["is_complex"] == 1
    for k in ("V", "W", "Er", "Ec", "S", "F"):
        assert np.array_equal(np.asarray(d[k]), np.asarray(f[k], dtype=np.complex128)), k


@pytest.mark.parametrize("name", list(CASES))
def test_complex_exact_mode_reproduces_dense_product(ctx, name):
    print(f"case complex exact {name}", flush=True)
    A, B = CASES[name]()
    dA, dB = _load(ctx, A, B)
    dC = h2.mmp(ctx, dA, dB, 0.0)
    ref = h2ops.to_dense(A) @ h2ops.to_dense(B)
    assert rel(h2.to_dense(ctx, dC, A.n), ref) < 1e-12
    C = H2Matrix.from_flat(h2.export(dC))
    assert C.blocks.same_as(A.blocks)


def _rank_agreement(Cg, info):
    rg = np.concatenate([np.asarray(Cg["krow"]), np.asarray(Cg["kcol"])])
    ro = []
    for key in ("ranks_row", "ranks_col"):
        flat = []
        for lev, r in enumerate(info[key]):
            flat.extend(r if lev >= info["lmin"] else [0] * len(r))
        ro.append(np.array(flat))
    d = np.abs(rg - np.concatenate(ro))
    return float(np.mean(d == 0)), int(d.max())


@pytest.mark.parametrize("name,eps", [("random_complex", 1e-4), ("helmholtz_sphere1k", 1e-3),
                                      ("helmholtz_sphere1k", 1e-6)])
def test_complex_accuracy_mode_matches_checker(ctx, name, eps):
    print(f"case complex accuracy {name} eps {eps}", flush=True)
    A, B = CASES[name]()
    dA, dB = _load(ctx, A, B)
    dC = h2.mmp(ctx, dA, dB, eps)
    Co, info = omp.h2_mmp(A, B, eps)
    ref = h2ops.to_dense(A) @ h2ops.to_dense(B)
    Dg = h2.to_dense(ctx, dC, A.n)
    Do = h2ops.to_dense(Co)
    assert rel(Dg, ref) <= eps
    assert np.linalg.norm(Dg - Do) <= eps * np.linalg.norm(Do)
    exp = h2.export(dC)
    frac, dmax = _rank_agreement(exp, info)
    assert frac >= 0.99 and dmax <= 2, (frac, dmax)
    C = H2Matrix.from_flat(exp)
    assert C.blocks.same_as(A.blocks)
    for v in C.V + C.W:
        assert np.abs(v.conj().T @ v - np.eye(v.shape[1])).max() < 1e-12


def test_complex_errors(ctx):
    A, B = CASES["random_complex"]()
    dA, dB = _load(ctx, A, B)
    with pytest.raises(h2.H2Error) as e:
        h2.mmp(ctx, dA, dB, 1e-4, precision="fp32_bulk")
    assert e.value.code == 6
    R, _ = cases.random_pair(512, 16, 5, 6, 21)
    dR = h2.load(ctx, R.to_flat())
    with pytest.raises(h2.H2Error) as e:
        h2.mmp(ctx, dA, dR, 1e-4)
    assert e.value.code == 1


def test_helmholtz_build_matches_input_builder(ctx):
    """h2_build with the Helmholtz kernel = the Python input builder (same
    tree, partition, Chebyshev bases; couplings and dense blocks to
    rounding), and its products agree with the checker's."""
    from h2inputs import points
    print("case helmholtz build sphere1k", flush=True)
    n, kappa = 1024, 20.0
    A, _ = cases.helmholtz_sphere(n, 32, 2, kappa)
    rho = 2.0 / np.sqrt(n)
    sv = 1 / (2 * np.pi * rho) - 1j * kappa / (4 * np.pi)
    M = h2.build(ctx, points.fibonacci_sphere(n), 32, 1.0, 2, sv, kernel="helmholtz",
                 wavenumber=kappa)
    d, f = h2.export(M), A.to_flat()
    for k in ("leaf_off", "perm", "node_off", "node_row", "node_col", "node_type", "krow", "kcol"):
        assert np.array_equal(np.asarray(d[k]), np.asarray(f[k])), k
    for k in ("V", "W", "Er", "Ec", "S", "F"):
        a, b = np.asarray(d[k]), np.asarray(f[k], dtype=np.complex128)
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max(), k
    dA = h2.load(ctx, f)
    C1 = h2.to_dense(ctx, h2.mmp(ctx, M, M, 1e-4), n)
    C2 = h2.to_dense(ctx, h2.mmp(ctx, dA, dA, 1e-4), n)
    assert rel(C1, C2) < 1e-10
