"""Newton-Schulz inverse by repeated products on the GPU (h2_scale_shift,
h2_newton_schulz through the C-ABI) against the oracle's iteration on the
same seeded inputs.

  * a M + b I equals the oracle's scale-and-shift to rounding (1e-15);
  * EXACT products: every iterate equals the oracle's (which equals the
    dense iteration, pinned on the CPU) to 1e-11;
  * ACCURACY products at eps = 1e-6: the converged iterates agree with the
    oracle's and with the dense inverse to 1e-7 (both limits lie within
    the products' accuracy of A^-1), the residual ||x - A X x|| / ||x||
    reaches 1e-8; FP32-bulk reaches the FP32 rounding level (1e-5)."""
import numpy as np
import pytest

import paper_1908_05218_amd as h2
from h2inputs import vectors
from oracle import h2ops, inverse
from tests import cases

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def ctx():
    c = h2.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def plates():
    A = cases.plates(1024)
    D = h2ops.to_dense(A)
    return A, D, 1.0 / np.linalg.eigvalsh(D).max()


def test_scale_shift_matches_oracle(ctx, plates):
    print("case scale_shift plates1024", flush=True)
    A, D, _ = plates
    dA = h2.load(ctx, A.to_flat())
    for a, b in ((-0.25, 2.0), (3.0, 0.0), (0.0, 1.5)):
        got = h2.to_dense(ctx, h2.scale_shift(ctx, dA, a, b), A.n)
        ref = h2ops.to_dense(inverse.scale_shift(A, a, b))
        assert np.abs(got - ref).max() <= 1e-15 * np.abs(ref).max()


def test_newton_schulz_exact_products(ctx, plates):
    print("case newton-schulz exact plates1024", flush=True)
    A, D, alpha = plates
    dA = h2.load(ctx, A.to_flat())
    for steps in (1, 3, 6):
        X = h2.newton_schulz(ctx, dA, alpha, steps, 0.0)
        Xo, _ = inverse.newton_schulz(A, 0.0, alpha, steps)
        assert rel(h2.to_dense(ctx, X, A.n), h2ops.to_dense(Xo)) < 1e-11


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_newton_schulz_converges(ctx, plates, precision):
    print(f"case newton-schulz eps 1e-6 {precision} plates1024", flush=True)
    A, D, alpha = plates
    dA = h2.load(ctx, A.to_flat())
    X = h2.newton_schulz(ctx, dA, alpha, 12, 1e-6, precision=precision)
    Dx = h2.to_dense(ctx, X, A.n)
    x = vectors.probes(A.n, 2, 7)
    r = x - h2.matvec(ctx, dA, h2.matvec(ctx, X, x))
    res = float(np.linalg.norm(r) / np.linalg.norm(x))
    Ainv = np.linalg.inv(D)
    if precision == "fp64":
        Xo, reso = inverse.newton_schulz(A, 1e-6, alpha, 12, probes=x)
        print(f"residual {res:.2e} (oracle {reso[-1]:.2e})", flush=True)
        assert res < 1e-8
        assert rel(Dx, h2ops.to_dense(Xo)) < 1e-7
        assert rel(Dx, Ainv) < 1e-7
    else:
        print(f"residual {res:.2e}", flush=True)
        assert res < 1e-5 and rel(Dx, Ainv) < 1e-5
