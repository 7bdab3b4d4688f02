"""The allocation-free exact mat-vec captured in a HIP graph (through torch's
graph capture on a torch stream) and replayed: every replay, with eager work
and synchronisations between replays, equals the eager library mat-vec bit
for bit, real and complex."""
import numpy as np
import pytest

import paper_1908_05218_amd as h2
from tests import cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = h2.Context(0)
    yield c
    c.close()


def _capture(ctx, M, x, y):
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        h2.matvec_noalloc(ctx, M, x, y, stream=s)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        h2.matvec_noalloc(ctx, M, x, y, stream=s)
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("nrhs", [1, 3])
def test_graph_replays_equal_eager_matvec(ctx, nrhs):
    import torch
    print(f"case graph matvec plates2048 nrhs={nrhs}", flush=True)
    A = cases.plates(2048)
    M = h2.load(ctx, A.to_flat())
    n = A.n
    x = torch.zeros((nrhs, n), dtype=torch.float64, device="cuda")  # column-major n x nrhs
    y = torch.zeros_like(x)
    g = _capture(ctx, M, x, y)
    rng = np.random.default_rng(4)
    for rep in range(4):
        xs = rng.standard_normal((nrhs, n))
        x.copy_(torch.from_numpy(xs))
        g.replay()
        torch.cuda.synchronize()
        want = h2.matvec(ctx, M, xs.T.copy() if nrhs > 1 else xs[0])
        got = y.cpu().numpy()
        got = got.T if nrhs > 1 else got[0]
        assert np.array_equal(got, want), rep
        # eager work of the program between replays
        torch.cuda.synchronize()
        (x * 2.0).sum().item()


def test_graph_replays_complex(ctx):
    import torch
    print("case graph matvec random_complex1024", flush=True)
    A, _ = cases.random_pair(1024, 32, 8, 6, 13, complex_=True)
    M = h2.load(ctx, A.to_flat())
    n = A.n
    x = torch.zeros(2 * n, dtype=torch.float64, device="cuda")  # planar: real, then imaginary
    y = torch.zeros_like(x)
    g = _capture(ctx, M, x, y)
    rng = np.random.default_rng(5)
    for rep in range(3):
        xs = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        x.copy_(torch.from_numpy(np.concatenate([xs.real, xs.imag])))
        g.replay()
        torch.cuda.synchronize()
        yy = y.cpu().numpy()
        got = yy[:n] + 1j * yy[n:]
        want = h2.matvec(ctx, M, xs)
        assert np.array_equal(got, want), rep
