"""The stream and allocator boundary of the C-ABI (h2_ctx_create with a
device-memory supplier, h2_mmp / h2_matvec on a caller stream, h2_sync),
driven through ctypes with PyTorch streams and PyTorch's caching allocator.
Products are deterministic, so results on any stream and from any memory
supplier are compared bit for bit."""
import numpy as np
import pytest

import paper_1908_05218_amd as h2
from tests import cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def test_torch_allocator_supplies_device_memory(torch):
    print("case torch allocator plates2048 eps 1e-4", flush=True)
    A = cases.plates(2048)
    ref_ctx = h2.Context(0)
    ctx = h2.Context(0, allocator="torch")
    try:
        before = torch.cuda.memory_allocated(0)
        dA = h2.load(ctx, A.to_flat())
        held = torch.cuda.memory_allocated(0) - before
        assert held > 0  # A's blocks live in torch's allocator
        torch.cuda.reset_peak_memory_stats(0)
        dC = h2.mmp(ctx, dA, dA, 1e-4, precision="fp32_bulk")
        assert torch.cuda.max_memory_allocated(0) > before + held
        rA = h2.load(ref_ctx, A.to_flat())
        rC = h2.mmp(ref_ctx, rA, rA, 1e-4, precision="fp32_bulk")
        e, r = h2.export(dC), h2.export(rC)
        for k in ("krow", "kcol", "V", "W", "Er", "Ec", "S", "F"):
            assert np.array_equal(np.asarray(e[k]), np.asarray(r[k])), k
        dC.free()
        dA.free()
    finally:
        ctx.close()
        ref_ctx.close()
    # every block went back to torch
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(0) == before


def test_product_and_matvec_ordered_on_a_torch_stream(torch):
    print("case stream ordering plates2048", flush=True)
    A = cases.plates(2048)
    ctx = h2.Context(0)
    try:
        dA = h2.load(ctx, A.to_flat())
        ref = h2.mmp(ctx, dA, dA, 1e-4)
        x = np.random.default_rng(4).standard_normal((A.n, 2))
        y_ref = h2.matvec(ctx, ref, x)
        s = torch.cuda.Stream(device=0)
        with torch.cuda.stream(s):
            # inputs produced on s, product and mat-vec queued on s without a
            # host wait in between, result consumed on s
            xt = torch.from_numpy(x).to("cuda:0", non_blocking=False).mul(1.0)
            C = h2.mmp(ctx, dA, dA, 1e-4, stream=s)
            yt = h2.matvec(ctx, C, xt, stream=s)
            out = (yt * 2.0).cpu()
        s.synchronize()
        h2.sync(C)
        assert np.array_equal(out.numpy(), 2.0 * y_ref)
        assert h2.stats(C)["mmp_ms"] > 0
        e, r = h2.export(C), h2.export(ref)
        assert np.array_equal(np.asarray(e["S"]), np.asarray(r["S"]))
    finally:
        ctx.close()


def test_async_products_on_two_streams(torch):
    """Two products queued on different caller streams of one context, then
    consumed: each equals the synchronous product."""
    print("case two streams cube1k", flush=True)
    A = cases.cube1k()
    ctx = h2.Context(0, allocator="torch")
    try:
        dA = h2.load(ctx, A.to_flat())
        ref = h2.to_dense(ctx, h2.mmp(ctx, dA, dA, 1e-6), A.n)
        s1, s2 = torch.cuda.Stream(device=0), torch.cuda.Stream(device=0)
        C1 = h2.mmp(ctx, dA, dA, 1e-6, stream=s1)
        C2 = h2.mmp(ctx, dA, dA, 1e-6, stream=s2)
        for C in (C1, C2):
            h2.sync(C)
            assert np.array_equal(h2.to_dense(ctx, C, A.n), ref)
    finally:
        ctx.close()


def test_torch_allocator_recompression_and_build(torch):
    """h2_build with recompression and h2_recompress drawing their device
    memory from torch's allocator give the same matrices, bit for bit, as a
    context with its own pool."""
    from h2inputs import configs
    print("case torch allocator: build + recompress plates4096", flush=True)
    w = configs.plates_n(4096)
    ref_ctx = h2.Context(0)
    ctx = h2.Context(0, allocator="torch")
    try:
        R1 = h2.build(ctx, w.pts, w.leaf_size, w.eta, w.order, w.kernel.self_value, recompress_eps=1e-5)
        R2 = h2.build(ref_ctx, w.pts, w.leaf_size, w.eta, w.order, w.kernel.self_value,
                      recompress_eps=1e-5)
        e, r = h2.export(R1), h2.export(R2)
        for k in ("krow", "kcol", "V", "W", "Er", "Ec", "S", "F"):
            assert np.array_equal(np.asarray(e[k]), np.asarray(r[k])), k
        R1.free()
        R2.free()
    finally:
        ctx.close()
        ref_ctx.close()
