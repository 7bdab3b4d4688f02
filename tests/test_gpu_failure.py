"""Products stopped by the context's device-memory budget.  A budget sweep
stops FP32-bulk products at many points of the upward pass, among them
after the products deferred to the helper stream have started: each failed
call raises H2_ERR_OOM, leaves A usable (its mat-vec unchanged, bit for bit)
and leaves no work behind that corrupts a later call; a budget that fits
gives the same C as an unbounded context.  The condition is forced from the
host (the allocator refuses), so every kernel ends normally."""
import numpy as np
import pytest

import paper_1908_05218_amd as h2
from tests import cases

pytestmark = pytest.mark.gpu


def test_out_of_budget_products_leave_the_context_usable():
    print("case budget sweep plates4096 fp32_bulk", flush=True)
    A = cases.plates(4096)
    x = np.random.default_rng(3).standard_normal(A.n)
    ref_ctx = h2.Context(0)
    try:
        rA = h2.load(ref_ctx, A.to_flat())
        rC = h2.mmp(ref_ctx, rA, rA, 1e-4, precision="fp32_bulk")
        peak = h2.stats(rC)["bytes_device"]
        y_a = h2.matvec(ref_ctx, rA, x)
        y_c = h2.matvec(ref_ctx, rC, x)
    finally:
        ref_ctx.close()
    assert peak > 0
    failed = ok = checked = 0
    for frac in np.linspace(0.3, 1.5, 25):
        ctx = h2.Context(0, hbm_budget=int(frac * peak))
        try:
            try:
                dA = h2.load(ctx, A.to_flat())
            except h2.H2Error as e:
                assert e.code == 3, e
                continue
            for attempt in range(2):  # the second call runs after the first one's failure
                try:
                    C = h2.mmp(ctx, dA, dA, 1e-4, precision="fp32_bulk")
                except h2.H2Error as e:
                    assert e.code == 3, e
                    failed += 1
                    try:
                        y = h2.matvec(ctx, dA, x)
                    except h2.H2Error as e2:  # A and its float copy may fill the budget
                        assert e2.code == 3, e2
                        continue
                    checked += 1
                    assert np.array_equal(y, y_a), frac
                    continue
                ok += 1
                assert np.array_equal(h2.matvec(ctx, C, x), y_c), frac
                C.free()
        finally:
            ctx.close()
    print(f"budget sweep: {failed} products stopped ({checked} mat-vecs after them), "
          f"{ok} completed", flush=True)
    assert failed > 0 and ok > 0 and checked > 0


def test_every_allocation_failure_of_a_product_is_recoverable():
    """The library's failure injection (H2_FAIL_ALLOC: the allocation with
    that index raises H2_ERR_OOM once) stops an FP32-bulk product at each of
    its allocations in turn, those inside the helper stream's deferred
    products and after them included.  Every stopped call raises
    H2_ERR_OOM; the same context then computes A's mat-vec and the whole
    product again, both bit-identical to an untouched context's."""
    import os
    print("case allocation failure sweep plates4096 fp32_bulk", flush=True)
    A = cases.plates(4096)
    x = np.random.default_rng(4).standard_normal(A.n)
    ref_ctx = h2.Context(0)
    try:
        rA = h2.load(ref_ctx, A.to_flat())
        y_a = h2.matvec(ref_ctx, rA, x)
        y_c = h2.matvec(ref_ctx, h2.mmp(ref_ctx, rA, rA, 1e-4, precision="fp32_bulk"), x)
    finally:
        ref_ctx.close()
    stopped = 0
    idx = 0
    try:
        while True:
            os.environ["H2_FAIL_ALLOC"] = str(idx)
            ctx = h2.Context(0)
            try:
                try:
                    dA = h2.load(ctx, A.to_flat())
                except h2.H2Error as e:  # the index falls inside the load
                    assert e.code == 3, e
                    idx += 1
                    continue
                try:
                    h2.mmp(ctx, dA, dA, 1e-4, precision="fp32_bulk").free()
                    break  # the index lies past the product's allocations
                except h2.H2Error as e:
                    assert e.code == 3 and "H2_FAIL_ALLOC" in str(e), e
                stopped += 1
                assert np.array_equal(h2.matvec(ctx, dA, x), y_a), idx
                C = h2.mmp(ctx, dA, dA, 1e-4, precision="fp32_bulk")
                assert np.array_equal(h2.matvec(ctx, C, x), y_c), idx
                C.free()
            finally:
                ctx.close()
            idx += 1
            assert idx < 5000
    finally:
        os.environ.pop("H2_FAIL_ALLOC", None)
    print(f"allocation sweep: the product stopped at each of {stopped} allocations", flush=True)
    assert stopped > 20


def test_every_allocation_failure_of_a_recompression_is_recoverable():
    """The same sweep over h2_recompress: each stopped call raises
    H2_ERR_OOM and the context then recompresses A again, bit-identical to
    an untouched context's result."""
    import os
    print("case allocation failure sweep recompress plates4096", flush=True)
    A = cases.plates(4096)
    keys = ("krow", "kcol", "V", "W", "Er", "Ec", "S", "F")
    ref_ctx = h2.Context(0)
    try:
        rA = h2.load(ref_ctx, A.to_flat())
        ref = h2.export(h2.recompress(ref_ctx, rA, 1e-4))
    finally:
        ref_ctx.close()
    stopped = 0
    idx = 0
    try:
        while True:
            os.environ["H2_FAIL_ALLOC"] = str(idx)
            ctx = h2.Context(0)
            try:
                try:
                    dA = h2.load(ctx, A.to_flat())
                except h2.H2Error as e:
                    assert e.code == 3, e
                    idx += 1
                    continue
                try:
                    h2.recompress(ctx, dA, 1e-4).free()
                    break
                except h2.H2Error as e:
                    assert e.code == 3 and "H2_FAIL_ALLOC" in str(e), e
                stopped += 1
                got = h2.export(h2.recompress(ctx, dA, 1e-4))
                for k in keys:
                    assert np.array_equal(np.asarray(got[k]), np.asarray(ref[k])), (idx, k)
            finally:
                ctx.close()
            idx += 1
            assert idx < 5000
    finally:
        os.environ.pop("H2_FAIL_ALLOC", None)
    print(f"allocation sweep: the recompression stopped at each of {stopped} allocations", flush=True)
    assert stopped > 10


def test_every_allocation_failure_of_a_build_is_recoverable():
    """The same sweep over h2_build with recompression: each stopped call
    raises H2_ERR_OOM and the context then builds the matrix again,
    bit-identical to an untouched context's."""
    import os
    from h2inputs import configs
    print("case allocation failure sweep build+recompress plates4096", flush=True)
    w = configs.plates_n(4096)
    args = (w.pts, w.leaf_size, w.eta, w.order, w.kernel.self_value)
    keys = ("krow", "kcol", "V", "W", "Er", "Ec", "S", "F")
    ref_ctx = h2.Context(0)
    try:
        ref = h2.export(h2.build(ref_ctx, *args, recompress_eps=1e-5))
    finally:
        ref_ctx.close()
    stopped = 0
    idx = 0
    try:
        while True:
            os.environ["H2_FAIL_ALLOC"] = str(idx)
            ctx = h2.Context(0)
            try:
                try:
                    h2.build(ctx, *args, recompress_eps=1e-5).free()
                    break
                except h2.H2Error as e:
                    assert e.code == 3 and "H2_FAIL_ALLOC" in str(e), e
                stopped += 1
                got = h2.export(h2.build(ctx, *args, recompress_eps=1e-5))
                for k in keys:
                    assert np.array_equal(np.asarray(got[k]), np.asarray(ref[k])), (idx, k)
            finally:
                ctx.close()
            idx += 1
            assert idx < 5000
    finally:
        os.environ.pop("H2_FAIL_ALLOC", None)
    print(f"allocation sweep: the build stopped at each of {stopped} allocations", flush=True)
    assert stopped > 10
