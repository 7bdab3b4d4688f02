"""Serving (h2_submit / h2_poll / h2_wait / h2_release): requests of mixed
size, family, eps and precision run through the context's worker; every
result meets the product's relative error criterion (equation `error`); the
HBM budget admits requests only next to the results still held."""
import math

import numpy as np
import pytest

import paper_1908_05218_amd as h2
from h2inputs import points
from h2inputs.build import panel_self_term

pytestmark = pytest.mark.gpu


def _request(i):
    rng = np.random.default_rng(100 + i)
    n = int(rng.choice([1024, 2048, 3000, 4096]))
    if i % 2 == 0:
        pts = points.cube(n, i)
        self_value = 1.0
    else:
        pts = points.plates_random(n, 0.1, 1e-3, i)
        half = n // 2
        a = (1.0 / half) ** 0.5
        self_value = panel_self_term(a, a)
    eps = 1e-4 if i % 3 else 1e-6
    prec = "fp32_bulk" if i % 4 < 2 else "fp64"
    return pts, self_value, eps, prec


def _check_result(ctx, res, n, eps, prec):
    assert res["status"] == 0
    A, C = res["A"], res["C"]
    x = np.random.default_rng(5).standard_normal(n)
    ref = h2.matvec(ctx, A, h2.matvec(ctx, A, x))
    e = np.linalg.norm(h2.matvec(ctx, C, x) - ref) / np.linalg.norm(ref)
    assert e <= 2 * eps + (2e-6 if prec == "fp32_bulk" else 0.0), e
    assert res["total_ms"] >= res["mmp_ms"] > 0 and res["queue_ms"] >= 0


def test_serving_mixed_requests():
    ctx = h2.Context(0)
    try:
        reqs = [_request(i) for i in range(8)]
        tickets = [h2.submit(ctx, p, 32, 1.0, 3, sv, eps, precision=prec)
                   for p, sv, eps, prec in reqs]
        print("submitted", tickets, flush=True)
        for t, (p, sv, eps, prec) in zip(tickets, reqs):
            res = h2.wait(ctx, t)
            assert h2.poll(ctx, t)
            _check_result(ctx, res, p.shape[0], eps, prec)
        for t in tickets:
            h2.release(ctx, t)
        with pytest.raises(h2.H2Error) as e:
            h2.poll(ctx, tickets[0])
        assert e.value.code == 1
    finally:
        ctx.close()


def test_serving_admission_by_budget():
    # estimate per request: 80 KB per point (rank 27) + 64 MiB
    est = 2048 * 80e3 + (64 << 20)
    budget = int(4.5 * est)
    ctx = h2.Context(0, hbm_budget=budget)
    try:
        with pytest.raises(h2.H2Error) as e:
            h2.submit(ctx, points.cube(65536, 0), 32, 1.0, 3, 1.0, 1e-4)
        assert e.value.code == 3
        tickets = [h2.submit(ctx, points.cube(2048, i), 32, 1.0, 3, 1.0, 1e-4) for i in range(5)]
        print("submitted", tickets, flush=True)
        for t in tickets[:4]:
            assert h2.wait(ctx, t)["status"] == 0
        # four results are held: the fifth waits for a release
        assert not h2.poll(ctx, tickets[4])
        with pytest.raises(h2.H2Error) as e:
            h2.release(ctx, tickets[4])
        assert e.value.code == 8
        h2.release(ctx, tickets[0])
        res = h2.wait(ctx, tickets[4])
        assert res["status"] == 0 and res["queue_ms"] > 0
        for t in tickets[1:]:
            h2.release(ctx, t)
    finally:
        ctx.close()


def test_serving_with_concurrent_calls():
    """Entry points of the context called while its worker runs are serialised
    with it (products on the caller's thread interleave with served ones)."""
    ctx = h2.Context(0)
    try:
        t = [h2.submit(ctx, points.cube(4096, i), 32, 1.0, 3, 1.0, 1e-4) for i in range(3)]
        own = h2.build(ctx, points.cube(2048, 9), 32, 1.0, 3, 1.0)
        C = h2.mmp(ctx, own, own, 1e-4)
        assert h2.stats(C)["mmp_ms"] > 0
        for x in t:
            assert h2.wait(ctx, x)["status"] == 0
    finally:
        ctx.close()
