"""Benchmark of the H^2 matrix-matrix product on one MI355X.

Workload: plates64k — N = 65,536 points on two parallel unit plates 0.1 apart
(128 x 256 cell-centre grid per plate, U[-1e-3, 1e-3] jitter, seed 1), leaf
size 32, eta = 1, 3x3x3 Chebyshev bases (rank 27), kernel 1/(4 pi r) with the
panel self-term; C = A A at eps = 1e-4 (ACCURACY truncation).  The headline is
the FP32-bulk product (FP32 MFMA block products, FP64 Gram sums and
eigen-decompositions); the plain FP64 product is timed beside it.

A step is one full product (every level: Grams, eigen-decompositions,
projections, collects, block products, split) on inputs already resident in
device memory.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 (matrix and vector)
FP32_PEAK_TFLOPS = 157.3  # MI355X dense FP32 MFMA


def cpu_baseline(patch=(64, 128)):
    """The CPU oracle (plain FP64 NumPy, as it stands) timed on a bounded
    sample of the headline workload: a patch of nx x ny cells of the plates64k
    grid on each plate (same spacing, gap, jitter, self-term, leaf size,
    Chebyshev order and eps; 2 nx ny unknowns), whole product C = A A.  The
    rate is unknowns per second of that product; the BLAS thread count is
    read from threadpoolctl."""
    import numpy as np
    from h2inputs import configs
    from oracle import mmp
    w = configs.plates64k_patch(*patch)
    A = w.build()
    t0 = time.perf_counter()
    Co, _ = mmp.h2_mmp(A, A, 1e-4)
    t = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0))
    blas = "unknown"
    try:
        import threadpoolctl
        info = [i for i in threadpoolctl.threadpool_info() if i.get("user_api") == "blas"]
        if info:
            cores = max(int(i.get("num_threads", 1)) for i in info)
            blas = f"{info[0].get('internal_api')} {info[0].get('version')}"
    except Exception:
        pass
    # the GPU products of the same matrix against the oracle's C (FP64):
    # ||(C_gpu - C_oracle) x|| / ||C_oracle x|| over seeded x
    import paper_1908_05218_amd as h2
    from oracle import h2ops
    ctx = h2.Context(0)
    dA = h2.load(ctx, A.to_flat())
    X = np.random.default_rng(17).standard_normal((A.n, 4))
    ref = h2ops.matvec(Co, X)
    vs = {}
    for prec in ("fp32_bulk", "fp64"):
        C = h2.mmp(ctx, dA, dA, 1e-4, precision=prec)
        vs[prec] = float(np.linalg.norm(h2.matvec(ctx, C, X) - ref) / np.linalg.norm(ref))
        C.free()
    ctx.close()
    return {"value": A.n / t, "unit": "unknowns/s", "cores": int(cores), "kind": "oracle",
            "blas": blas,
            "sample": f"plates64k patch: {patch[0]} x {patch[1]} cells of its 128 x 256 grid per "
                      f"plate (N = {A.n}, same spacing, jitter, self-term, leaf, order, eps 1e-4), "
                      f"whole oracle product C = A A in {t:.1f} s",
            "gpu_vs_oracle_rel": vs}


PEAK = {"fp64": FP64_PEAK_TFLOPS, "fp32_bulk": FP32_PEAK_TFLOPS}


def newton_schulz_leg(n=16384, eps=1e-2, steps=12):
    """Downstream workload: Newton-Schulz approximate inverse of the plates
    family matrix at N = n (grid recipe of plates64k at another size) by
    repeated products (h2_newton_schulz, FP32-bulk products at eps),
    alpha = 1 / (1.02 lambda_max) from 40 power iterations; the residual
    ||x - A X x|| / ||x|| over two seeded probes."""
    import numpy as np
    import paper_1908_05218_amd as h2
    from h2inputs import configs, vectors
    w = configs.plates_n(n)
    ctx = h2.Context(0)
    A = h2.build(ctx, w.pts, w.leaf_size, w.eta, w.order, w.kernel.self_value)
    x = np.random.default_rng(1).standard_normal(n)
    lam = 0.0
    for _ in range(40):
        y = h2.matvec(ctx, A, x)
        lam = float(np.linalg.norm(y) / np.linalg.norm(x))
        x = y / np.linalg.norm(y)
    alpha = 1.0 / (1.02 * lam)
    t0 = time.perf_counter()
    X = h2.newton_schulz(ctx, A, alpha, steps, eps, precision="fp32_bulk")
    secs = time.perf_counter() - t0
    xp = vectors.probes(n, 2, 7)
    r = xp - h2.matvec(ctx, A, h2.matvec(ctx, X, xp))
    out = {"workload": f"plates{n // 1024}k inverse", "N": n, "eps": eps, "steps": steps,
           "products": 2 * (steps - 1), "seconds": secs,
           "residual": float(np.linalg.norm(r) / np.linalg.norm(xp)),
           "rank_max": h2.stats(X)["rank_max_r"], "precision": "fp32_bulk"}
    ctx.close()
    return out


def serve_stream(n_req, precision, seed=3, slots=2, budget_gib=192, mean_gap_s=0.05,
                 n_max=32768):
    """Served latency: a seeded stream of C = A A requests through the
    library's request loop (h2_submit / h2_wait) with `slots` requests on the
    device at once, admitted against a device-memory budget of budget_gib.
    Recipe: N = round(exp(U[ln 4096, ln n_max])), the unit cube or the two-plate family with probability
    1/2 each (plates: random points on both plates, panel self-term), leaf 32,
    eta 1, Chebyshev 3x3x3, eps 1e-4 or 1e-6 with probability 1/2,
    exponential inter-arrival times of mean mean_gap_s (50 ms: 20 requests per
    second); the points are generated before the clock starts.  Latency =
    submission to completion (build of A on the device plus the product);
    service = build plus product of one request."""
    import math
    import numpy as np
    import paper_1908_05218_amd as h2
    from h2inputs import points
    from h2inputs.build import panel_self_term
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n_req):
        n = int(round(math.exp(rng.uniform(math.log(4096), math.log(n_max)))))
        cube = rng.random() < 0.5
        eps = 1e-4 if rng.random() < 0.5 else 1e-6
        gap = float(rng.exponential(1.0))
        if cube:
            pts, sv = points.cube(n, 1000 + i), 1.0
        else:
            pts = points.plates_random(n, 0.1, 1e-3, 1000 + i)
            a = (1.0 / (n // 2)) ** 0.5
            sv = panel_self_term(a, a)
        reqs.append((n, eps, gap, pts, sv))
    ctx = h2.Context(0, hbm_budget=int(budget_gib * 2**30))
    h2.serve_slots(ctx, slots)
    n0, eps0, _, p0, s0 = reqs[0]
    warm = h2.submit(ctx, p0, 32, 1.0, 3, s0, eps0, precision=precision)
    h2.wait(ctx, warm)
    h2.release(ctx, warm)
    tickets = []
    t0 = time.perf_counter()
    rejected = {}
    for n, eps, gap, pts, sv in reqs:
        time.sleep(gap * mean_gap_s)
        try:
            tickets.append((h2.submit(ctx, pts, 32, 1.0, 3, sv, eps, precision=precision), n))
        except h2.H2Error as e:  # its device-memory estimate exceeds the whole budget
            key = str(e).split(":")[0]
            rejected[key] = rejected.get(key, 0) + 1
    lat, svc, bad, reasons = [], [], 0, {}
    for i, (t, n) in enumerate(tickets):
        r = h2.wait(ctx, t)
        print(f"[bench] {precision} served {i + 1}/{len(tickets)}: N {n}, status {r['status']}, "
              f"{r['total_ms']:.0f} ms", file=sys.stderr, flush=True)
        if r["status"] != 0:
            bad += 1
            key = r["message"][:60]
            reasons[key] = reasons.get(key, 0) + 1
        else:
            lat.append(r["total_ms"])
            svc.append(r["build_ms"] + r["mmp_ms"])
        h2.release(ctx, t)
    wall = time.perf_counter() - t0
    ctx.close()
    lat = np.array(lat)
    return {"precision": precision, "requests": n_req, "failed": int(bad), "slots": slots,
            "n_max": n_max, "rejected_at_submit": rejected, "failures": reasons,
            "budget_gib": budget_gib, "arrivals_per_s": 1.0 / mean_gap_s,
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
            "service_p50_ms": float(np.percentile(svc, 50)) if svc else None,
            "service_p99_ms": float(np.percentile(svc, 99)) if svc else None,
            "mean_service_ms": float(np.mean(svc)) if svc else None,
            "unknowns_per_s": float(sum(n for (t, n) in tickets) / wall)}
def sphere_leg(n, steps, eps=1e-3):
    """Scattering-shaped complex128 product C = A B on a Fibonacci sphere:
    exp(-j kappa r)/(4 pi r) with kappa such that the point spacing
    sqrt(4 pi / N) is a tenth of a wavelength, B at kappa / 2, leaf 64, eta 1,
    Chebyshev 3x3x3 bases, self-term 1/(2 pi rho) - j kappa/(4 pi) with
    rho = 2/sqrt(N); both matrices built on the device (h2_build).  Timed
    products after one warm-up; eps_rel by the exact H^2 mat-vec."""
    import math
    import numpy as np
    import paper_1908_05218_amd as h2
    from h2inputs import points
    ctx = h2.Context(0)
    kappa = 2 * math.pi / (10 * math.sqrt(4 * math.pi / n))
    rho = 2.0 / math.sqrt(n)
    pts = points.fibonacci_sphere(n)
    A = h2.build(ctx, pts, 64, 1.0, 3, 1 / (2 * math.pi * rho) - 1j * kappa / (4 * math.pi),
                 kernel="helmholtz", wavenumber=kappa)
    B = h2.build(ctx, pts, 64, 1.0, 3, 1 / (2 * math.pi * rho) - 1j * kappa / (8 * math.pi),
                 kernel="helmholtz", wavenumber=kappa / 2, share_tree_with=A)
    h2.mmp(ctx, A, B, eps).free()
    walls = []
    for _ in range(steps):
        t0 = time.perf_counter()
        C = h2.mmp(ctx, A, B, eps)
        walls.append(time.perf_counter() - t0)
        st = h2.stats(C)
        if len(walls) < steps:
            C.free()
    x = np.random.default_rng(1).standard_normal(n) + 1j * np.random.default_rng(2).standard_normal(n)
    ref = h2.matvec(ctx, A, h2.matvec(ctx, B, x))
    erel = float(np.linalg.norm(h2.matvec(ctx, C, x) - ref) / np.linalg.norm(ref))
    ctx.close()
    ms = 1e3 * float(np.mean(walls))
    return {"workload": f"sphere{n // 1024}k", "N": n, "dtype": "complex128", "kappa": kappa,
            "leaf_size": 64, "basis": "chebyshev 3x3x3 (rank 27)", "eps": eps, "product": "A*B",
            "ms_per_step": ms, "unknowns_per_s": n / (ms * 1e-3),
            "gflops": st["flops"] / (ms * 1e-3) / 1e9, "eps_rel": erel,
            "rank_max": st["rank_max_r"], "peak_bytes": st["bytes_device"]}


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "plates64k_fp32bulk_hbm_by_class.md")


def measured_traffic(kind):
    """HBM bytes per launch of kernel class `kind` in FP32-bulk products of
    plates64k, from the committed FETCH_SIZE/WRITE_SIZE summary, or None when
    the kernel sources have changed since those counters were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    csrc = os.path.join(ROOT, "paper_1908_05218_amd", "csrc")
    blob = b"".join(open(os.path.join(csrc, f), "rb").read() for f in ("kernels.hip", "eig.hip"))
    h = hashlib.sha256(blob).hexdigest()[:16]
    val, rec = None, None
    for line in text.splitlines():
        if line.startswith(f"traffic_bytes_per_launch[{kind}]:"):
            val = float(line.split(":")[1])
        if line.startswith("kernel sources sha256 (first 16 hex):"):
            rec = line.split(":")[1].strip()
    return val if (val is not None and rec == h) else None


def run_precision(h2, ctx, dA, n, prec, steps, warmup, eps):
    """Warm-up, then `steps` timed products (per-launch HIP events on the
    library's stream give the per-kernel-class split); returns the timing,
    the relative error of the last product and the breakdown."""
    import numpy as np
    for i in range(warmup):
        C = h2.mmp(ctx, dA, dA, eps, precision=prec)
        print(f"[bench] {prec} warmup {i}: {h2.stats(C)['mmp_ms']:.1f} ms", file=sys.stderr, flush=True)
        C.free()
    ctx.set_profiling(True)
    walls, dev_ms = [], []
    prof = {"contraction_ms": 0.0, "contraction_launches": 0, "eig_ms": 0.0, "eig_launches": 0,
            "gram_ms": 0.0, "gram_launches": 0, "gram_flops": 0.0, "other_ms": 0.0,
            "other_launches": 0, "contraction_flops": 0.0, "target_ms": 0.0,
            "target_launches": 0, "eig_tri_ms": 0.0, "eig_val_ms": 0.0, "eig_vec_ms": 0.0}
    C = None
    for i in range(steps):
        if C is not None:
            C.free()
        t1 = time.perf_counter()
        C = h2.mmp(ctx, dA, dA, eps, precision=prec)
        walls.append(time.perf_counter() - t1)
        st = h2.stats(C)
        dev_ms.append(st["mmp_ms"])
        for k in prof:
            prof[k] += st[k]
        print(f"[bench] {prec} step {i}: wall {walls[-1] * 1e3:.1f} ms, device {dev_ms[-1]:.1f} ms",
              file=sys.stderr, flush=True)
    ctx.set_profiling(False)
    # relative error criterion (equation `error`) on the last product: the
    # largest ratio over three seeded probe vectors, each column on its own
    from h2inputs.vectors import probes
    X = probes(n, 3, 7)
    ref = h2.matvec(ctx, dA, h2.matvec(ctx, dA, X))
    got = h2.matvec(ctx, C, X)
    erel = float(max(np.linalg.norm(got[:, j] - ref[:, j]) / np.linalg.norm(ref[:, j])
                     for j in range(X.shape[1])))
    st = h2.stats(C)
    C.free()
    K = steps
    ms = 1e3 * float(np.mean(walls))
    # kernel classes: summed device time of their launches (HIP events on the
    # library's stream around each launch), and the algorithmic work each
    # class performs per product at the actual ranks (h2_stats): one
    # contraction per evaluated block product (k_bgemm_triple), the products
    # that apply the projections once per target (k_bgemm_target; its count
    # also holds the leaf targets' rank-form terms, which the leaf products
    # absorb), 2 d^2 per Gram column, 9 d^3 per eigen-decomposition
    classes = {
        "triple_contraction": (prof["contraction_ms"], prof["contraction_launches"],
                               st["flops_triple"], "mfma", PEAK[prec]),
        "target_products": (prof["target_ms"], prof["target_launches"], st["flops_target"],
                            "mfma", PEAK[prec]),
        "gram_products": (prof["gram_ms"], prof["gram_launches"], st["flops_gram"], "mfma",
                          FP64_PEAK_TFLOPS),
        # the eigensolver's three kernels (one launch each per level)
        "eig_tridiagonalisation": (prof["eig_tri_ms"], prof["eig_launches"] / 3,
                                   st["eig_tri_flops"], "alu", FP64_PEAK_TFLOPS),
        "eig_values": (prof["eig_val_ms"], prof["eig_launches"] / 3, None, "alu", None),
        "eig_vectors": (prof["eig_vec_ms"], prof["eig_launches"] / 3, st["eig_vec_flops"], "alu",
                        FP64_PEAK_TFLOPS),
        "other_products": (prof["other_ms"], prof["other_launches"], None, "hbm", None),
    }
    breakdown = {}
    for k, (cms, cl, alg, bound, peak) in classes.items():
        e = {"ms_per_step": cms / K, "launches_per_step": cl / K, "bound": bound}
        if k == "gram_products":
            # executed (padded) flops: the leaf case-1 sum goes through
            # sum_j F_ij (sum_k F_jk F_jk^T) F_ij^T, fewer flops than its definition
            e["executed_gflop_per_step"] = prof["gram_flops"] / K / 1e9
        if alg:
            e["algorithmic_gflop_per_step"] = alg / 1e9
            e["achieved_tflops"] = alg / (cms / K * 1e-3) / 1e12 if cms > 0 else None
            e["frac"] = e["achieved_tflops"] / peak if e["achieved_tflops"] else None
        breakdown[k] = e
    # the dominant kernel class by device time among those with an
    # algorithmic count (the projections / collects / split class and the
    # eigenvalue kernel have none)
    dom = max((k for k in classes if classes[k][2]), key=lambda k: classes[k][0])
    dms, dl, alg, bound, peak = classes[dom]
    achieved = alg / (dms / K * 1e-3) / 1e12 if dms > 0 else None
    traffic = measured_traffic(dom) if prec == "fp32_bulk" else None
    roof = {"bound": bound, "unit": "TFLOP/s", "peak": peak, "kernel": dom,
            "achieved": achieved, "frac": achieved / peak if achieved else None,
            "traffic": traffic, "traffic_unit": "bytes per launch",
            "algorithmic_gflop_per_launch": alg / 1e9 / max(dl / K, 1),
            "avg_launch_ms": dms / max(dl, 1), "launches_per_step": dl / K,
            "time_share": dms / (sum(v[0] for v in classes.values()) or 1)}
    return {"ms": ms, "device_ms": float(np.mean(dev_ms)), "eps_rel": erel, "stats": st,
            "breakdown": breakdown, "roofline": roof}


def fixed_basis_leg(h2, ctx, dA, n, eps):
    """The fixed-basis (formatted) product (Section I, Table IV): time and
    relative error beside the proposed product's at the same eps."""
    import numpy as np
    h2.mmp(ctx, dA, dA, eps, mode="fixed", precision="fp32_bulk").free()
    t1 = time.perf_counter()
    C = h2.mmp(ctx, dA, dA, eps, mode="fixed", precision="fp32_bulk")
    ms = 1e3 * (time.perf_counter() - t1)
    x = np.random.default_rng(7).standard_normal(n)
    ref = h2.matvec(ctx, dA, h2.matvec(ctx, dA, x))
    erel = float(np.linalg.norm(h2.matvec(ctx, C, x) - ref) / np.linalg.norm(ref))
    rmax = h2.stats(C)["rank_max_r"]
    C.free()
    return {"ms": ms, "eps_rel": erel, "rank_max": rmax, "precision": "fp32_bulk"}


def matvec_graph_leg(h2, ctx, dA, n, reps=100):
    """The exact mat-vec of the input with device vectors (the inner step of
    an iterative solver): `reps` eager calls of h2_matvec_noalloc against
    `reps` replays of one HIP graph that captured it (torch's graph capture
    on a torch stream), both timed with events on that stream; the graph's
    result is checked against the eager one."""
    import torch
    x = torch.randn(n, dtype=torch.float64, device="cuda", generator=None)
    y = torch.empty_like(x)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        h2.matvec_noalloc(ctx, dA, x, y, stream=s)
    torch.cuda.synchronize()
    ref = y.clone()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        h2.matvec_noalloc(ctx, dA, x, y, stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    eager_us = 1e3 * e0.elapsed_time(e1) / reps
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        h2.matvec_noalloc(ctx, dA, x, y, stream=s)
    torch.cuda.synchronize()
    y.zero_()
    e0.record(s)
    with torch.cuda.stream(s):
        for _ in range(reps):
            g.replay()
    e1.record(s)
    torch.cuda.synchronize()
    graph_us = 1e3 * e0.elapsed_time(e1) / reps
    same = bool(torch.equal(y, ref))
    print(f"[bench] mat-vec: eager {eager_us:.1f} us, graph replay {graph_us:.1f} us", file=sys.stderr,
          flush=True)
    return {"eager_us_per_call": eager_us, "graph_us_per_call": graph_us, "calls": reps,
            "graph_equals_eager": same}


def cube_recompressed_leg(n=65536, eps=1e-4, steps=2):
    """The 2^20-point cube workload's pipeline at a sixteenth of its size
    (the product's leaf-level temporaries, n_pad^2 doubles per leaf block,
    keep the full size beyond one GPU's memory): N uniform points in the unit
    cube (seed 0), leaf 64, eta 1, 1/(4 pi r) with unit diagonal, Chebyshev
    4x4x4 bases recompressed on the device at eps, then C = A A at eps in
    FP32-bulk; eps_rel by the exact H^2 mat-vec."""
    import numpy as np
    import paper_1908_05218_amd as h2
    from h2inputs import points
    ctx = h2.Context(0)
    pts = points.cube(n, 0)
    t0 = time.perf_counter()
    A = h2.build(ctx, pts, 64, 1.0, 4, 1.0, recompress_eps=eps)
    build_ms = 1e3 * (time.perf_counter() - t0)
    h2.mmp(ctx, A, A, eps, precision="fp32_bulk").free()
    walls = []
    C = None
    for _ in range(steps):
        if C is not None:
            C.free()
        t0 = time.perf_counter()
        C = h2.mmp(ctx, A, A, eps, precision="fp32_bulk")
        walls.append(time.perf_counter() - t0)
    st = h2.stats(C)
    x = np.random.default_rng(1).standard_normal(n)
    ref = h2.matvec(ctx, A, h2.matvec(ctx, A, x))
    erel = float(np.linalg.norm(h2.matvec(ctx, C, x) - ref) / np.linalg.norm(ref))
    out = {"workload": f"cube{n // 1024}k", "N": n, "leaf_size": 64,
           "basis": "chebyshev 4x4x4 recompressed on the device", "eps": eps,
           "build_and_recompress_ms": build_ms, "input_rank_max": h2.stats(A)["rank_max_r"],
           "ms_per_step": 1e3 * float(np.mean(walls)), "unknowns_per_s": n / float(np.mean(walls)),
           "eps_rel": erel, "rank_max": st["rank_max_r"], "peak_bytes": st["bytes_device"],
           "precision": "fp32_bulk"}
    ctx.close()
    print(f"[bench] cube {n}: {out['ms_per_step']:.0f} ms per product, eps_rel {erel:.2e}",
          file=sys.stderr, flush=True)
    return out


def recompress_leg(h2, ctx, dA, n, eps, steps=3):
    """The input recompressed at eps on the device (h2_recompress; the paper
    cites its input construction without describing it, Section VI): its
    time, the new rank profile (the input has rank 27 everywhere), and the
    FP32-bulk product of the recompressed inputs at eps with its time and its
    error against the exact product of the original inputs."""
    import numpy as np
    h2.recompress(ctx, dA, eps).free()
    t = time.perf_counter()
    R = h2.recompress(ctx, dA, eps)
    rec_ms = 1e3 * (time.perf_counter() - t)
    x = np.random.default_rng(7).standard_normal(n)
    erel_in = float(np.linalg.norm(h2.matvec(ctx, R, x) - h2.matvec(ctx, dA, x)) /
                    np.linalg.norm(h2.matvec(ctx, dA, x)))
    h2.mmp(ctx, R, R, eps, precision="fp32_bulk").free()
    t = time.perf_counter()
    for _ in range(steps):
        h2.mmp(ctx, R, R, eps, precision="fp32_bulk").free()
    ms = 1e3 * (time.perf_counter() - t) / steps
    C = h2.mmp(ctx, R, R, eps, precision="fp32_bulk")
    ref = h2.matvec(ctx, dA, h2.matvec(ctx, dA, x))
    erel = float(np.linalg.norm(h2.matvec(ctx, C, x) - ref) / np.linalg.norm(ref))
    out = {"recompress_ms": rec_ms, "eps": eps, "input_eps_rel": erel_in,
           "rank_max_input": 27, "rank_max_recompressed": h2.stats(R)["rank_max_r"],
           "rank_mean_recompressed": h2.stats(R)["rank_mean_r"],
           "product_ms": ms, "product_value": n / (ms * 1e-3), "product_eps_rel": erel,
           "product_rank_max": h2.stats(C)["rank_max_r"]}
    C.free()
    R.free()
    print(f"[bench] recompression {rec_ms:.1f} ms, product of recompressed inputs {ms:.1f} ms "
          f"(eps_rel {erel:.2e})", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--precision", choices=["fp32_bulk", "fp64"], default="fp32_bulk",
                    help="precision of the headline product (the other one is timed beside it)")
    ap.add_argument("--no-compare", action="store_true", help="skip the second precision")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-slots", type=int, default=2,
                    help="concurrent requests of the serving loop")
    ap.add_argument("--serve-requests", type=int, default=24,
                    help="requests of the served-latency stream (0: skip)")
    ap.add_argument("--serve-nmax", type=int, default=32768,
                    help="largest N of the served stream (131072: the full served workload, "
                         "FP32-bulk only, no below-capacity run)")
    ap.add_argument("--inverse-n", type=int, default=16384,
                    help="points of the Newton-Schulz inverse leg (0: skip)")
    ap.add_argument("--sphere-n", type=int, default=32768,
                    help="points of the complex Helmholtz sphere product (0: skip)")
    ap.add_argument("--cube-n", type=int, default=65536,
                    help="points of the recompressed-cube product leg (0: skip)")
    ap.add_argument("--no-legs", action="store_true",
                    help="only the headline products (no fixed-basis, recompression, sphere, "
                         "serving, inverse or CPU legs): the command the kernel traces profile")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run three plain 1 GiB device copies (scale of the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = 1 << 27  # doubles: 1 GiB
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_each": n * 8, "copy_bytes_written_each": n * 8,
                          "copies": 3}))
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import paper_1908_05218_amd as h2
    from h2inputs import configs

    t0 = time.perf_counter()
    A = configs.plates64k().build()
    t_build = time.perf_counter() - t0
    flat = A.to_flat()
    ctx = h2.Context(0)
    # end to end on a fresh context: upload (H2D), symbolic phase and the
    # numeric phase of the first product
    t1 = time.perf_counter()
    dA = h2.load(ctx, flat)
    load_ms = 1e3 * (time.perf_counter() - t1)
    t1 = time.perf_counter()
    C0 = h2.mmp(ctx, dA, dA, args.eps, precision=args.precision)
    first_ms = 1e3 * (time.perf_counter() - t1)
    symbolic_ms = h2.stats(C0)["symbolic_ms"]
    C0.free()
    print(f"[bench] inputs built in {t_build:.1f}s, loaded in {load_ms:.0f} ms, first product "
          f"{first_ms:.0f} ms (symbolic {symbolic_ms:.0f} ms)", file=sys.stderr, flush=True)
    head = run_precision(h2, ctx, dA, A.n, args.precision, args.steps, args.warmup, args.eps)
    other = None
    if not args.no_compare:
        op = "fp64" if args.precision == "fp32_bulk" else "fp32_bulk"
        other = run_precision(h2, ctx, dA, A.n, op, args.steps, args.warmup, args.eps)
    if args.no_legs:
        args.sphere_n = args.serve_requests = args.inverse_n = args.cube_n = 0
        args.no_cpu_baseline = True
    fixed = None if args.no_legs else fixed_basis_leg(h2, ctx, dA, A.n, args.eps)
    recomp = None if args.no_legs else recompress_leg(h2, ctx, dA, A.n, args.eps)
    mvg = None if args.no_legs else matvec_graph_leg(h2, ctx, dA, A.n)
    ctx.close()
    st = head["stats"]
    ms = head["ms"]
    out = {
        "metric": "H2-MMP unknowns/s (C = A A, eps = 1e-4)",
        "value": A.n / (ms * 1e-3),
        "unit": "unknowns/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32_bulk" else "f64",
        "data": "synthetic",
        "config": {"workload": "plates64k", "N": int(A.n), "leaf_size": 32, "eta": 1.0,
                   "basis": "chebyshev 3x3x3 (rank 27)", "eps": args.eps,
                   "truncation": "accuracy", "precision": args.precision,
                   "arithmetic": ("FP32 MFMA block products; FP64 Gram sums, eigen-decompositions "
                                  "and bases" if args.precision == "fp32_bulk" else "FP64 throughout"),
                   "product": "A*A"},
        "gflops": st["flops"] / (ms * 1e-3) / 1e9,
        "algorithmic_gflop_per_step": {"total": st["flops"] / 1e9,
                                       "triple": st["flops_triple"] / 1e9,
                                       "target": st["flops_target"] / 1e9,
                                       "gram": st["flops_gram"] / 1e9,
                                       "eig": st["eig_flops"] / 1e9},
        "device_ms_per_step": head["device_ms"],
        "symbolic_ms": symbolic_ms, "load_ms": load_ms,
        "end_to_end_ms": load_ms + first_ms,
        "eps_rel": head["eps_rel"],
        "rank_max": st["rank_max_r"], "lmin": st["lmin"], "n_triples": st["n_triples"],
        "sparsity_constant": st["sparsity_constant"],
        "breakdown": head["breakdown"],
        "roofline": head["roofline"],
    }
    if other is not None:
        key = "fp64_plain" if args.precision == "fp32_bulk" else "fp32_bulk"
        out[key] = {"ms_per_step": other["ms"], "value": A.n / (other["ms"] * 1e-3),
                    "device_ms_per_step": other["device_ms"], "eps_rel": other["eps_rel"],
                    "speedup_of_headline": other["ms"] / ms,
                    "breakdown": other["breakdown"], "roofline": other["roofline"]}
    if fixed is not None:
        out["fixed_basis"] = fixed
    if recomp is not None:
        out["recompressed_inputs"] = recomp
    if mvg is not None:
        out["matvec_graph"] = mvg
    if args.sphere_n > 0:
        out["sphere_complex"] = sphere_leg(args.sphere_n, args.steps)
    if args.cube_n > 0:
        out["cube_recompressed"] = cube_recompressed_leg(args.cube_n)
    if args.serve_requests > 0:
        precs = ("fp32_bulk", "fp64") if args.serve_nmax <= 32768 else ("fp32_bulk",)
        out["serving"] = {p: serve_stream(args.serve_requests, p, slots=args.serve_slots,
                                          n_max=args.serve_nmax) for p in precs}
        # the same stream at an arrival rate below the measured capacity
        # (slots / mean service time), where latency is service, not backlog
        fb = out["serving"]["fp32_bulk"]
        if args.serve_nmax <= 32768 and fb["mean_service_ms"]:
            cap = fb["slots"] / (fb["mean_service_ms"] * 1e-3)
            out["serving"]["fp32_bulk_below_capacity"] = serve_stream(
                args.serve_requests, "fp32_bulk", slots=args.serve_slots,
                mean_gap_s=1.0 / (0.7 * cap))
    if args.inverse_n > 0:
        out["newton_schulz"] = newton_schulz_leg(args.inverse_n)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
