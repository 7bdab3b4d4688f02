"""Writes the stored oracle results that the GPU parity tests at sizes too
large to run the oracle inside a test compare against.

Each archive `<name>.npz` holds, for C = A B from `oracle.mmp.h2_mmp`:
  ranks_row, ranks_col  kept rank of every cluster (all levels, heap order
                        2^l - 1 + c, zero above l_min);
  rows, y               C x at the sampled rows for seeded probe vectors x
                        (`h2inputs.vectors.probes(n, 3, 2024)`);
  eps, eps_rel          the prescribed eps and the oracle's own error
                        (equation `error` of Section VI);
  flops_triple, flops_target, flops_gram, flops_eig
                        the algorithmic work at the oracle's ranks
                        (`oracle.flops.flop_counts`);
  seconds, threads      the oracle's wall time and the BLAS thread count.
Only `oracle/` and the seeded input generators are called.

Run: python -m tests.golden.make_golden [name ...]   (plates64k: minutes)
"""
import os
import sys
import time

import numpy as np

from h2inputs import configs, vectors
from oracle import flops, h2ops, mmp
from tests import cases

HERE = os.path.dirname(os.path.abspath(__file__))


def _sphere_kappa(n):
    """Wavenumber that puts the Fibonacci lattice spacing at a tenth of the
    wavelength."""
    return 2 * np.pi / (10 * np.sqrt(4 * np.pi / n))


# name -> (pair builder, eps, row sampling step)
CASES = {
    "plates64k_eps1e-4": (lambda: (configs.plates64k().build(),) * 2, 1e-4, 8),
    "plates8192_eps1e-6": (lambda: (cases.plates(8192),) * 2, 1e-6, 1),
    "cube8192_eps1e-5": (lambda: (cases.cube(8192),) * 2, 1e-5, 1),
    "sphere4096_eps1e-3": (lambda: cases.helmholtz_sphere(4096, 32, 3, _sphere_kappa(4096)),
                           1e-3, 1),
}


def flat_ranks(info, key):
    out = []
    for lev, r in enumerate(info[key]):
        out.extend(r if lev >= info["lmin"] else [0] * len(r))
    return np.asarray(out, dtype=np.int32)


def make(name):
    build, eps, step = CASES[name]
    A, B = build()
    t0 = time.perf_counter()
    C, info = mmp.h2_mmp(A, B, eps)
    secs = time.perf_counter() - t0
    x = vectors.probes(A.n, 3, 2024, np.iscomplexobj(A.V[0]))
    y = h2ops.matvec(C, x)
    ref = h2ops.matvec(A, h2ops.matvec(B, x))
    e = max(float(np.linalg.norm(y[:, c] - ref[:, c]) / np.linalg.norm(ref[:, c]))
            for c in range(x.shape[1]))
    rows = np.arange(0, A.n, step, dtype=np.int64)
    fc = flops.flop_counts(A, B, info)
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, ranks_row=flat_ranks(info, "ranks_row"),
                        ranks_col=flat_ranks(info, "ranks_col"), rows=rows, y=y[rows],
                        eps=eps, eps_rel=e, seconds=secs, threads=len(os.sched_getaffinity(0)),
                        flops_triple=fc["triple"], flops_target=fc["target"],
                        flops_gram=fc["gram"], flops_eig=fc["eig"])
    rmax = [max(r) if len(r) else 0 for r in info["ranks_row"]]
    print(f"{name}: oracle {secs:.1f} s, eps_rel {e:.3e}, row ranks max per level {rmax}",
          flush=True)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(CASES)):
        make(nm)
