"""Calibration of the ACCURACY-mode truncation factor theta.

ACCURACY mode keeps the eigenvalues of each normalised Gram sum above
(theta * eps / n_t)^2 * lambda_1, with n_t the number of truncated levels
(the reading of Section III-C's truncation that aims at
||C - AB|| <= eps ||AB||).  theta is fixed once, here, on small members of
each input family: the largest theta of a short grid whose worst measured
error ratio eps_rel / eps (equation `error` of Section VI, three seeded x)
stays at or below 1/2 on every case, the factor 2 leaving room for deeper
trees than the calibration cases have.  The chosen value is the oracle's
THETA and the library's; the printed table is quoted in the design notes.

Run: python -m oracle.calibrate_theta   (about five minutes on 8 cores).

Part of the CPU checker: test infrastructure only.
"""
import sys
import time

import numpy as np

from h2inputs import configs, points
from h2inputs.build import HelmholtzKernel, chebyshev_h2
from h2inputs.structure import BlockTree, ClusterTree

from . import h2ops, mmp

GRID = (1.0, 0.5, 0.25)
BOUND = 0.5


def _sphere(n, leaf=32, order=3):
    """Helmholtz pair on the Fibonacci sphere with the lattice spacing at a
    tenth of the wavelength (B at half the wavenumber)."""
    kappa = 2 * np.pi / (10 * np.sqrt(4 * np.pi / n))
    t = ClusterTree(points.fibonacci_sphere(n), leaf)
    b = BlockTree(t, 1.0)
    rho = 2.0 / np.sqrt(n)
    A = chebyshev_h2(t, b, HelmholtzKernel(kappa, 1 / (2 * np.pi * rho) - 1j * kappa / (4 * np.pi)),
                     order)
    B = chebyshev_h2(t, b, HelmholtzKernel(kappa / 2,
                                           1 / (2 * np.pi * rho) - 1j * kappa / (8 * np.pi)), order)
    return A, B


def cases():
    cube = configs.cube1k().build()
    plates = configs.plates_n(2048).build()
    A, B = _sphere(4096)
    return [("cube1k", cube, cube, (1e-2, 1e-3, 1e-4)),
            ("plates2048", plates, plates, (1e-2, 1e-3, 1e-4, 1e-6)),
            ("sphere4096", A, B, (1e-2, 1e-3, 1e-4))]


def eps_rel(C, A, B, seed=5):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((A.n, 3))
    if np.iscomplexobj(A.V[0]):
        x = x + 1j * rng.standard_normal((A.n, 3))
    ref = h2ops.matvec(A, h2ops.matvec(B, x))
    y = h2ops.matvec(C, x)
    return max(float(np.linalg.norm(y[:, c] - ref[:, c]) / np.linalg.norm(ref[:, c]))
               for c in range(3))


def main(out=sys.stdout):
    worst = {th: 0.0 for th in GRID}
    for name, A, B, epss in cases():
        for eps in epss:
            for th in GRID:
                t0 = time.perf_counter()
                C, info = mmp.h2_mmp(A, B, eps, theta=th)
                r = eps_rel(C, A, B) / eps
                worst[th] = max(worst[th], r)
                rmax = max(max(rr) for rr in info["ranks_row"] if len(rr))
                print(f"{name:11s} eps {eps:7.0e} theta {th:4.2f}: eps_rel/eps {r:6.3f}  "
                      f"max rank {rmax:3d}  ({time.perf_counter() - t0:5.1f} s)", file=out, flush=True)
    ok = [th for th in GRID if worst[th] <= BOUND]
    chosen = max(ok) if ok else min(GRID)
    for th in GRID:
        print(f"theta {th:4.2f}: worst eps_rel/eps {worst[th]:.3f}", file=out)
    print(f"chosen theta = {chosen}", file=out)
    return chosen


if __name__ == "__main__":
    main()
