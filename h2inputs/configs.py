"""Named synthetic workloads (seeded) and small test families.

  cube1k     N=1,024 uniform in the unit cube (seed 0), leaf 32, eta 1,
             Chebyshev 2x2x2 (rank 8), 1/(4 pi r) with diagonal 1, eps 1e-6.
  plates64k  N=65,536 on two unit plates 0.1 apart, a 128x256 cell-centre
             grid per plate with U[-1e-3,1e-3] jitter (seed 1), leaf 32,
             eta 1, Chebyshev 3x3x3 (rank 27), 1/(4 pi r) with the panel
             self-term of a 1/128 x 1/256 panel, eps 1e-4.
Smaller members of the same families (cube_n, plates_n) use the same
recipes at other N for tests.
"""
import math
from dataclasses import dataclass

from . import points
from .build import LaplaceKernel, chebyshev_h2, panel_self_term
from .structure import BlockTree, ClusterTree


@dataclass
class Workload:
    name: str
    pts: object
    leaf_size: int
    eta: float
    order: int
    kernel: object
    eps: float

    def tree(self):
        return ClusterTree(self.pts, self.leaf_size)

    def build(self):
        t = self.tree()
        b = BlockTree(t, self.eta)
        return chebyshev_h2(t, b, self.kernel, self.order)


def cube1k():
    return Workload("cube1k", points.cube(1024, 0), 32, 1.0, 2,
                    LaplaceKernel(1.0), 1e-6)


def plates64k():
    return Workload("plates64k", points.plates_grid(128, 256, 0.1, 1e-3, 1), 32, 1.0, 3,
                    LaplaceKernel(panel_self_term(1 / 128, 1 / 256)), 1e-4)


def plates64k_patch(nx, ny):
    """A patch of the plates64k workload: nx x ny cells of its 128 x 256 grid
    per plate (same spacing, gap, jitter, self-term, leaf size, order, eps;
    2 nx ny points), a bounded sample of the same problem."""
    return Workload(f"plates64k_patch{nx}x{ny}",
                    points.plates_grid(nx, ny, 0.1, 1e-3, 1, cells=(128, 256)), 32, 1.0, 3,
                    LaplaceKernel(panel_self_term(1 / 128, 1 / 256)), 1e-4)


def cube_n(n, seed=0, leaf=32, order=3, eps=1e-4):
    return Workload(f"cube{n}", points.cube(n, seed), leaf, 1.0, order,
                    LaplaceKernel(1.0), eps)


def plates_n(n, seed=1, leaf=32, order=3, eps=1e-4):
    """Same family as plates64k at other sizes: a grid of nx x ny per plate
    with nx*ny = n/2 and ny = 2 nx when possible, else random plates."""
    half = n // 2
    nx = math.isqrt(max(1, half // 2))
    if nx * 2 * nx == half:
        pts = points.plates_grid(nx, 2 * nx, 0.1, 1e-3, seed)
        a, b = 1.0 / nx, 1.0 / (2 * nx)
    else:
        pts = points.plates_random(n, 0.1, 1e-3, seed)
        a = b = (1.0 / half) ** 0.5
    return Workload(f"plates{n}", pts, leaf, 1.0, order,
                    LaplaceKernel(panel_self_term(a, b)), eps)
