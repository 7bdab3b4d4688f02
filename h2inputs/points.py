"""Seeded synthetic point clouds shaped like the paper's workloads.

The paper measures on capacitance-extraction and volume-integral-equation
matrices (Section VI) that are not available here; these generators give
point sets of the same families (a 3-D volume, two parallel plates, a
closed surface) from which kernel matrices of the same character are built.
Every generator takes an explicit seed and is deterministic.
"""
import math

import numpy as np


def cube(n, seed):
    """n points i.i.d. uniform in the unit cube."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(n, 3))


def plates_grid(nx, ny, gap, jitter, seed, cells=None):
    """Two parallel plates at z=0 and z=gap, an nx-by-ny cell-centre grid on
    each (x=(i+1/2)/cx, y=(j+1/2)/cy with (cx, cy) = cells, default (nx, ny):
    unit plates), every coordinate perturbed by U[-jitter, jitter].  Returns
    2*nx*ny points, lower plate first."""
    rng = np.random.default_rng(seed)
    cx, cy = cells if cells is not None else (nx, ny)
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    x = ((ix + 0.5) / cx).ravel()
    y = ((iy + 0.5) / cy).ravel()
    pts = []
    for z in (0.0, gap):
        pts.append(np.stack([x, y, np.full_like(x, z)], axis=1))
    p = np.concatenate(pts, axis=0)
    p += rng.uniform(-jitter, jitter, size=p.shape)
    return p


def plates_random(n, gap, jitter, seed):
    """Two parallel unit plates 'gap' apart, n//2 (and n - n//2) points
    uniform on each plate, every coordinate perturbed by U[-jitter, jitter]."""
    rng = np.random.default_rng(seed)
    n0 = n // 2
    n1 = n - n0
    a = np.concatenate([rng.uniform(0, 1, (n0, 2)), np.zeros((n0, 1))], axis=1)
    b = np.concatenate([rng.uniform(0, 1, (n1, 2)), np.full((n1, 1), gap)], axis=1)
    p = np.concatenate([a, b], axis=0)
    p += rng.uniform(-jitter, jitter, size=p.shape)
    return p


def fibonacci_sphere(n):
    """Quasi-uniform points on the unit sphere: z_i = 1-(2i+1)/n,
    azimuth i*pi*(3-sqrt(5))."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
