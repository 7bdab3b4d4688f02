"""Seeded probe vectors for the relative-error criterion (equation `error`
of Section VI) and for comparing two products through their mat-vecs."""
import numpy as np


def probes(n, count, seed, complex_=False):
    """n x count standard normal vectors (complex normal when complex_)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, count))
    if complex_:
        x = x + 1j * rng.standard_normal((n, count))
    return x
