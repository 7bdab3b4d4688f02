"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function the header declares, its symbolic phase matches the CPU
checker's triple and accumulator counts, and invalid input is rejected."""
import ctypes

import numpy as np
import pytest

import paper_1908_05218_amd as h2
from oracle import mmp as omp
from tests import cases


def test_library_exports_declared_functions():
    lib = h2.lib()
    names = h2.declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert lib.h2_version() >= 1


def test_context_without_device_is_an_error():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(h2.H2Error) as e:
        h2.Context(0)
    assert e.value.code == 2


def _oracle_counts(A):
    sym = omp.Symbolic(A.blocks)
    L = A.L
    tri = [0] * (L + 1)
    blue = [set() for _ in range(L + 2)]
    merged = [0] * (L + 1)
    for lev in range(L, sym.lmin - 1, -1):
        t = sym.triples(lev)
        tri[lev] = len(t)
        for (i, j, k, *_r) in t:
            if sym.target(lev, i, k)[0] == omp.BLUE:
                blue[lev].add((i, k))
        if lev < L:
            parents = {(a >> 1, b >> 1) for (a, b) in blue[lev + 1]}
            merged[lev] = len(parents)
            for (i, k) in parents:
                if sym.target(lev, i, k)[0] == omp.BLUE:
                    blue[lev].add((i, k))
    if sym.lmin >= 1:
        merged[sym.lmin - 1] = len({(a >> 1, b >> 1) for (a, b) in blue[sym.lmin]})
    return tri, [len(b) for b in blue[:L + 1]], merged, sym.lmin


@pytest.mark.parametrize("which", ["cube1k", "plates2048", "ragged", "cube4096"])
def test_symbolic_phase_matches_checker(which):
    A = {"cube1k": cases.cube1k, "plates2048": lambda: cases.plates(2048),
         "ragged": lambda: cases.ragged_plates(777, 12),
         "cube4096": lambda: cases.cube(4096)}[which]()
    info = h2.plan_info(A.to_flat())
    tri, blue, merged, lmin = _oracle_counts(A)
    assert info["lmin"] == lmin
    assert info["triples"] == tri
    assert info["blue"] == blue
    assert info["merged"][lmin:] == merged[lmin:]


def test_invalid_structure_rejected():
    A = cases.plates(1024)
    flat = dict(A.to_flat())
    bad = flat["node_type"].copy()
    bad[0] = 1  # root marked dense above the leaf level
    flat["node_type"] = bad
    with pytest.raises(h2.H2Error) as e:
        h2.plan_info(flat)
    assert e.value.code == 1
    flat = dict(A.to_flat())
    perm = flat["perm"].copy()
    perm[0] = perm[1]
    flat["perm"] = perm
    with pytest.raises(h2.H2Error):
        h2.plan_info(flat)
