"""Seeded input generators shared by the product path's tests, the CPU
checker and the benchmark: point clouds, the cluster and block trees, and
construction of the input H^2 matrices.  Nothing here computes a
matrix-matrix product."""
from .structure import R, F, NL, ClusterTree, BlockTree  # noqa: F401
from .h2data import H2Matrix, cluster_index  # noqa: F401
