"""CPU checker for the H^2 matrix-matrix product: plain FP64 / complex128
NumPy written from the paper (Ma and Jiao, arXiv 1908.05218).

Test infrastructure only.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg import this package; the product library never
does, and this package imports nothing from it.
"""
