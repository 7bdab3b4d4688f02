"""MI355X-native accuracy-controlled H^2 matrix-matrix product (Ma and Jiao,
arXiv 1908.05218): a C-ABI HIP library (libh2mmp.so, include/h2mmp.h) and
its ctypes binding."""
from .binding import (Borrowed, Context, Matrix, H2Error, build,  # noqa: F401
                      declared_functions, export, lib, load, load_file, matvec, matvec_noalloc, mmp,
                      newton_schulz, plan_info, poll, recompress, scale_shift,
                      release, save, serve_slots, stats, submit, sync, to_dense, wait)
