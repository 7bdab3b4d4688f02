"""ctypes binding of libh2mmp.so (include/h2mmp.h).  Argument marshalling
only: every step of the product runs in the library's HIP kernels.  The
library must be built (paper_1908_05218_amd/build.py); a missing library is
an error, there is no fallback."""
import ctypes as C
import os
import re
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libh2mmp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "h2mmp.h")

H2_OK = 0
H2_ERR_BUSY = 8
STATUS_NAMES = {0: "H2_OK", 1: "H2_ERR_ARG", 2: "H2_ERR_DEVICE", 3: "H2_ERR_OOM",
                4: "H2_ERR_STRUCTURE", 5: "H2_ERR_NUMERIC", 6: "H2_ERR_UNSUPPORTED",
                7: "H2_ERR_INTERNAL"}
TRUNC = {"accuracy": 0, "paper": 1, "exact": 2, "fixed": 3}
PREC = {"fp64": 0, "fp32_bulk": 1}
MAX_LEVELS = 40


class H2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class _HostMatrix(C.Structure):
    _fields_ = [("n", C.c_int64), ("L", C.c_int64), ("is_complex", C.c_int64)] + \
        [(k, C.c_void_p) for k in ("leaf_off", "perm", "node_off", "node_row", "node_col",
                                   "node_type", "krow", "kcol", "V", "W", "Er", "Ec", "S", "F",
                                   "V_off", "W_off", "Er_off", "Ec_off", "S_off", "F_off")]


class _ExportSizes(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("n", "L", "nnodes", "len_V", "len_W", "len_Er",
                                          "len_Ec", "len_S", "len_F", "is_complex")]


class _ExportBuffers(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("leaf_off", "perm", "node_off", "node_row", "node_col",
                                          "node_type", "krow", "kcol", "V", "W", "Er", "Ec", "S",
                                          "F", "V_off", "W_off", "Er_off", "Ec_off", "S_off",
                                          "F_off")]


class _Stats(C.Structure):
    _fields_ = [("L", C.c_int64), ("lmin", C.c_int64),
                ("rank_max_r", C.c_int64 * MAX_LEVELS), ("rank_max_c", C.c_int64 * MAX_LEVELS),
                ("rank_mean_r", C.c_double * MAX_LEVELS), ("rank_mean_c", C.c_double * MAX_LEVELS),
                ("flops", C.c_double), ("mmp_ms", C.c_double), ("symbolic_ms", C.c_double),
                ("n_triples", C.c_int64), ("sparsity_constant", C.c_int64),
                ("contraction_ms", C.c_double), ("contraction_launches", C.c_int64),
                ("contraction_flops", C.c_double), ("eig_ms", C.c_double),
                ("bytes_device", C.c_int64), ("gram_ms", C.c_double), ("other_ms", C.c_double),
                ("eig_launches", C.c_int64), ("gram_launches", C.c_int64),
                ("other_launches", C.c_int64), ("gram_flops", C.c_double),
                ("other_flops", C.c_double), ("eig_flops", C.c_double),
                ("flops_triple", C.c_double), ("flops_target", C.c_double),
                ("flops_gram", C.c_double), ("target_ms", C.c_double),
                ("target_launches", C.c_int64), ("eig_tri_ms", C.c_double),
                ("eig_val_ms", C.c_double), ("eig_vec_ms", C.c_double),
                ("eig_tri_flops", C.c_double), ("eig_vec_flops", C.c_double)]


class _Kernel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("self_value", C.c_double), ("wavenumber", C.c_double),
                ("self_value_imag", C.c_double)]


class _BuildOpts(C.Structure):
    _fields_ = [("leaf_size", C.c_int64), ("eta", C.c_double), ("cheb_order", C.c_int32),
                ("recompress_eps", C.c_double)]


KERNELS = {"laplace": 0, "helmholtz": 1}


class _Request(C.Structure):
    _fields_ = [("xyz", C.c_void_p), ("n", C.c_int64), ("kernel", _Kernel), ("opts", _BuildOpts),
                ("eps", C.c_double), ("trunc_mode", C.c_int32), ("precision", C.c_int32)]


class _Result(C.Structure):
    _fields_ = [("status", C.c_int), ("A", C.c_void_p), ("C", C.c_void_p),
                ("queue_ms", C.c_double), ("build_ms", C.c_double), ("mmp_ms", C.c_double),
                ("total_ms", C.c_double), ("message", C.c_char * 160), ("bytes", C.c_int64)]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_1908_05218_amd/build.py")
        # One HIP runtime per process: PyTorch ships its own libamdhip64.so.7,
        # and whichever copy is loaded first serves both (same soname).  Load
        # PyTorch's first, so that its streams and its caching allocator and
        # the library's launches share one runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.h2_ctx_create.argtypes = [C.c_int, C.c_size_t, C.POINTER(_Allocator), C.POINTER(vp)]
        L.h2_ctx_destroy.argtypes = [vp]
        L.h2_load.argtypes = [vp, C.POINTER(_HostMatrix), C.POINTER(vp)]
        L.h2_mmp.argtypes = [vp, vp, vp, C.c_double, C.c_int, C.c_int, vp, C.POINTER(vp)]
        L.h2_matvec.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_int, vp]
        L.h2_sync.argtypes = [vp]
        L.h2_scale_shift.argtypes = [vp, vp, C.c_double, C.c_double, C.POINTER(vp)]
        L.h2_recompress.argtypes = [vp, vp, C.c_double, C.POINTER(vp)]
        L.h2_newton_schulz.argtypes = [vp, vp, C.c_double, C.c_int, C.c_double, C.c_int, C.c_int,
                                       C.POINTER(vp)]
        L.h2_matvec_noalloc.argtypes = [vp, vp, vp, vp, C.c_int64, vp]
        L.h2_to_dense.argtypes = [vp, vp, vp, C.c_int64]
        L.h2_export_size.argtypes = [vp, C.POINTER(_ExportSizes)]
        L.h2_export.argtypes = [vp, C.POINTER(_ExportBuffers)]
        L.h2_stats.argtypes = [vp, C.POINTER(_Stats)]
        L.h2_set_profiling.argtypes = [vp, C.c_int]
        L.h2_free.argtypes = [vp]
        L.h2_plan_info.argtypes = [C.POINTER(_HostMatrix), C.c_int64, vp, vp, vp, vp]
        L.h2_build.argtypes = [vp, vp, C.c_int64, C.POINTER(_Kernel), C.POINTER(_BuildOpts), vp,
                               C.POINTER(vp)]
        L.h2_submit.argtypes = [vp, C.POINTER(_Request), C.POINTER(C.c_uint64)]
        L.h2_poll.argtypes = [vp, C.c_uint64]
        L.h2_wait.argtypes = [vp, C.c_uint64, C.POINTER(_Result)]
        L.h2_release.argtypes = [vp, C.c_uint64]
        L.h2_serve_slots.argtypes = [vp, C.c_int]
        L.h2_save.argtypes = [vp, C.c_char_p]
        L.h2_load_file.argtypes = [vp, C.c_char_p, C.POINTER(vp)]
        L.h2_last_error.restype = C.c_char_p
        L.h2_version.restype = C.c_int
        for f in ("h2_ctx_create", "h2_load", "h2_build", "h2_submit", "h2_poll", "h2_wait",
                  "h2_release", "h2_plan_info", "h2_mmp", "h2_matvec", "h2_to_dense",
                  "h2_export_size", "h2_export", "h2_stats", "h2_set_profiling", "h2_serve_slots",
                  "h2_save", "h2_load_file", "h2_sync", "h2_matvec_noalloc",
                  "h2_scale_shift", "h2_newton_schulz", "h2_recompress"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def declared_functions():
    """Function names declared in include/h2mmp.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(h2_[a-z_]+)\s*\(", text)))


def _check(code):
    if code != H2_OK:
        raise H2Error(code, lib().h2_last_error().decode())


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p)


class _Allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", C.c_void_p)]


def _torch_alloc(user, nbytes, device, stream):
    import torch
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), int(device), int(stream or 0))
    except RuntimeError:
        return None


def _torch_free(user, ptr, nbytes, device, stream):
    import torch
    torch.cuda.caching_allocator_delete(int(ptr))


# kept alive for the lifetime of the module (the library holds the pointers)
_TORCH_ALLOCATOR = _Allocator(_ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free), None)


def _stream_handle(stream):
    """hipStream_t of a torch stream, an integer handle, or None."""
    if stream is None:
        return None
    h = getattr(stream, "cuda_stream", stream)
    return C.c_void_p(int(h)) if int(h) else None


class Context:
    """A library context on one device.  allocator="torch": every device
    allocation of the context comes from PyTorch's caching allocator (on the
    context's stream), so the memory shows in torch.cuda.memory_allocated()."""

    def __init__(self, device=0, hbm_budget=0, allocator=None):
        h = C.c_void_p()
        if allocator not in (None, "torch"):
            raise ValueError("allocator must be None or 'torch'")
        hook = C.byref(_TORCH_ALLOCATOR) if allocator == "torch" else None
        _check(lib().h2_ctx_create(device, hbm_budget, hook, C.byref(h)))
        self.h = h
        self._mats = weakref.WeakSet()

    def close(self):
        """Frees every matrix of this context, then the context."""
        if self.h:
            for m in list(self._mats):
                m.free()
            lib().h2_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_profiling(self, on):
        _check(lib().h2_set_profiling(self.h, 1 if on else 0))


class Matrix:
    def __init__(self, ctx, h):
        self.ctx = ctx
        self.h = h
        ctx._mats.add(self)

    def free(self):
        if self.h and self.ctx.h:
            lib().h2_free(self.h)
        self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


_I64 = ("leaf_off", "perm", "node_off", "krow", "kcol", "V_off", "W_off", "Er_off", "Ec_off",
        "S_off", "F_off")
_I32 = ("node_row", "node_col", "node_type")
_F64 = ("V", "W", "Er", "Ec", "S", "F")


def _host_matrix(flat, keep):
    """Complex data (is_complex, or complex arrays) go as interleaved
    (real, imaginary) pairs."""
    hm = _HostMatrix()
    hm.n = int(flat["n"])
    hm.L = int(flat["L"])
    cplx = bool(int(flat.get("is_complex", 0))) or any(np.iscomplexobj(flat[k]) for k in _F64)
    hm.is_complex = 1 if cplx else 0
    for k in _I64:
        keep[k] = np.ascontiguousarray(flat[k], dtype=np.int64)
        setattr(hm, k, keep[k].ctypes.data)
    for k in _I32:
        keep[k] = np.ascontiguousarray(flat[k], dtype=np.int32)
        setattr(hm, k, keep[k].ctypes.data)
    for k in _F64:
        if cplx:
            keep[k] = np.ascontiguousarray(flat[k], dtype=np.complex128).view(np.float64)
        else:
            keep[k] = np.ascontiguousarray(flat[k], dtype=np.float64)
        setattr(hm, k, keep[k].ctypes.data if keep[k].size else None)
    return hm


def plan_info(flat):
    """Symbolic-phase counts per level (host only)."""
    keep = {}
    hm = _host_matrix(flat, keep)
    n = MAX_LEVELS
    t, b, m = (np.zeros(n, np.int64) for _ in range(3))
    lmin = C.c_int64()
    _check(lib().h2_plan_info(C.byref(hm), n, _ptr(t), _ptr(b), _ptr(m), C.byref(lmin)))
    L = int(flat["L"])
    return dict(triples=t[:L + 1].tolist(), blue=b[:L + 1].tolist(), merged=m[:L + 1].tolist(),
                lmin=lmin.value)


def load(ctx, flat):
    """Upload an H^2 matrix given in the flat interchange layout (a dict of
    arrays as described in include/h2mmp.h)."""
    keep = {}
    hm = _host_matrix(flat, keep)
    h = C.c_void_p()
    _check(lib().h2_load(ctx.h, C.byref(hm), C.byref(h)))
    return Matrix(ctx, h)


def save(M, path):
    """h2_save: write M to `path` as a NumPy .npz archive in the flat layout."""
    _check(lib().h2_save(M.h, os.fsencode(path)))


def load_file(ctx, path):
    """h2_load_file: upload the .npz archive at `path` (flat layout)."""
    h = C.c_void_p()
    _check(lib().h2_load_file(ctx.h, os.fsencode(path), C.byref(h)))
    return Matrix(ctx, h)


def build(ctx, points, leaf_size, eta, order, self_value, kernel="laplace", share_tree_with=None,
          wavenumber=0.0, recompress_eps=0.0):
    """h2_build: the H^2 matrix of the kernel over `points` (n x 3), built by
    the library (tree and bases on the host, couplings and dense blocks on
    the device).  kernel "helmholtz": exp(-j wavenumber r)/(4 pi r), complex
    self_value.  recompress_eps > 0: recompressed at that accuracy."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    if pts.ndim != 2 or pts.shape[1] != 3:
        raise ValueError("points must be n x 3")
    sv = complex(self_value)
    k = _Kernel(KERNELS[kernel], sv.real, float(wavenumber), sv.imag)
    o = _BuildOpts(int(leaf_size), float(eta), int(order), float(recompress_eps))
    h = C.c_void_p()
    _check(lib().h2_build(ctx.h, _ptr(pts), pts.shape[0], C.byref(k), C.byref(o),
                          share_tree_with.h if share_tree_with is not None else None, C.byref(h)))
    return Matrix(ctx, h)


class Borrowed:
    """A matrix owned by the library (a served result); valid until the
    request is released."""

    def __init__(self, ctx, h):
        self.ctx = ctx
        self.h = h

    def free(self):
        pass


def serve_slots(ctx, slots):
    """Concurrent requests of the context's serving loop (before the first
    submit)."""
    _check(lib().h2_serve_slots(ctx.h, int(slots)))


def submit(ctx, points, leaf_size, eta, order, self_value, eps, mode="accuracy",
           precision="fp64"):
    """Queue C = A A for the H^2 matrix of 1/(4 pi r) over `points`; returns
    the ticket."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    if pts.ndim != 2 or pts.shape[1] != 3:
        raise ValueError("points must be n x 3")
    r = _Request(pts.ctypes.data, pts.shape[0], _Kernel(0, float(self_value), 0.0, 0.0),
                 _BuildOpts(int(leaf_size), float(eta), int(order)), float(eps), TRUNC[mode],
                 PREC[precision])
    t = C.c_uint64()
    _check(lib().h2_submit(ctx.h, C.byref(r), C.byref(t)))
    return t.value


def poll(ctx, ticket):
    """True when the request has finished."""
    code = lib().h2_poll(ctx.h, ticket)
    if code == H2_ERR_BUSY:
        return False
    _check(code)
    return True


def wait(ctx, ticket):
    res = _Result()
    _check(lib().h2_wait(ctx.h, ticket, C.byref(res)))
    return dict(status=res.status, A=Borrowed(ctx, C.c_void_p(res.A)) if res.A else None,
                C=Borrowed(ctx, C.c_void_p(res.C)) if res.C else None, queue_ms=res.queue_ms,
                build_ms=res.build_ms, mmp_ms=res.mmp_ms, total_ms=res.total_ms,
                message=res.message.decode(errors="replace"), bytes=res.bytes)


def release(ctx, ticket):
    _check(lib().h2_release(ctx.h, ticket))


def mmp(ctx, A, B, eps, mode="accuracy", precision="fp64", stream=None):
    """C = A B.  stream: a torch stream or hipStream_t handle; the product is
    ordered on it and the call may return before its last kernels finish
    (sync(C) waits).  Without a stream the call returns when C is complete."""
    h = C.c_void_p()
    _check(lib().h2_mmp(ctx.h, A.h, B.h, float(eps), TRUNC[mode], PREC[precision],
                        _stream_handle(stream), C.byref(h)))
    return Matrix(ctx, h)


def scale_shift(ctx, M, a, b):
    """a M + b I (same partition and bases) as a new matrix."""
    h = C.c_void_p()
    _check(lib().h2_scale_shift(ctx.h, M.h, float(a), float(b), C.byref(h)))
    return Matrix(ctx, h)


def recompress(ctx, M, eps):
    """h2_recompress: M recompressed at accuracy eps as a new matrix."""
    h = C.c_void_p()
    _check(lib().h2_recompress(ctx.h, M.h, float(eps), C.byref(h)))
    return Matrix(ctx, h)


def newton_schulz(ctx, A, alpha, steps, eps, mode="accuracy", precision="fp64"):
    """Newton-Schulz approximate inverse X_steps of A (h2_newton_schulz)."""
    h = C.c_void_p()
    _check(lib().h2_newton_schulz(ctx.h, A.h, float(alpha), int(steps), float(eps), TRUNC[mode],
                                  PREC[precision], C.byref(h)))
    return Matrix(ctx, h)


def sync(M):
    """Wait for the launches of the call that produced M."""
    _check(lib().h2_sync(M.h))


def is_complex(M):
    sz = _ExportSizes()
    _check(lib().h2_export_size(M.h, C.byref(sz)))
    return bool(sz.is_complex)


def matvec(ctx, M, x, stream=None):
    """y = M x.  x: numpy array (host) or a torch tensor on the GPU
    (float64, n or n x nrhs, column-major for nrhs > 1 means x.T contiguous;
    the product is ordered on `stream`, a torch stream or handle, when given,
    else on the current torch stream).
    Complex matrices: numpy x (complex), passed planar (real parts, then
    imaginary parts)."""
    if is_complex(M):
        x = np.asarray(x, dtype=np.complex128)
        vec = x.ndim == 1
        X = x.reshape(x.shape[0], -1)
        nrhs = X.shape[1]
        P = np.concatenate([np.asfortranarray(X.real).ravel(order="F"),
                            np.asfortranarray(X.imag).ravel(order="F")])
        Q = np.empty_like(P)
        _check(lib().h2_matvec(ctx.h, M.h, P.ctypes.data_as(C.c_void_p),
                               Q.ctypes.data_as(C.c_void_p), nrhs, 0, None))
        m = X.shape[0] * nrhs
        Y = (Q[:m] + 1j * Q[m:]).reshape(X.shape, order="F")
        return Y[:, 0] if vec else Y
    try:
        import torch
        is_t = isinstance(x, torch.Tensor)
    except ImportError:
        is_t = False
    if is_t:
        vec = x.dim() == 1
        xx = x.reshape(x.shape[0], -1)
        nrhs = xx.shape[1]
        xc = xx.t().contiguous()  # column-major
        yc = torch.empty_like(xc)
        st = stream if stream is not None else torch.cuda.current_stream(xc.device)
        _check(lib().h2_matvec(ctx.h, M.h, C.c_void_p(xc.data_ptr()), C.c_void_p(yc.data_ptr()),
                               nrhs, 1, _stream_handle(st)))
        y = yc.t()
        return y[:, 0] if vec else y
    x = np.asarray(x, dtype=np.float64)
    vec = x.ndim == 1
    X = np.asfortranarray(x.reshape(x.shape[0], -1))
    Y = np.empty_like(X, order="F")
    _check(lib().h2_matvec(ctx.h, M.h, X.ctypes.data_as(C.c_void_p), Y.ctypes.data_as(C.c_void_p),
                           X.shape[1], 0, None))
    return Y[:, 0] if vec else Y


def matvec_noalloc(ctx, M, x, y, stream=None):
    """y = M x through h2_matvec_noalloc: x, y torch tensors on the GPU
    (float64, n x nrhs, column-major: x.t() contiguous), nothing allocated
    by the call; launched on `stream` (a torch stream or handle), else on the
    context's stream.  Complex M: x, y planar (real parts, then imaginary
    parts) in tensors of 2 n nrhs doubles."""
    nrhs = x.numel() // ((2 if is_complex(M) else 1) * _npoints(M))
    _check(lib().h2_matvec_noalloc(ctx.h, M.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                   nrhs, _stream_handle(stream)))


def _npoints(M):
    """Number of points of M."""
    sz = _ExportSizes()
    _check(lib().h2_export_size(M.h, C.byref(sz)))
    return int(sz.n)


def to_dense(ctx, M, n):
    out = np.empty((n, n), dtype=np.complex128 if is_complex(M) else np.float64, order="F")
    _check(lib().h2_to_dense(ctx.h, M.h, out.ctypes.data_as(C.c_void_p), n))
    return out


def export(M):
    """Copy M to host in the flat interchange layout."""
    sz = _ExportSizes()
    _check(lib().h2_export_size(M.h, C.byref(sz)))
    nleaf = 1 << sz.L
    ncl = (2 << sz.L) - 1
    fdt = np.complex128 if sz.is_complex else np.float64
    out = dict(
        leaf_off=np.zeros(nleaf + 1, np.int64), perm=np.zeros(sz.n, np.int64),
        node_off=np.zeros(sz.L + 2, np.int64), node_row=np.zeros(sz.nnodes, np.int32),
        node_col=np.zeros(sz.nnodes, np.int32), node_type=np.zeros(sz.nnodes, np.int32),
        krow=np.zeros(ncl, np.int64), kcol=np.zeros(ncl, np.int64),
        V=np.zeros(sz.len_V, fdt), W=np.zeros(sz.len_W, fdt), Er=np.zeros(sz.len_Er, fdt),
        Ec=np.zeros(sz.len_Ec, fdt), S=np.zeros(sz.len_S, fdt), F=np.zeros(sz.len_F, fdt),
        V_off=np.zeros(nleaf + 1, np.int64), W_off=np.zeros(nleaf + 1, np.int64),
        Er_off=np.zeros(ncl + 1, np.int64), Ec_off=np.zeros(ncl + 1, np.int64),
        S_off=np.zeros(sz.nnodes + 1, np.int64), F_off=np.zeros(sz.nnodes + 1, np.int64))
    eb = _ExportBuffers()
    for k, v in out.items():
        setattr(eb, k, v.ctypes.data if v.size else None)
    _check(lib().h2_export(M.h, C.byref(eb)))
    out["n"] = np.int64(sz.n)
    out["L"] = np.int64(sz.L)
    out["is_complex"] = np.int64(1 if sz.is_complex else 0)
    return out


def stats(M):
    s = _Stats()
    _check(lib().h2_stats(M.h, C.byref(s)))
    L = s.L
    return dict(L=L, lmin=s.lmin,
                rank_max_r=list(s.rank_max_r[:L + 1]), rank_max_c=list(s.rank_max_c[:L + 1]),
                rank_mean_r=list(s.rank_mean_r[:L + 1]), rank_mean_c=list(s.rank_mean_c[:L + 1]),
                flops=s.flops, mmp_ms=s.mmp_ms, symbolic_ms=s.symbolic_ms,
                n_triples=s.n_triples, sparsity_constant=s.sparsity_constant,
                contraction_ms=s.contraction_ms, contraction_launches=s.contraction_launches,
                contraction_flops=s.contraction_flops, eig_ms=s.eig_ms,
                bytes_device=s.bytes_device, gram_ms=s.gram_ms, other_ms=s.other_ms,
                eig_launches=s.eig_launches, gram_launches=s.gram_launches,
                other_launches=s.other_launches, gram_flops=s.gram_flops,
                other_flops=s.other_flops, eig_flops=s.eig_flops,
                flops_triple=s.flops_triple, flops_target=s.flops_target,
                flops_gram=s.flops_gram, target_ms=s.target_ms,
                target_launches=s.target_launches, eig_tri_ms=s.eig_tri_ms,
                eig_val_ms=s.eig_val_ms, eig_vec_ms=s.eig_vec_ms,
                eig_tri_flops=s.eig_tri_flops, eig_vec_flops=s.eig_vec_flops)
