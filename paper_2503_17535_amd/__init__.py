"""MI355X-native hierarchical Poincare-Steklov (HPS) fast direct solver.

Thin Python binding over the C ABI of ``libhps.so`` (declared in
``include/hps.h``): argument marshalling only, every step of the build and the
solve runs in the library's HIP kernels.  PyTorch supplies device memory and
streams.  Importing this package does not need a GPU; building or solving
does, and fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhps.so")

HPS_OK, HPS_EINVAL, HPS_ENOMEM, HPS_ESINGULAR, HPS_EDEVICE, HPS_EUNSUPPORTED = range(6)
FLAG_ROOT_T, FLAG_NO_CHECK, FLAG_TIMING, FLAG_FP32_COPY, FLAG_FULL_PIVOT, FLAG_FP32_ONLY = 1, 2, 4, 8, 16, 32
FLAG_TEST_NO_REFINE = 1 << 30
FP64, FP32_REFINED = 0, 1

# every entry point include/hps.h declares
EXPORTS = ("hps_sizes", "hps_leaf_points", "hps_boundary_points", "hps_op_footprint",
           "hps_build", "hps_solve", "hps_solve_adjoint", "hps_stage_times",
           "hps_op_bytes", "hps_free", "hps_last_error", "hps_precompute_matrix",
           "hps_debug_download", "hps_debug_gemm", "hps_coeff_grad", "hps_interp_weights",
           "hps_batcher_create", "hps_solve_batch", "hps_batcher_free", "hps_refine_sweeps",
           "hps_debug_gemm_f32", "hps_level_info", "hps_solve_noalloc", "hps_mem_stats",
           "hps_build_subtrees", "hps_build_iti", "hps_set_allocator",
           "hps_build_solve", "hps_build_adaptive", "hps_adaptive_root_size", "hps_adaptive_points", "hps_adaptive_root_points",
           "hps_adaptive_check", "hps_adaptive_split", "hps_adaptive_union", "hps_adaptive_balance")


# allocator callback types of hps_set_allocator
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_allocator_refs = []  # the installed callbacks stay referenced while the library may call them


class HPSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"HPS error {code}: {msg}")
        self.code = code


class Tree(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("depth", ctypes.c_int),
                ("lo", ctypes.c_double), ("hi", ctypes.c_double)]


class ATree(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double), ("hi", ctypes.c_double),
                ("n_leaves", ctypes.c_longlong), ("leaves", ctypes.c_void_p)]


class Sizes(ctypes.Structure):
    _fields_ = [("n_leaves", ctypes.c_longlong), ("pts_per_leaf", ctypes.c_int),
                ("n_terms", ctypes.c_int), ("n_root_bdry", ctypes.c_longlong),
                ("n_interior", ctypes.c_int), ("n_leaf_bdry", ctypes.c_int),
                ("n_levels", ctypes.c_int), ("root_D", ctypes.c_longlong)]


class LevelInfo(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int), ("m", ctypes.c_int), ("nodes", ctypes.c_longlong),
                ("block_inverse", ctypes.c_int), ("ns_steps", ctypes.c_int),
                ("residual0", ctypes.c_double), ("residual", ctypes.c_double),
                ("worst_node", ctypes.c_longlong)]


class BatchItem(ctypes.Structure):
    _fields_ = [("op", ctypes.c_void_p), ("nrhs", ctypes.c_int),
                ("bdry", ctypes.c_void_p * 16), ("src", ctypes.c_void_p * 16),
                ("u", ctypes.c_void_p * 16)]


_lib = None


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2503_17535_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I, D, LL, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong, ctypes.c_size_t
        TP = ctypes.POINTER(Tree)
        L.hps_sizes.argtypes = [TP, I, ctypes.POINTER(Sizes)]
        L.hps_leaf_points.argtypes = [TP, I, P]
        L.hps_boundary_points.argtypes = [TP, I, P]
        L.hps_op_footprint.argtypes = [TP, I, I]
        L.hps_op_footprint.restype = S
        L.hps_build.argtypes = [TP, I, P, I, P, ctypes.POINTER(P)]
        L.hps_build_subtrees.argtypes = [TP, I, P, I, I, P, ctypes.POINTER(P)]
        L.hps_build_iti.argtypes = [TP, I, D, P, I, P, ctypes.POINTER(P)]
        L.hps_build_solve.argtypes = [TP, I, P, I, P, P, P, I, P, ctypes.POINTER(P)]
        L.hps_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, P]
        AP = ctypes.POINTER(ATree)
        L.hps_build_adaptive.argtypes = [AP, I, P, I, P, ctypes.POINTER(P)]
        L.hps_adaptive_root_size.argtypes = [P, ctypes.POINTER(LL)]
        L.hps_adaptive_root_size.restype = LL
        L.hps_adaptive_points.argtypes = [AP, I, I, P]
        L.hps_adaptive_root_points.argtypes = [AP, I]
        L.hps_adaptive_root_points.restype = LL
        L.hps_adaptive_check.argtypes = [I, LL, P, P, D, P, P]
        L.hps_adaptive_split.argtypes = [P, LL, P, P, LL]
        L.hps_adaptive_split.restype = LL
        L.hps_adaptive_union.argtypes = [P, LL, P, LL, P, LL]
        L.hps_adaptive_union.restype = LL
        L.hps_adaptive_balance.argtypes = [P, LL, P, LL]
        L.hps_adaptive_balance.restype = LL
        L.hps_solve.argtypes = [P, P, P, P, I, I, P]
        L.hps_solve_noalloc.argtypes = [P, P, P, P, I, P]
        L.hps_mem_stats.argtypes = [ctypes.POINTER(S), ctypes.POINTER(S), I]
        L.hps_mem_stats.restype = None
        L.hps_solve_adjoint.argtypes = [P, P, P, P, I, P]
        L.hps_stage_times.argtypes = [P, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(D), I]
        L.hps_op_bytes.argtypes = [P]
        L.hps_op_bytes.restype = S
        L.hps_free.argtypes = [P]
        L.hps_free.restype = None
        L.hps_last_error.restype = ctypes.c_char_p
        L.hps_debug_download.argtypes = [P, I, I, P, LL]
        L.hps_debug_download.restype = LL
        L.hps_debug_gemm.argtypes = [I, I, I, D, P, I, I, P, I, I, D, P, I, P]
        L.hps_coeff_grad.argtypes = [P, P, P, I, P, P]
        L.hps_interp_weights.argtypes = [TP, I, P, LL, P, P]
        L.hps_refine_sweeps.argtypes = [P, I]
        F = ctypes.c_float
        L.hps_debug_gemm_f32.argtypes = [I, I, I, F, P, I, I, P, I, I, F, P, I, P]
        L.hps_batcher_create.argtypes = [ctypes.POINTER(P)]
        L.hps_solve_batch.argtypes = [P, ctypes.POINTER(BatchItem), I, P]
        L.hps_batcher_free.argtypes = [P]
        L.hps_batcher_free.restype = None
        L.hps_precompute_matrix.argtypes = [I, I, I, P, LL, ctypes.POINTER(I), ctypes.POINTER(I)]
        L.hps_level_info.argtypes = [P, ctypes.POINTER(LevelInfo), I]
        for name in EXPORTS:
            if name not in ("hps_op_footprint", "hps_op_bytes", "hps_free", "hps_last_error", "hps_batcher_free",
                            "hps_mem_stats", "hps_adaptive_root_size", "hps_adaptive_root_points",
                            "hps_adaptive_split", "hps_adaptive_union", "hps_adaptive_balance",
                            "hps_debug_download", "hps_debug_gemm", "hps_coeff_grad", "hps_interp_weights",
           "hps_batcher_create", "hps_solve_batch", "hps_batcher_free", "hps_refine_sweeps",
           "hps_debug_gemm_f32"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def set_allocator(alloc=None, free=None):
    """hps_set_allocator: alloc(nbytes) -> device pointer (int) or None, and
    free(ptr, nbytes), called for every device block of the operators built
    afterwards; both None restores the library's own pool.  Earlier
    callbacks stay referenced (blocks go back through the allocator that
    supplied them)."""
    if (alloc is None) != (free is None):
        raise ValueError("alloc and free must both be given or both be None")
    if alloc is None:
        _check(lib().hps_set_allocator(_ALLOC_FN(), _FREE_FN(), None))
        return

    def _a(n, ctx):
        try:
            p = alloc(int(n))
        except Exception:  # an exception becomes an allocation failure (HPS_ENOMEM)
            return None
        return p or None

    def _f(p, n, ctx):
        free(int(p), int(n))
    ca, cf = _ALLOC_FN(_a), _FREE_FN(_f)
    _allocator_refs.append((ca, cf))
    _check(lib().hps_set_allocator(ca, cf, None))


def use_torch_allocator(enable: bool = True):
    """Route the library's device memory through PyTorch's caching allocator
    (torch.cuda.caching_allocator_alloc / caching_allocator_delete on the
    current device and stream), or back to the library's pool."""
    if not enable:
        set_allocator(None, None)
        return
    import torch
    set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n),
                  lambda p, n: torch.cuda.caching_allocator_delete(p))


def mem_stats(reset_peak: bool = False) -> tuple[int, int]:
    """(bytes in use, high-water mark) of the library's device memory."""
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    lib().hps_mem_stats(ctypes.byref(a), ctypes.byref(b), int(reset_peak))
    return a.value, b.value


def _check(rc):
    if rc != HPS_OK:
        raise HPSError(rc, lib().hps_last_error().decode())


def tree(dim: int, depth: int, lo: float = -1.0, hi: float = 1.0) -> Tree:
    return Tree(dim, depth, lo, hi)


def sizes(t: Tree, p: int) -> Sizes:
    s = Sizes()
    _check(lib().hps_sizes(ctypes.byref(t), p, ctypes.byref(s)))
    return s


def leaf_points(t: Tree, p: int) -> np.ndarray:
    s = sizes(t, p)
    out = np.empty((s.n_leaves, s.pts_per_leaf, t.dim))
    _check(lib().hps_leaf_points(ctypes.byref(t), p, out.ctypes.data))
    return out


def boundary_points(t: Tree, p: int) -> np.ndarray:
    s = sizes(t, p)
    out = np.empty((s.n_root_bdry, t.dim))
    _check(lib().hps_boundary_points(ctypes.byref(t), p, out.ctypes.data))
    return out


def footprint(t: Tree, p: int, flags: int = 0) -> int:
    return int(lib().hps_op_footprint(ctypes.byref(t), p, flags))


def precompute_matrix(dim: int, p: int, which: int) -> np.ndarray:
    cap = max(p ** dim * 6 * (p - 2) ** (dim - 1), p * p) * 2
    buf = np.empty(cap)
    r, c = ctypes.c_int(), ctypes.c_int()
    _check(lib().hps_precompute_matrix(dim, p, which, buf.ctypes.data, cap, ctypes.byref(r), ctypes.byref(c)))
    return buf[: r.value * c.value].reshape(r.value, c.value).copy()


def interp_weights(t: Tree, p: int, x) -> tuple[np.ndarray, np.ndarray]:
    """Containing leaf [m] and barycentric weights [m, p^dim] of the points
    x [m, dim] (see hps_interp_weights)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    m = x.shape[0]
    s = sizes(t, p)
    leaf = np.empty(m, dtype=np.int64)
    w = np.empty((m, s.pts_per_leaf))
    _check(lib().hps_interp_weights(ctypes.byref(t), p, x.ctypes.data, m, leaf.ctypes.data, w.ctypes.data))
    return leaf, w


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, name, shape=None, dtype=None):
    import torch
    dtype = dtype or torch.float64
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype:
        raise TypeError(f"{name} must be a CUDA {str(dtype).replace('torch.', '')} tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Operator:
    """A built HPS solution operator, resident in device memory."""

    def __init__(self, t: Tree, p: int, coeffs, flags: int = 0, stream=None, subtree_depth: int = 0):
        self.tree, self.p, self.flags = t, p, flags
        self.subtree_depth = subtree_depth
        self.sizes = sizes(t, p)
        s = self.sizes
        ptr = _dev_ptr(coeffs, "coeffs", (s.n_leaves, s.n_terms, s.pts_per_leaf))
        h = ctypes.c_void_p()
        if subtree_depth > 0:
            _check(lib().hps_build_subtrees(ctypes.byref(t), p, ptr, flags, subtree_depth, _stream_ptr(stream),
                                            ctypes.byref(h)))
        else:
            _check(lib().hps_build(ctypes.byref(t), p, ptr, flags, _stream_ptr(stream), ctypes.byref(h)))
        self._h = h

    def solve(self, bdry, src=None, out=None, stream=None, precision: int = FP64):
        import torch
        s = self.sizes
        nrhs = bdry.shape[0]
        bptr = _dev_ptr(bdry, "bdry", (nrhs, s.n_root_bdry))
        sptr = None if src is None else _dev_ptr(src, "src", (nrhs, s.n_leaves, s.pts_per_leaf))
        if out is None:
            out = torch.empty((nrhs, s.n_leaves, s.pts_per_leaf), dtype=torch.float64, device=bdry.device)
        uptr = _dev_ptr(out, "u", (nrhs, s.n_leaves, s.pts_per_leaf))
        _check(lib().hps_solve(self._h, bptr, sptr, uptr, nrhs, precision, _stream_ptr(stream)))
        return out

    def solve_noalloc(self, bdry, src, out, stream=None):
        """hps_solve_noalloc: the fp64 solve on the library's static device
        workspace; `out` must be given (the call allocates nothing)."""
        s = self.sizes
        nrhs = bdry.shape[0]
        bptr = _dev_ptr(bdry, "bdry", (nrhs, s.n_root_bdry))
        sptr = None if src is None else _dev_ptr(src, "src", (nrhs, s.n_leaves, s.pts_per_leaf))
        uptr = _dev_ptr(out, "u", (nrhs, s.n_leaves, s.pts_per_leaf))
        _check(lib().hps_solve_noalloc(self._h, bptr, sptr, uptr, nrhs, _stream_ptr(stream)))
        return out

    def solve_adjoint(self, w, lam_src=None, lam_bdry=None, stream=None):
        import torch
        s = self.sizes
        nrhs = w.shape[0]
        wptr = _dev_ptr(w, "w", (nrhs, s.n_leaves, s.pts_per_leaf))
        if lam_src is None:
            lam_src = torch.empty_like(w)
        lptr = _dev_ptr(lam_src, "lam_src", (nrhs, s.n_leaves, s.pts_per_leaf))
        bptr = None if lam_bdry is None else _dev_ptr(lam_bdry, "lam_bdry", (nrhs, s.n_root_bdry))
        _check(lib().hps_solve_adjoint(self._h, wptr, lptr, bptr, nrhs, _stream_ptr(stream)))
        return lam_src, lam_bdry

    def refine_sweeps(self, sweeps: int = 0) -> int:
        """Set the number of fp64 refinement sweeps of FP32_REFINED solves
        (0 only queries); returns the previous value."""
        rc = lib().hps_refine_sweeps(self._h, sweeps)
        if rc < 0:
            _check(-rc)
        return rc

    def coeff_grad(self, u, lam, out=None, stream=None):
        """dJ/dc [n_leaves, n_terms, p^dim] from u and lam_src (both
        [nrhs, n_leaves, p^dim]), summed over the right-hand sides."""
        import torch
        s = self.sizes
        nrhs = u.shape[0]
        uptr = _dev_ptr(u, "u", (nrhs, s.n_leaves, s.pts_per_leaf))
        lptr = _dev_ptr(lam, "lam", (nrhs, s.n_leaves, s.pts_per_leaf))
        if out is None:
            out = torch.empty((s.n_leaves, s.n_terms, s.pts_per_leaf), dtype=torch.float64, device=u.device)
        gptr = _dev_ptr(out, "grad", (s.n_leaves, s.n_terms, s.pts_per_leaf))
        _check(lib().hps_coeff_grad(self._h, uptr, lptr, nrhs, gptr, _stream_ptr(stream)))
        return out

    def level_info(self):
        """Per-level merge-inverse accuracy (see hps_level_info): a list of
        dicts, index = tree level (0 = root)."""
        cap = self.sizes.n_levels
        arr = (LevelInfo * max(1, cap))()
        n = lib().hps_level_info(self._h, arr, cap)
        if n < 0:
            _check(-n)
        return [{k: getattr(arr[i], k) for k, _ in LevelInfo._fields_} for i in range(n)]

    def stage_times(self):
        names = (ctypes.c_char_p * 64)()
        ms = (ctypes.c_double * 64)()
        n = lib().hps_stage_times(self._h, names, ms, 64)
        if n < 0:
            _check(-n)
        return [(names[i].decode(), ms[i]) for i in range(n)]

    def download(self, which: int, level: int = 0, cap: int = 1 << 28) -> np.ndarray:
        """Copy of an internal device buffer (see hps_debug_download)."""
        out = np.empty(cap)
        n = lib().hps_debug_download(self._h, which, level, out.ctypes.data, cap)
        if n < 0:
            _check(-n)
        return out[:n].copy()

    @property
    def nbytes(self) -> int:
        return int(lib().hps_op_bytes(self._h))

    def free(self):
        if getattr(self, "_h", None):
            lib().hps_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Batcher:
    """Batched solve over several resident operators (see hps_solve_batch)."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib().hps_batcher_create(ctypes.byref(h)))
        self._h = h

    def solve(self, items, stream=None):
        """items: sequence of (Operator, [bdry_j], [src_j or None], [u_j]) with
        per-rhs CUDA float64 vectors (bdry_j [n_root_bdry], src_j and u_j
        [n_leaves, p^2]).  The tensors must stay alive until the work queued
        on `stream` has completed."""
        arr = (BatchItem * len(items))()
        for k, (op, bd, sr, uu) in enumerate(items):
            s = op.sizes
            n = len(bd)
            if not (1 <= n <= 16) or len(uu) != n or (sr is not None and len(sr) != n):
                raise ValueError("each item needs 1..16 right-hand sides and matching lists")
            it = arr[k]
            it.op = op._h.value
            it.nrhs = n
            for j in range(n):
                it.bdry[j] = _dev_ptr(bd[j], "bdry", (s.n_root_bdry,)).value
                it.u[j] = _dev_ptr(uu[j], "u", (s.n_leaves, s.pts_per_leaf)).value
                if sr is not None and sr[j] is not None:
                    it.src[j] = _dev_ptr(sr[j], "src", (s.n_leaves, s.pts_per_leaf)).value
        _check(lib().hps_solve_batch(self._h, arr, len(items), _stream_ptr(stream)))

    def free(self):
        if getattr(self, "_h", None):
            lib().hps_batcher_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def debug_gemm(A, B, C, alpha=1.0, beta=0.0, trans_a=False, trans_b=False, stream=None):
    """C = alpha op(A) op(B) + beta C with the library's MFMA GEMM (test hook).
    Tensors are CUDA float64 (or all float32), column-major views (pass X.T.contiguous().T or
    Fortran-ordered data via .t())."""
    import torch
    m, n = C.shape
    k = A.shape[0] if trans_a else A.shape[1]
    for X, nm in ((A, "A"), (B, "B"), (C, "C")):
        if X.stride(0) != 1:
            raise ValueError(f"{nm} must be column-major (stride(0) == 1)")
    fn = lib().hps_debug_gemm_f32 if C.dtype == torch.float32 else lib().hps_debug_gemm
    _check(fn(m, n, k, alpha, ctypes.c_void_p(A.data_ptr()), A.stride(1), int(trans_a),
                                ctypes.c_void_p(B.data_ptr()), B.stride(1), int(trans_b), beta,
                                ctypes.c_void_p(C.data_ptr()), C.stride(1), _stream_ptr(stream)))
    return C


def build(t: Tree, p: int, coeffs, flags: int = 0, stream=None) -> Operator:
    return Operator(t, p, coeffs, flags, stream)


def build_solve(t: Tree, p: int, coeffs, bdry, src=None, out=None, flags: int = 0, stream=None):
    """hps_build_solve: build and first solve in one call (the sources' leaf
    part overlaps the top merge levels); returns (operator, u)."""
    import torch
    s = sizes(t, p)
    ptr = _dev_ptr(coeffs, "coeffs", (s.n_leaves, s.n_terms, s.pts_per_leaf))
    nrhs = bdry.shape[0]
    bptr = _dev_ptr(bdry, "bdry", (nrhs, s.n_root_bdry))
    sptr = None if src is None else _dev_ptr(src, "src", (nrhs, s.n_leaves, s.pts_per_leaf))
    if out is None:
        out = torch.empty((nrhs, s.n_leaves, s.pts_per_leaf), dtype=torch.float64, device=bdry.device)
    uptr = _dev_ptr(out, "u", (nrhs, s.n_leaves, s.pts_per_leaf))
    h = ctypes.c_void_p()
    _check(lib().hps_build_solve(ctypes.byref(t), p, ptr, flags, bptr, sptr, uptr, nrhs, _stream_ptr(stream),
                                 ctypes.byref(h)))
    op = Operator.__new__(Operator)
    op.tree, op.p, op.flags, op.subtree_depth, op.sizes = t, p, flags, 0, s
    op._h = h
    return op, out


class ItiOperator(Operator):
    """An operator of the ItI variant (hps_build_iti): complex128 boundary
    data (incoming impedance u_n + i eta u at the root Gauss points), sources
    and solutions."""

    def __init__(self, t: Tree, p: int, coeffs, eta: float, flags: int = 0, stream=None):
        self.tree, self.p, self.flags, self.eta = t, p, flags, eta
        self.subtree_depth = 0
        self.sizes = sizes(t, p)
        s = self.sizes
        ptr = _dev_ptr(coeffs, "coeffs", (s.n_leaves, s.n_terms, s.pts_per_leaf))
        h = ctypes.c_void_p()
        _check(lib().hps_build_iti(ctypes.byref(t), p, float(eta), ptr, flags, _stream_ptr(stream), ctypes.byref(h)))
        self._h = h

    def solve(self, bdry, src=None, out=None, stream=None, precision: int = FP64):
        import torch
        s, c = self.sizes, torch.complex128
        nrhs = bdry.shape[0]
        bptr = _dev_ptr(bdry, "bdry", (nrhs, s.n_root_bdry), c)
        sptr = None if src is None else _dev_ptr(src, "src", (nrhs, s.n_leaves, s.pts_per_leaf), c)
        if out is None:
            out = torch.empty((nrhs, s.n_leaves, s.pts_per_leaf), dtype=c, device=bdry.device)
        uptr = _dev_ptr(out, "u", (nrhs, s.n_leaves, s.pts_per_leaf), c)
        _check(lib().hps_solve(self._h, bptr, sptr, uptr, nrhs, precision, _stream_ptr(stream)))
        return out


def build_iti(t: Tree, p: int, coeffs, eta: float, flags: int = 0, stream=None) -> ItiOperator:
    """hps_build_iti: the impedance-to-impedance variant (2D)."""
    return ItiOperator(t, p, coeffs, eta, flags, stream)


def build_subtrees(t: Tree, p: int, coeffs, subtree_depth: int, flags: int = 0, stream=None) -> Operator:
    """hps_build_subtrees: only the top depth - subtree_depth merge levels stay
    resident; every solve rebuilds the subtrees below them."""
    if subtree_depth < 1:
        raise ValueError("subtree_depth must be >= 1")
    return Operator(t, p, coeffs, flags, stream, subtree_depth=subtree_depth)


# ---------------------------------------------------------------------------
# adaptive 3D discretization (Section 4.2)
# ---------------------------------------------------------------------------
def _edit(fn, *args):
    """Run a tree edit (hps_adaptive_split / union / balance) with a growing
    output buffer; returns the new leaves [n, 4] (int32)."""
    cap = 1024
    while True:
        out = np.empty((cap, 4), dtype=np.int32)
        n = fn(*args, out.ctypes.data, cap)
        if n < 0:
            _check(int(-n))
        if n <= cap:
            return out[:n].copy()
        cap = int(n)


class AdaptiveTree:
    """Leaves (level, ix, iy, iz) of an octree over [lo, hi]^3 in depth-first
    order (int32 [n, 4], host)."""

    def __init__(self, leaves, lo: float = 0.0, hi: float = 1.0):
        self.leaves = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 4))
        self.lo, self.hi = float(lo), float(hi)

    @property
    def n_leaves(self) -> int:
        return int(self.leaves.shape[0])

    def struct(self) -> ATree:
        return ATree(self.lo, self.hi, self.n_leaves, self.leaves.ctypes.data)

    @staticmethod
    def uniform(depth: int, lo: float = 0.0, hi: float = 1.0) -> "AdaptiveTree":
        t = AdaptiveTree(np.zeros((1, 4), dtype=np.int32), lo, hi)
        for _ in range(depth):
            t = t.split(np.ones(t.n_leaves, dtype=np.int32))
        return t

    def split(self, flags) -> "AdaptiveTree":
        flags = np.ascontiguousarray(np.asarray(flags, dtype=np.int32))
        L = lib()
        return AdaptiveTree(_edit(L.hps_adaptive_split, self.leaves.ctypes.data, self.n_leaves, flags.ctypes.data),
                            self.lo, self.hi)

    def union(self, other: "AdaptiveTree") -> "AdaptiveTree":
        L = lib()
        return AdaptiveTree(_edit(L.hps_adaptive_union, self.leaves.ctypes.data, self.n_leaves,
                                  other.leaves.ctypes.data, other.n_leaves), self.lo, self.hi)

    def balance(self) -> "AdaptiveTree":
        L = lib()
        return AdaptiveTree(_edit(L.hps_adaptive_balance, self.leaves.ctypes.data, self.n_leaves), self.lo, self.hi)

    def points(self, p: int, which: int = 0) -> np.ndarray:
        """0: leaf Chebyshev points [n, p^3, 3]; 1: the children's [n, 8, p^3, 3];
        2: root Gauss boundary points [n_root, 3]."""
        t = self.struct()
        if which == 0:
            out = np.empty((self.n_leaves, p ** 3, 3))
        elif which == 1:
            out = np.empty((self.n_leaves, 8, p ** 3, 3))
        else:
            n = lib().hps_adaptive_root_points(ctypes.byref(t), p)
            if n < 0:
                _check(int(-n))
            out = np.empty((int(n), 3))
        _check(lib().hps_adaptive_points(ctypes.byref(t), p, which, out.ctypes.data))
        return out


def adaptive_check(p: int, f0, f1, eps: float, stream=None) -> np.ndarray:
    """hps_adaptive_check: split flags (int32 [nl]) of eq. refinement_check
    from samples f0 [nl, p^3] and f1 [nl, 8, p^3] (CUDA float64)."""
    nl = f0.shape[0]
    out = np.empty(nl, dtype=np.int32)
    _check(lib().hps_adaptive_check(p, nl, _dev_ptr(f0, "f0", (nl, p ** 3)), _dev_ptr(f1, "f1", (nl, 8, p ** 3)),
                                    float(eps), out.ctypes.data, _stream_ptr(stream)))
    return out


def adaptive_tree(funcs, p: int, eps: float, max_level: int, lo: float = 0.0, hi: float = 1.0,
                  device="cuda:0") -> AdaptiveTree:
    """Section 4.2's tree: for each function (callable on points [N, 3] -> [N])
    split every leaf that fails the criterion until none does (or the level
    cap is reached), then the union of the trees and the level restriction.
    The criterion runs on the GPU (hps_adaptive_check)."""
    import torch
    trees = []
    for f in funcs:
        t = AdaptiveTree(np.zeros((1, 4), dtype=np.int32), lo, hi)
        while True:
            x0 = t.points(p, 0)
            x1 = t.points(p, 1)
            f0 = torch.tensor(np.asarray(f(x0.reshape(-1, 3)), dtype=np.float64).reshape(t.n_leaves, p ** 3),
                              device=device)
            f1 = torch.tensor(np.asarray(f(x1.reshape(-1, 3)), dtype=np.float64).reshape(t.n_leaves, 8, p ** 3),
                              device=device)
            flags = adaptive_check(p, f0, f1, eps)
            flags[t.leaves[:, 0] >= max_level] = 0
            if not flags.any():
                break
            t = t.split(flags)
        trees.append(t)
    out = trees[0]
    for t in trees[1:]:
        out = out.union(t)
    return out.balance()


class AdaptiveOperator:
    """An operator over an adaptive octree (hps_build_adaptive), resident in
    device memory."""

    def __init__(self, t: AdaptiveTree, p: int, coeffs, flags: int = 0, stream=None):
        self.tree, self.p, self.flags = t, p, flags
        self.n_leaves, self.pts_per_leaf = t.n_leaves, p ** 3
        ptr = _dev_ptr(coeffs, "coeffs", (t.n_leaves, 10, p ** 3))
        self._t = t.struct()
        h = ctypes.c_void_p()
        _check(lib().hps_build_adaptive(ctypes.byref(self._t), p, ptr, flags, _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        d = ctypes.c_longlong()
        n = lib().hps_adaptive_root_size(self._h, ctypes.byref(d))
        if n < 0:
            _check(int(-n))
        self.n_root_bdry, self.root_D = int(n), int(d.value)

    def solve(self, bdry, src=None, out=None, stream=None):
        import torch
        nrhs = bdry.shape[0]
        shp = (nrhs, self.n_leaves, self.pts_per_leaf)
        bptr = _dev_ptr(bdry, "bdry", (nrhs, self.n_root_bdry))
        sptr = None if src is None else _dev_ptr(src, "src", shp)
        if out is None:
            out = torch.empty(shp, dtype=torch.float64, device=bdry.device)
        uptr = _dev_ptr(out, "u", shp)
        _check(lib().hps_solve(self._h, bptr, sptr, uptr, nrhs, FP64, _stream_ptr(stream)))
        return out

    @property
    def nbytes(self) -> int:
        return int(lib().hps_op_bytes(self._h))

    def free(self):
        if getattr(self, "_h", None):
            lib().hps_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_adaptive(t: AdaptiveTree, p: int, coeffs, flags: int = 0, stream=None) -> AdaptiveOperator:
    """hps_build_adaptive: the adaptive 3D discretization (Section 4.2)."""
    return AdaptiveOperator(t, p, coeffs, flags, stream)

