"""Python binding of the C ABI in include/dfacto.h (argument marshalling only).

Every computation runs in the HIP library ``libdfacto.so``; this module only
checks tensor shapes/dtypes and passes device pointers and the current HIP
stream through ctypes.  There is no fallback: if the library is missing or
fails to load, every call raises.

Names follow the C entry points without the ``dfacto_`` prefix.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdfacto.so")

OK, E_INVALID, E_RANGE, E_NOMEM, E_DEVICE, E_NUMERIC, E_UNSUPPORTED, E_AGAIN = range(8)
F32, BF16 = 0, 1
STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_RANGE", 3: "E_NOMEM", 4: "E_DEVICE",
                5: "E_NUMERIC", 6: "E_UNSUPPORTED", 7: "E_AGAIN"}

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = (
    "dfacto_ctx_create", "dfacto_ctx_set_stream", "dfacto_ctx_synchronize", "dfacto_ctx_destroy",
    "dfacto_ctx_freeze",
    "dfacto_last_error", "dfacto_build_flattenings", "dfacto_build_flattenings_ex",
    "dfacto_tensor_get_info",
    "dfacto_tensor_export", "dfacto_tensor_destroy", "dfacto_mttkrp", "dfacto_als_iter",
    "dfacto_gd_grad", "dfacto_gd_step", "dfacto_build_ratings", "dfacto_joint_grad",
    "dfacto_joint_als_iter", "dfacto_group_create", "dfacto_group_als", "dfacto_group_get_info",
    "dfacto_group_destroy", "dfacto_group_set_form", "dfacto_server_create", "dfacto_server_submit", "dfacto_server_poll",
    "dfacto_server_wait", "dfacto_server_get_stats", "dfacto_server_destroy",
    "dfacto_profile_enable", "dfacto_profile_read", "dfacto_gather_probe",
    "dfacto_mttkrp_noalloc", "dfacto_tensor_gather_order",
)
GROUP_GRAPH, GROUP_TUNE, GROUP_CTX_STREAM, GROUP_OWN_FACTORS = 1, 2, 4, 8


class DfactoError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Info(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int64 * 3), ("nnz", ctypes.c_int64),
                ("nfib", ctypes.c_int64 * 3), ("nroot", ctypes.c_int64 * 3),
                ("nentry", ctypes.c_int64 * 3), ("nchunk", ctypes.c_int64 * 3),
                ("normsq", ctypes.c_double), ("bytes", ctypes.c_size_t),
                ("relabeled", ctypes.c_int), ("chunk_len", ctypes.c_int)]


class _LineSearch(ctypes.Structure):
    _fields_ = [("alpha0", ctypes.c_double), ("shrink", ctypes.c_double), ("c", ctypes.c_double),
                ("max_trials", ctypes.c_int)]


class _GdStepInfo(ctypes.Structure):
    _fields_ = [("f0", ctypes.c_double), ("f", ctypes.c_double), ("gnorm2", ctypes.c_double),
                ("alpha", ctypes.c_double), ("trials", ctypes.c_int), ("accepted", ctypes.c_int)]


class _GroupInfo(ctypes.Structure):
    _fields_ = [("members", ctypes.c_int), ("launches_per_iter", ctypes.c_int),
                ("bytes", ctypes.c_size_t), ("graph", ctypes.c_int),
                ("mttkrp_classes", ctypes.c_int), ("mttkrp_grid", ctypes.c_int * 16),
                ("mttkrp_cpl", ctypes.c_int * 16), ("mttkrp_lanes", ctypes.c_int * 16),
                ("mttkrp_chunks_per_group", ctypes.c_int * 16), ("mttkrp_forms", ctypes.c_int * 16)]


class _Request(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int64 * 3), ("nnz", ctypes.c_int64),
                ("i", ctypes.c_void_p), ("j", ctypes.c_void_p), ("k", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("R", ctypes.c_int), ("dtype", ctypes.c_int),
                ("reg", ctypes.c_double), ("init", ctypes.c_void_p * 3), ("tol", ctypes.c_double),
                ("max_iters", ctypes.c_int), ("out_F", ctypes.c_void_p * 3),
                ("out_lambda", ctypes.c_void_p)]


class _RequestStatus(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int), ("status", ctypes.c_int), ("fit", ctypes.c_double),
                ("iters", ctypes.c_int), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("pending", ctypes.c_int64), ("running", ctypes.c_int64),
                ("finished", ctypes.c_int64), ("peak_active", ctypes.c_int),
                ("iterations", ctypes.c_int64), ("budget", ctypes.c_size_t),
                ("t_admit", ctypes.c_double), ("t_build", ctypes.c_double),
                ("t_groups", ctypes.c_double),
                ("t_iterate", ctypes.c_double), ("t_deliver", ctypes.c_double)]


_lib = None


def load():
    """Load libdfacto.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    PP = ctypes.POINTER(ctypes.c_void_p)
    lib.dfacto_ctx_create.argtypes = [I, P, P, PP]
    lib.dfacto_ctx_set_stream.argtypes = [P, P]
    lib.dfacto_ctx_synchronize.argtypes = [P]
    lib.dfacto_ctx_freeze.argtypes = [P, I]
    lib.dfacto_ctx_destroy.argtypes = [P]
    lib.dfacto_ctx_destroy.restype = None
    lib.dfacto_last_error.argtypes = [P]
    lib.dfacto_last_error.restype = ctypes.c_char_p
    lib.dfacto_build_flattenings.argtypes = [P, ctypes.POINTER(ctypes.c_int64), I64, P, P, P, P, PP]
    lib.dfacto_build_flattenings_ex.argtypes = [P, ctypes.POINTER(ctypes.c_int64), I64, P, P, P, P,
                                                I, I, PP]
    lib.dfacto_tensor_get_info.argtypes = [P, ctypes.POINTER(_Info)]
    lib.dfacto_tensor_export.argtypes = [P, P, I, P, P, P, P, P, P]
    lib.dfacto_tensor_gather_order.argtypes = [P, P, I, I, P]
    lib.dfacto_tensor_destroy.argtypes = [P]
    lib.dfacto_tensor_destroy.restype = None
    lib.dfacto_mttkrp.argtypes = [P, P, I, I, I, PP, P]
    lib.dfacto_mttkrp_noalloc.argtypes = [P, P, I, I, I, PP, P]
    lib.dfacto_als_iter.argtypes = [P, P, I, I, D, PP, P, P]
    lib.dfacto_gd_grad.argtypes = [P, P, I, I, D, PP, PP, P]
    lib.dfacto_gd_step.argtypes = [P, P, I, I, D, PP, PP, ctypes.POINTER(_LineSearch),
                                   ctypes.POINTER(_GdStepInfo)]
    lib.dfacto_build_ratings.argtypes = [P, ctypes.POINTER(ctypes.c_int64), I64, P, P, P, PP]
    lib.dfacto_joint_grad.argtypes = [P, P, P, I, I, D, D, PP, PP, P]
    lib.dfacto_joint_als_iter.argtypes = [P, P, P, I, I, D, D, PP]
    lib.dfacto_group_create.argtypes = [P, I, PP, ctypes.POINTER(ctypes.c_int), I, D, PP, PP, P,
                                        I, PP]
    lib.dfacto_group_als.argtypes = [P, P, I]
    lib.dfacto_group_get_info.argtypes = [P, ctypes.POINTER(_GroupInfo)]
    lib.dfacto_group_set_form.argtypes = [P, I, I, I]
    lib.dfacto_group_destroy.argtypes = [P]
    lib.dfacto_group_destroy.restype = None
    lib.dfacto_server_create.argtypes = [I, ctypes.c_size_t, I, PP]
    lib.dfacto_server_submit.argtypes = [P, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_int64)]
    lib.dfacto_server_poll.argtypes = [P, I64, ctypes.POINTER(_RequestStatus)]
    lib.dfacto_server_wait.argtypes = [P, I64, ctypes.POINTER(_RequestStatus)]
    lib.dfacto_server_get_stats.argtypes = [P, ctypes.POINTER(_ServerStats)]
    lib.dfacto_server_destroy.argtypes = [P]
    lib.dfacto_server_destroy.restype = None
    lib.dfacto_profile_enable.argtypes = [P, I]
    lib.dfacto_profile_read.argtypes = [P, P, P, P, P]
    lib.dfacto_gather_probe.argtypes = [P, P, I, I, I, PP, I, P]
    for name in EXPORTS:
        if name not in ("dfacto_ctx_destroy", "dfacto_last_error", "dfacto_tensor_destroy",
                        "dfacto_group_destroy", "dfacto_server_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _ptrs(ts) -> ctypes.Array:
    return (ctypes.c_void_p * 3)(*[(x.data_ptr() if x is not None else None) for x in ts])


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.bfloat16:
        return BF16
    raise TypeError(f"factor dtype must be float32 or bfloat16, got {t.dtype}")


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", ctypes.c_void_p)]


class TorchAllocator:
    """A dfacto_allocator served by torch's caching allocator: the library's
    device memory is torch memory (counted by torch.cuda.memory_allocated and
    reused by torch once freed, in the order of the stream it was allocated
    on).  An allocation torch cannot serve becomes DFACTO_E_NOMEM."""

    def __init__(self, device: int = 0):
        self.device = int(device)

        def _alloc(nbytes, stream, user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), self.device, stream or 0)
            except Exception:
                return None

        def _free(ptr, stream, user):
            try:
                torch.cuda.caching_allocator_delete(ptr)
            except Exception:  # torch already torn down at interpreter exit
                pass

        self._fns = (_ALLOC_FN(_alloc), _FREE_FN(_free))
        self.struct = _Allocator(self._fns[0], self._fns[1], None)


class Context:
    """A dfacto_ctx bound to a device and a HIP stream (torch's current one
    unless given).  allocator: None (the library allocates), "torch" (a
    TorchAllocator) or an object with a ctypes `struct` field laid out as
    dfacto_allocator; it is kept alive by the context and by every tensor
    built with it."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None,
                 allocator=None):
        lib = load()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        if allocator == "torch":
            allocator = TorchAllocator(device)
        self.allocator = allocator
        h = ctypes.c_void_p()
        st = lib.dfacto_ctx_create(int(device), ctypes.c_void_p(stream.cuda_stream),
                                   ctypes.byref(allocator.struct) if allocator else None,
                                   ctypes.byref(h))
        if st != OK:
            raise DfactoError(st, "dfacto_ctx_create failed")
        self.handle = h
        self.device = device

    def check(self, st: int):
        if st != OK:
            raise DfactoError(st, load().dfacto_last_error(self.handle).decode())

    def set_stream(self, stream: torch.cuda.Stream):
        self._stream = stream
        self.check(load().dfacto_ctx_set_stream(self.handle, ctypes.c_void_p(stream.cuda_stream)))

    def synchronize(self):
        self.check(load().dfacto_ctx_synchronize(self.handle))

    def freeze(self, on: bool = True):
        """While frozen, a call that would grow a workspace fails (E_INVALID)."""
        self.check(load().dfacto_ctx_freeze(self.handle, 1 if on else 0))

    def last_error(self) -> str:
        return load().dfacto_last_error(self.handle).decode()

    def close(self):
        if getattr(self, "handle", None):
            load().dfacto_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tensor:
    """A built dfacto_tensor (the three flattenings, resident on the device)."""

    def __init__(self, handle, allocator=None):
        self.handle = handle
        self._allocator = allocator  # frees the flattenings in close()

    def info(self) -> dict:
        inf = _Info()
        st = load().dfacto_tensor_get_info(self.handle, ctypes.byref(inf))
        if st != OK:
            raise DfactoError(st, "dfacto_tensor_get_info failed")
        return dict(dims=tuple(inf.dims), nnz=inf.nnz, nfib=tuple(inf.nfib),
                    nroot=tuple(inf.nroot), nentry=tuple(inf.nentry), nchunk=tuple(inf.nchunk),
                    normsq=inf.normsq, bytes=inf.bytes, relabeled=bool(inf.relabeled),
                    chunk_len=inf.chunk_len)

    def close(self):
        if getattr(self, "handle", None):
            load().dfacto_tensor_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ctx_create(device: int = 0, stream=None, allocator=None) -> Context:
    return Context(device, stream, allocator)


BUILD_RELABEL, BUILD_NO_RELABEL = 1, 2


def build_flattenings(ctx: Context, dims, i: torch.Tensor, j: torch.Tensor, k: torch.Tensor,
                      val: torch.Tensor, relabel: bool | None = None,
                      chunk_len: int = 0) -> Tensor:
    """relabel: None (by size), True or False (dfacto_build_flattenings_ex flags);
    chunk_len: stream entries per MTTKRP work chunk (0: the library's default)."""
    for x in (i, j, k):
        if x.dtype not in (torch.int32, torch.uint32) or not x.is_contiguous() or not x.is_cuda:
            raise TypeError("indices must be contiguous int32/uint32 CUDA tensors")
    if val.dtype != torch.float32 or not val.is_contiguous() or not val.is_cuda:
        raise TypeError("values must be a contiguous float32 CUDA tensor")
    n = int(val.numel())
    if not (i.numel() == j.numel() == k.numel() == n):
        raise ValueError("index and value arrays differ in length")
    d = (ctypes.c_int64 * 3)(*[int(x) for x in dims])
    h = ctypes.c_void_p()
    flags = 0 if relabel is None else (BUILD_RELABEL if relabel else BUILD_NO_RELABEL)
    ctx.check(load().dfacto_build_flattenings_ex(ctx.handle, d, n, _ptr(i), _ptr(j), _ptr(k),
                                                 _ptr(val), flags, int(chunk_len),
                                                 ctypes.byref(h)))
    return Tensor(h, ctx.allocator)


def build_ratings(ctx: Context, dims, i: torch.Tensor, j: torch.Tensor, y: torch.Tensor) -> Tensor:
    """The joint model's ratings matrix (users x items, observed entries)."""
    for x in (i, j):
        if x.dtype not in (torch.int32, torch.uint32) or not x.is_contiguous() or not x.is_cuda:
            raise TypeError("indices must be contiguous int32/uint32 CUDA tensors")
    if y.dtype != torch.float32 or not y.is_contiguous() or not y.is_cuda:
        raise TypeError("ratings must be a contiguous float32 CUDA tensor")
    n = int(y.numel())
    if not (i.numel() == j.numel() == n):
        raise ValueError("index and rating arrays differ in length")
    d = (ctypes.c_int64 * 2)(*[int(x) for x in dims])
    h = ctypes.c_void_p()
    ctx.check(load().dfacto_build_ratings(ctx.handle, d, n, _ptr(i), _ptr(j), _ptr(y),
                                          ctypes.byref(h)))
    return Tensor(h, ctx.allocator)


def joint_grad(ctx: Context, X: Tensor, Y: Tensor, factors, grads, f: torch.Tensor, mu: float,
               lam: float):
    """Gradients and objective of the joint matrix completion + tensor
    factorization model at one point."""
    dims, R, code = _check_factors(X, factors)
    for m, g in enumerate(grads):
        if g.dtype != torch.float32 or not g.is_contiguous() or tuple(g.shape) != (dims[m], R):
            raise ValueError("gradients must be contiguous float32 (dims[m], R) tensors")
    if f.dtype != torch.float64 or f.numel() < 1 or not f.is_cuda:
        raise ValueError("f must be a float64 CUDA tensor")
    ctx.check(load().dfacto_joint_grad(ctx.handle, X.handle, Y.handle, R, code, float(mu),
                                       float(lam), _ptrs(factors), _ptrs(grads), _ptr(f)))


def joint_als_iter(ctx: Context, X: Tensor, Y: Tensor, factors, mu: float, lam: float):
    """One ALS iteration of the joint model; factors updated in place."""
    dims, R, code = _check_factors(X, factors)
    ctx.check(load().dfacto_joint_als_iter(ctx.handle, X.handle, Y.handle, R, code, float(mu),
                                           float(lam), _ptrs(factors)))


def tensor_get_info(t: Tensor) -> dict:
    return t.info()


def tensor_export(ctx: Context, t: Tensor, mode: int) -> dict:
    import numpy as np
    inf = t.info()
    nr, nf, nz = inf["nroot"][mode], inf["nfib"][mode], inf["nnz"]
    root_id = np.empty(max(nr, 1), np.uint32)
    root_ptr = np.empty(nr + 1, np.int64)
    fib_mid = np.empty(max(nf, 1), np.uint32)
    fib_ptr = np.empty(nf + 1, np.int64)
    leaf = np.empty(max(nz, 1), np.uint32)
    val = np.empty(max(nz, 1), np.float32)
    c = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    ctx.check(load().dfacto_tensor_export(ctx.handle, t.handle, int(mode), c(root_id), c(root_ptr),
                                          c(fib_mid), c(fib_ptr), c(leaf), c(val)))
    return dict(root_id=root_id[:nr], root_ptr=root_ptr, fib_mid=fib_mid[:nf], fib_ptr=fib_ptr,
                leaf=leaf[:nz], val=val[:nz])


def gather_order(ctx: Context, t: Tensor, mode: int, table: int):
    """A relabeled mode's row order: table 0 the leaf table, 1 the mid table
    (dfacto_tensor_gather_order)."""
    import numpy as np
    dims = t.info()["dims"]
    rows = dims[(mode + 1) % 3] if table == 0 else dims[(mode + 2) % 3]
    out = np.empty(rows, np.uint32)
    ctx.check(load().dfacto_tensor_gather_order(ctx.handle, t.handle, int(mode), int(table),
                                                out.ctypes.data_as(ctypes.c_void_p)))
    return out


def _check_factors(t: Tensor, factors, R: int | None = None, skip: int | None = None):
    dims = t.info()["dims"]
    code = None
    for m, F in enumerate(factors):
        if F is None:
            if m == skip:
                continue
            raise ValueError(f"factor {m} is None")
        if not F.is_cuda or not F.is_contiguous() or F.dim() != 2:
            raise TypeError("factors must be contiguous 2-D CUDA tensors")
        if F.shape[0] != dims[m]:
            raise ValueError(f"factor {m} has {F.shape[0]} rows, expected {dims[m]}")
        if R is None:
            R = int(F.shape[1])
        if F.shape[1] != R:
            raise ValueError("factors disagree on R")
        c = _dtype_code(F)
        if code is not None and c != code:
            raise TypeError("factors must share one dtype")
        code = c
    return dims, R, code


def mttkrp(ctx: Context, t: Tensor, mode: int, factors, out: torch.Tensor | None = None):
    """out[dims[mode], R] (float32) = MTTKRP of ``mode`` with factors (A, B, C)."""
    dims, R, code = _check_factors(t, factors, skip=mode)
    if out is None:
        out = torch.empty((dims[mode], R), dtype=torch.float32, device=f"cuda:{ctx.device}")
    if out.dtype != torch.float32 or not out.is_contiguous() or tuple(out.shape) != (dims[mode], R):
        raise ValueError("out must be a contiguous float32 tensor of shape (dims[mode], R)")
    ctx.check(load().dfacto_mttkrp(ctx.handle, t.handle, int(mode), R, code, _ptrs(factors),
                                   _ptr(out)))
    return out


def mttkrp_noalloc(ctx: Context, t: Tensor, mode: int, factors, out: torch.Tensor):
    """dfacto_mttkrp with the library's fixed scratch array (no allocation;
    calls on one GPU must not overlap)."""
    dims, R, code = _check_factors(t, factors, skip=mode)
    if out.dtype != torch.float32 or not out.is_contiguous() or tuple(out.shape) != (dims[mode], R):
        raise ValueError("out must be a contiguous float32 tensor of shape (dims[mode], R)")
    ctx.check(load().dfacto_mttkrp_noalloc(ctx.handle, t.handle, int(mode), R, code,
                                           _ptrs(factors), _ptr(out)))
    return out


def gather_probe(ctx: Context, t: Tensor, mode: int, factors, pattern: int,
                 sink: torch.Tensor | None = None) -> torch.Tensor:
    """The MTTKRP main kernel's memory requests for ``mode`` without its
    arithmetic (pattern 0 own rows, 1 uniform random rows, 2 rows among the
    first 4096, 3 no gathers, 4 rows among the first 32, 5 rows of a small
    LDS table); returns the sink buffer."""
    dims, R, code = _check_factors(t, factors, skip=mode)
    n = 64 * max(1, int(t.info()["nchunk"][mode]))
    if sink is None or sink.numel() < n:
        sink = torch.empty(n, dtype=torch.float32, device=f"cuda:{ctx.device}")
    ctx.check(load().dfacto_gather_probe(ctx.handle, t.handle, int(mode), R, code,
                                         _ptrs(factors), int(pattern), _ptr(sink)))
    return sink


def als_iter(ctx: Context, t: Tensor, factors, lam: torch.Tensor, fit: torch.Tensor,
             reg: float = 0.0):
    """One CP-ALS iteration in place on ``factors``; lam (R,) and fit (1,) are
    float64 device tensors written on the stream."""
    dims, R, code = _check_factors(t, factors)
    if lam.dtype != torch.float64 or lam.numel() < R or not lam.is_cuda:
        raise ValueError("lam must be a float64 CUDA tensor with R elements")
    if fit.dtype != torch.float64 or fit.numel() < 1 or not fit.is_cuda:
        raise ValueError("fit must be a float64 CUDA tensor")
    ctx.check(load().dfacto_als_iter(ctx.handle, t.handle, R, code, float(reg), _ptrs(factors),
                                     _ptr(lam), _ptr(fit)))


def gd_grad(ctx: Context, t: Tensor, factors, grads, f: torch.Tensor, reg: float = 0.0):
    """Gradients (float32, shapes of the factors) and objective f (float64)."""
    dims, R, code = _check_factors(t, factors)
    for m, g in enumerate(grads):
        if g.dtype != torch.float32 or not g.is_contiguous() or tuple(g.shape) != (dims[m], R):
            raise ValueError("gradients must be contiguous float32 (dims[m], R) tensors")
    if f.dtype != torch.float64 or f.numel() < 1 or not f.is_cuda:
        raise ValueError("f must be a float64 CUDA tensor")
    ctx.check(load().dfacto_gd_grad(ctx.handle, t.handle, R, code, float(reg), _ptrs(factors),
                                    _ptrs(grads), _ptr(f)))


def gd_step(ctx: Context, t: Tensor, factors, grads, reg: float = 0.0, alpha0: float = 1.0,
            shrink: float = 0.5, c: float = 1e-4, max_trials: int = 30) -> dict:
    """One GD iteration with an Armijo backtracking line search; the factors
    are updated in place, grads receive the gradients at the input point.
    Returns dict(f0, f, gnorm2, alpha, trials, accepted)."""
    dims, R, code = _check_factors(t, factors)
    for m, g in enumerate(grads):
        if g.dtype != torch.float32 or not g.is_contiguous() or tuple(g.shape) != (dims[m], R):
            raise ValueError("gradients must be contiguous float32 (dims[m], R) tensors")
    ls = _LineSearch(float(alpha0), float(shrink), float(c), int(max_trials))
    info = _GdStepInfo()
    ctx.check(load().dfacto_gd_step(ctx.handle, t.handle, R, code, float(reg), _ptrs(factors),
                                    _ptrs(grads), ctypes.byref(ls), ctypes.byref(info)))
    return dict(f0=info.f0, f=info.f, gnorm2=info.gnorm2, alpha=info.alpha, trials=info.trials,
                accepted=bool(info.accepted))


class Group:
    """Grouped CP-ALS over several built tensors (dfacto_group_*).

    factors[t] = (A, B, C) device tensors of member t (one dtype for all,
    16-byte aligned rows), lams[t] float64 (R_t,), fits float64 (n,).  The
    tensors and buffers must stay alive while the group lives (the group
    keeps references)."""

    def __init__(self, ctx: Context, tensors, factors, lams, fits: torch.Tensor,
                 reg: float = 0.0, graph: bool = False, tune: bool = False,
                 ctx_stream: bool = False, own_factors: bool = False):
        n = len(tensors)
        if not (len(factors) == len(lams) == n) or n < 1:
            raise ValueError("tensors, factors and lams must have one entry per member")
        if fits.dtype != torch.float64 or fits.numel() < n or not fits.is_cuda:
            raise ValueError("fits must be a float64 CUDA tensor with one entry per member")
        ranks, code, ptrs = [], None, []
        for t, (T, F, lam) in enumerate(zip(tensors, factors, lams)):
            _, R, c = _check_factors(T, F)
            if code is not None and c != code:
                raise TypeError("every member must use one factor dtype")
            code = c
            if lam.dtype != torch.float64 or lam.numel() < R or not lam.is_cuda:
                raise ValueError("lam must be a float64 CUDA tensor with R elements")
            ranks.append(R)
            ptrs.extend(x.data_ptr() for x in F)
        self._keep = (list(tensors), [list(F) for F in factors], list(lams), fits)
        th = (ctypes.c_void_p * n)(*[T.handle.value for T in tensors])
        rk = (ctypes.c_int * n)(*ranks)
        fp = (ctypes.c_void_p * (3 * n))(*ptrs)
        lp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in lams])
        flags = ((GROUP_GRAPH if graph else 0) | (GROUP_TUNE if tune else 0)
                 | (GROUP_CTX_STREAM if ctx_stream else 0)
                 | (GROUP_OWN_FACTORS if own_factors else 0))
        h = ctypes.c_void_p()
        ctx.check(load().dfacto_group_create(ctx.handle, n, th, rk, code, float(reg), fp, lp,
                                             _ptr(fits), flags, ctypes.byref(h)))
        self.handle = h
        self.ctx = ctx

    def als(self, iters: int = 1):
        self.ctx.check(load().dfacto_group_als(self.ctx.handle, self.handle, int(iters)))

    def info(self) -> dict:
        inf = _GroupInfo()
        st = load().dfacto_group_get_info(self.handle, ctypes.byref(inf))
        if st != OK:
            raise DfactoError(st, "dfacto_group_get_info failed")
        nc = min(16, inf.mttkrp_classes)
        return dict(members=inf.members, launches_per_iter=inf.launches_per_iter, bytes=inf.bytes,
                    graph=bool(inf.graph), mttkrp_classes=inf.mttkrp_classes,
                    mttkrp_grid=list(inf.mttkrp_grid)[:nc], mttkrp_cpl=list(inf.mttkrp_cpl)[:nc],
                    mttkrp_lanes=list(inf.mttkrp_lanes)[:nc],
                    mttkrp_chunks_per_group=list(inf.mttkrp_chunks_per_group)[:nc],
                    mttkrp_forms=list(inf.mttkrp_forms)[:nc])

    def set_form(self, cls: int, form: int, grid: int):
        st = load().dfacto_group_set_form(self.handle, int(cls), int(form), int(grid))
        if st != OK:
            raise DfactoError(st, "dfacto_group_set_form failed")

    def close(self):
        if getattr(self, "handle", None):
            load().dfacto_group_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def group_create(ctx, tensors, factors, lams, fits, reg=0.0, graph=False, tune=False) -> Group:
    return Group(ctx, tensors, factors, lams, fits, reg, graph, tune)


def group_als(ctx, g: Group, iters: int = 1):
    g.als(iters)


def group_get_info(g: Group) -> dict:
    return g.info()


def group_destroy(g: Group):
    g.close()


class Server:
    """A dfacto_server: CP-ALS solves submitted at any time, run with
    continuous batching on one device.  Inputs are host numpy arrays (kept
    alive here until the request is collected); results come back as host
    numpy arrays."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, max_slots: int = 16):
        h = ctypes.c_void_p()
        st = load().dfacto_server_create(int(device), int(hbm_budget), int(max_slots),
                                         ctypes.byref(h))
        if st != OK:
            raise DfactoError(st, "dfacto_server_create failed")
        self.handle = h
        self._reqs = {}

    def submit(self, dims, i, j, k, val, R: int, init, dtype: str = "f32", reg: float = 0.0,
               tol: float = 1e-4, max_iters: int = 50) -> int:
        import numpy as np
        arrs = [np.ascontiguousarray(x, dtype=np.uint32) for x in (i, j, k)]
        v = np.ascontiguousarray(val, dtype=np.float32)
        n = int(v.size)
        if not all(a.size == n for a in arrs):
            raise ValueError("index and value arrays differ in length")
        ini = [np.ascontiguousarray(f, dtype=np.float32) for f in init]
        for m in range(3):
            if ini[m].shape != (int(dims[m]), int(R)):
                raise ValueError(f"init[{m}] must have shape (dims[{m}], R)")
        outF = [np.empty((int(dims[m]), int(R)), np.float32) for m in range(3)]
        outL = np.empty(int(R), np.float64)
        rq = _Request()
        rq.dims = (ctypes.c_int64 * 3)(*[int(d) for d in dims])
        rq.nnz = n
        rq.i, rq.j, rq.k = (a.ctypes.data for a in arrs)
        rq.val = v.ctypes.data
        rq.R = int(R)
        rq.dtype = F32 if dtype == "f32" else BF16
        rq.reg = float(reg)
        rq.init = (ctypes.c_void_p * 3)(*[f.ctypes.data for f in ini])
        rq.tol = float(tol)
        rq.max_iters = int(max_iters)
        rq.out_F = (ctypes.c_void_p * 3)(*[f.ctypes.data for f in outF])
        rq.out_lambda = outL.ctypes.data
        rid = ctypes.c_int64()
        st = load().dfacto_server_submit(self.handle, ctypes.byref(rq), ctypes.byref(rid))
        if st != OK:
            raise DfactoError(st, "dfacto_server_submit failed")
        self._reqs[rid.value] = (arrs, v, ini, outF, outL)
        return rid.value

    def _result(self, rid, s: _RequestStatus) -> dict:
        _, _, _, outF, outL = self._reqs.pop(rid)
        return dict(status=s.status, fit=s.fit, iters=s.iters, t_submit=s.t_submit,
                    t_admit=s.t_admit, t_done=s.t_done, factors=outF, lam=outL)

    def poll(self, rid: int):
        """The result dict once done, else None."""
        s = _RequestStatus()
        st = load().dfacto_server_poll(self.handle, int(rid), ctypes.byref(s))
        if st == E_AGAIN:
            return None
        if st != OK:
            raise DfactoError(st, "dfacto_server_poll failed")
        return self._result(rid, s)

    def wait(self, rid: int) -> dict:
        s = _RequestStatus()
        st = load().dfacto_server_wait(self.handle, int(rid), ctypes.byref(s))
        if st != OK:
            raise DfactoError(st, "dfacto_server_wait failed")
        return self._result(rid, s)

    def stats(self) -> dict:
        s = _ServerStats()
        st = load().dfacto_server_get_stats(self.handle, ctypes.byref(s))
        if st != OK:
            raise DfactoError(st, "dfacto_server_get_stats failed")
        return dict(pending=s.pending, running=s.running, finished=s.finished,
                    peak_active=s.peak_active, iterations=s.iterations, budget=s.budget,
                    t_admit=s.t_admit, t_build=s.t_build, t_groups=s.t_groups,
                    t_iterate=s.t_iterate,
                    t_deliver=s.t_deliver)

    def close(self):
        if getattr(self, "handle", None):
            load().dfacto_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def server_create(device=0, hbm_budget=0, max_slots=16) -> Server:
    return Server(device, hbm_budget, max_slots)


def profile_enable(ctx: Context, on: bool = True):
    ctx.check(load().dfacto_profile_enable(ctx.handle, 1 if on else 0))


def profile_read(ctx: Context) -> dict:
    """Main-kernel MTTKRP launches recorded since enable/last read."""
    n = ctypes.c_int64()
    ms, b, f = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    ctx.check(load().dfacto_profile_read(ctx.handle, ctypes.byref(n), ctypes.byref(ms),
                                         ctypes.byref(b), ctypes.byref(f)))
    return dict(launches=n.value, ms=ms.value, bytes=b.value, flops=f.value)
