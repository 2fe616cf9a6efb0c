"""FP64 CPU oracle for the DFacTo hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its Python
binding) never imports, links or calls it, and it imports nothing from the
product package.

The arithmetic lives in ``oracle.c`` (plain double-precision loops over
coordinate-format nonzeros, written from the paper's definitions); this module
only marshals numpy arrays through ctypes.  Citations for each function are in
the C source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c with the host C compiler (no fast-math: IEEE FP64)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-pthread", "-o", tmp,
                               _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_config.argtypes = [ctypes.c_int, ctypes.c_int]
        lib.oracle_config.restype = None
        lib.oracle_mttkrp.argtypes = [i64, P, P, P, P, P, ctypes.c_int, P, P, P, ctypes.c_int, P]
        lib.oracle_mttkrp.restype = None
        lib.oracle_flatten.argtypes = [i64, P, P, P, P, ctypes.c_int, P, P, P, P, P, P, P, P]
        lib.oracle_flatten.restype = i64
        lib.oracle_fiber_partials.argtypes = [i64, P, P, P, P, ctypes.c_int, ctypes.c_int, P, P]
        lib.oracle_fiber_partials.restype = i64
        lib.oracle_normsq.argtypes = [i64, P, P, P, P]
        lib.oracle_normsq.restype = ctypes.c_double
        lib.oracle_inner.argtypes = [i64, P, P, P, P, ctypes.c_int, P, P, P, P]
        lib.oracle_inner.restype = ctypes.c_double
        lib.oracle_als_iter.argtypes = [i64, P, P, P, P, P, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_int, P, P, P, P, P]
        lib.oracle_als_iter.restype = ctypes.c_int
        lib.oracle_gd_grad.argtypes = [i64, P, P, P, P, P, ctypes.c_int, ctypes.c_double,
                                       P, P, P, P, P, P]
        lib.oracle_gd_grad.restype = ctypes.c_double
        lib.oracle_objective.argtypes = [i64, P, P, P, P, P, ctypes.c_int, ctypes.c_double,
                                         P, P, P]
        lib.oracle_objective.restype = ctypes.c_double
        lib.oracle_gd_step.argtypes = [i64, P, P, P, P, P, ctypes.c_int, ctypes.c_double,
                                       P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_int, P]
        lib.oracle_gd_step.restype = ctypes.c_int
        lib.oracle_joint_grad.argtypes = [i64, P, P, P, P, P, i64, P, P, P, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_double, P, P, P, P, P, P]
        lib.oracle_joint_grad.restype = ctypes.c_double
        lib.oracle_joint_als_iter.argtypes = [i64, P, P, P, P, P, i64, P, P, P, ctypes.c_int,
                                              ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                              P, P, P]
        lib.oracle_joint_als_iter.restype = ctypes.c_double
        lib.oracle_joint_als_rows.argtypes = [i64, P, P, P, P, P, i64, P, P, P, ctypes.c_int,
                                              ctypes.c_double, ctypes.c_double, P, P, P,
                                              ctypes.c_int, i64, P, P]
        lib.oracle_joint_als_rows.restype = None
        _lib = lib
    return _lib


def config(threads: int = 1, assume_distinct: bool = False):
    """Worker threads of the oracle's loops (results are bitwise the same for
    any count) and whether the caller guarantees distinct coordinates (then
    ||X||^2 sums the values in input order instead of sorting them)."""
    _load().oracle_config(int(threads), int(bool(assume_distinct)))


def host_threads() -> int:
    """Host cores this process may run on (sched_getaffinity)."""
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def host_threads_capped(cap: int = 16) -> int:
    """host_threads(), at most `cap` (a one-GPU share of a large host)."""
    return max(1, min(host_threads(), int(cap)))


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _coo(i, j, k, val):
    i, j, k, val = _u32(i), _u32(j), _u32(k), _f64(val)
    assert i.shape == j.shape == k.shape == val.shape
    return i, j, k, val


def mttkrp(i, j, k, val, dims, factors, mode: int) -> np.ndarray:
    """MTTKRP of ``mode`` (0, 1, 2) by its per-nonzero element form."""
    lib = _load()
    i, j, k, val = _coo(i, j, k, val)
    A, B, C = (_f64(f) for f in factors)
    R = A.shape[1]
    d = np.asarray(dims, dtype=np.int64)
    out = np.empty((int(dims[mode]), R), dtype=np.float64)
    lib.oracle_mttkrp(len(val), _p(i), _p(j), _p(k), _p(val), _p(d), R, _p(A), _p(B), _p(C),
                      int(mode), _p(out))
    return out


def flatten(i, j, k, val, mode: int) -> dict:
    """Distinct nonzeros of ``mode``'s flattening in (root, mid, leaf) order."""
    lib = _load()
    i, j, k, val = _coo(i, j, k, val)
    n = len(val)
    root_id = np.empty(max(n, 1), np.uint32)
    root_ptr = np.empty(n + 1, np.int64)
    fib_mid = np.empty(max(n, 1), np.uint32)
    fib_ptr = np.empty(n + 1, np.int64)
    leaf = np.empty(max(n, 1), np.uint32)
    v = np.empty(max(n, 1), np.float64)
    nroot = np.zeros(1, np.int64)
    nfib = np.zeros(1, np.int64)
    m = lib.oracle_flatten(n, _p(i), _p(j), _p(k), _p(val), int(mode), _p(root_id), _p(root_ptr),
                           _p(fib_mid), _p(fib_ptr), _p(leaf), _p(v), _p(nroot), _p(nfib))
    nr, nf = int(nroot[0]), int(nfib[0])
    return dict(nnz=int(m), root_id=root_id[:nr].copy(), root_ptr=root_ptr[:nr + 1].copy(),
                fib_mid=fib_mid[:nf].copy(), fib_ptr=fib_ptr[:nf + 1].copy(),
                leaf=leaf[:m].copy(), val=v[:m].copy())


def fiber_partials(i, j, k, val, mode: int, Fleaf) -> np.ndarray:
    """Stage-1 values P[f, :] = sum_leaf x * Fleaf[leaf, :] per nonempty fiber."""
    lib = _load()
    i, j, k, val = _coo(i, j, k, val)
    Fleaf = _f64(Fleaf)
    R = Fleaf.shape[1]
    P = np.empty((max(len(val), 1), R), np.float64)
    nf = lib.oracle_fiber_partials(len(val), _p(i), _p(j), _p(k), _p(val), int(mode), R,
                                   _p(Fleaf), _p(P))
    return P[:nf].copy()


def normsq(i, j, k, val) -> float:
    lib = _load()
    i, j, k, val = _coo(i, j, k, val)
    return float(lib.oracle_normsq(len(val), _p(i), _p(j), _p(k), _p(val)))


def inner(i, j, k, val, factors, lam=None) -> float:
    lib = _load()
    i, j, k, val = _coo(i, j, k, val)
    A, B, C = (_f64(f) for f in factors)
    lp = None
    if lam is not None:
        lam = _f64(lam)
        lp = _p(lam)
    return float(lib.oracle_inner(len(val), _p(i), _p(j), _p(k), _p(val), A.shape[1],
                                  _p(A), _p(B), _p(C), lp))


def als_iter(i, j, k, val, dims, factors, reg: float = 0.0, store: str = "f64"):
    """One CP-ALS iteration.  Returns (A, B, C, lam, info) with new arrays.
    store="bf16": every new factor is rounded to BF16 before later use.

    info = dict(fit, inner_direct, normsq, xhat_sq, pinv_mask)."""
    if store not in ("f64", "bf16"):
        raise ValueError("store must be 'f64' or 'bf16'")
    lib = _load()
    i, j, k, val = _coo(i, j, k, val)
    A, B, C = (np.array(f, dtype=np.float64, order="C", copy=True) for f in factors)
    R = A.shape[1]
    d = np.asarray(dims, dtype=np.int64)
    lam = np.empty(R, np.float64)
    out = np.empty(4, np.float64)
    mask = lib.oracle_als_iter(len(val), _p(i), _p(j), _p(k), _p(val), _p(d), R, float(reg),
                               int(store == "bf16"), _p(A), _p(B), _p(C), _p(lam), _p(out))
    info = dict(fit=float(out[0]), inner_direct=float(out[1]), normsq=float(out[2]),
                xhat_sq=float(out[3]), pinv_mask=int(mask))
    return A, B, C, lam, info


def gd_grad(i, j, k, val, dims, factors, reg: float = 0.0):
    """Gradients of f at one point.  Returns ((gA, gB, gC), f)."""
    lib = _load()
    i, j, k, val = _coo(i, j, k, val)
    A, B, C = (_f64(f) for f in factors)
    R = A.shape[1]
    d = np.asarray(dims, dtype=np.int64)
    g = [np.empty((int(dims[m]), R), np.float64) for m in range(3)]
    f = lib.oracle_gd_grad(len(val), _p(i), _p(j), _p(k), _p(val), _p(d), R, float(reg),
                           _p(A), _p(B), _p(C), _p(g[0]), _p(g[1]), _p(g[2]))
    return tuple(g), float(f)


def objective(i, j, k, val, dims, factors, reg: float = 0.0) -> float:
    """GD objective f at one point (unit weights)."""
    lib = _load()
    i, j, k, val = _coo(i, j, k, val)
    A, B, C = (_f64(f) for f in factors)
    d = np.asarray(dims, dtype=np.int64)
    return float(lib.oracle_objective(len(val), _p(i), _p(j), _p(k), _p(val), _p(d), A.shape[1],
                                      float(reg), _p(A), _p(B), _p(C)))


def gd_step(i, j, k, val, dims, factors, reg: float = 0.0, alpha0: float = 1.0,
            shrink: float = 0.5, c: float = 1e-4, max_trials: int = 30, store: str = "f64"):
    """One GD iteration with an Armijo backtracking line search.  Returns
    (A, B, C, info) with new arrays; info = dict(f0, f, gnorm2, alpha, trials,
    accepted).  store="bf16": trial factors are rounded to BF16 storage."""
    if store not in ("f64", "bf16"):
        raise ValueError("store must be 'f64' or 'bf16'")
    lib = _load()
    i, j, k, val = _coo(i, j, k, val)
    A, B, C = (np.array(f, dtype=np.float64, order="C", copy=True) for f in factors)
    d = np.asarray(dims, dtype=np.int64)
    out = np.zeros(5, np.float64)
    acc = lib.oracle_gd_step(len(val), _p(i), _p(j), _p(k), _p(val), _p(d), A.shape[1], float(reg),
                             _p(A), _p(B), _p(C), float(alpha0), float(shrink), float(c),
                             int(max_trials), 1 if store == "bf16" else 0, _p(out))
    info = dict(f0=float(out[0]), f=float(out[1]), gnorm2=float(out[2]), alpha=float(out[3]),
                trials=int(out[4]), accepted=bool(acc))
    return A, B, C, info


def _ratings(yi, yj, yv):
    yi, yj, yv = _u32(yi), _u32(yj), _f64(yv)
    assert yi.shape == yj.shape == yv.shape
    return yi, yj, yv


def joint_grad(i, j, k, val, dims, yi, yj, yv, factors, mu: float, lam: float):
    """Joint matrix completion + tensor factorization: gradients of f at one
    point and f.  Returns ((gA, gB, gC), f)."""
    lib = _load()
    i, j, k, val = _coo(i, j, k, val)
    yi, yj, yv = _ratings(yi, yj, yv)
    A, B, C = (_f64(f) for f in factors)
    R = A.shape[1]
    d = np.asarray(dims, dtype=np.int64)
    g = [np.empty((int(dims[m]), R), np.float64) for m in range(3)]
    f = lib.oracle_joint_grad(len(val), _p(i), _p(j), _p(k), _p(val), _p(d), len(yv), _p(yi),
                              _p(yj), _p(yv), R, float(mu), float(lam), _p(A), _p(B), _p(C),
                              _p(g[0]), _p(g[1]), _p(g[2]))
    return tuple(g), float(f)


def joint_als_iter(i, j, k, val, dims, yi, yj, yv, factors, mu: float, lam: float,
                   store: str = "f64"):
    """One ALS iteration of the joint model (A, B, C in order).  Returns
    (A, B, C, f) with new arrays; f at the new point.  store="bf16": every
    new factor is rounded to BF16 before later use."""
    if store not in ("f64", "bf16"):
        raise ValueError("store must be 'f64' or 'bf16'")
    lib = _load()
    i, j, k, val = _coo(i, j, k, val)
    yi, yj, yv = _ratings(yi, yj, yv)
    A, B, C = (np.array(f, dtype=np.float64, order="C", copy=True) for f in factors)
    R = A.shape[1]
    d = np.asarray(dims, dtype=np.int64)
    f = lib.oracle_joint_als_iter(len(val), _p(i), _p(j), _p(k), _p(val), _p(d), len(yv), _p(yi),
                                  _p(yj), _p(yv), R, float(mu), float(lam), int(store == "bf16"),
                                  _p(A), _p(B), _p(C))
    return A, B, C, float(f)


def joint_als_rows(i, j, k, val, dims, yi, yj, yv, factors, mu: float, lam: float, mode: int,
                   rows) -> np.ndarray:
    """The listed rows of the users' (mode 0) or items' (mode 1) block of one
    joint ALS iteration, from the factors as given (for mode 1 pass the
    updated A), each solved as joint_als_iter solves it; (len(rows), R)."""
    if mode not in (0, 1):
        raise ValueError("mode must be 0 (users) or 1 (items)")
    lib = _load()
    i, j, k, val = _coo(i, j, k, val)
    yi, yj, yv = _ratings(yi, yj, yv)
    A, B, C = (_f64(f) for f in factors)
    R = A.shape[1]
    d = np.asarray(dims, dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((len(rows), R), dtype=np.float64)
    lib.oracle_joint_als_rows(len(val), _p(i), _p(j), _p(k), _p(val), _p(d), len(yv), _p(yi),
                              _p(yj), _p(yv), R, float(mu), float(lam), _p(A), _p(B), _p(C),
                              int(mode), len(rows), _p(rows), _p(out))
    return out
