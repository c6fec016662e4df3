"""ctypes wrappers around the C oracle (FP64, canonical lexicographic layout).

Every function takes numpy complex128 arrays in the canonical layout:
links ``[V, 4, 3, 3]``, colour vectors ``[V, 3]`` over the full lattice.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None


def library_path() -> str:
    return _build.OUT


def _lib():
    global _LIB
    if _LIB is None:
        # HISQ_ORACLE_LIB: a differently built oracle (the mutation tests load
        # copies with planted mistakes through it)
        path = os.environ.get("HISQ_ORACLE_LIB") or _build.OUT
        if path == _build.OUT and (not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC)):
            _build.build(force=True, quiet=True)
        lib = C.CDLL(path)
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
        lib.oracle_dslash.argtypes = [ip, dp, dp, dp, dp, C.c_int]
        lib.oracle_dslash_phased.argtypes = [ip, dp, dp, dp, dp, C.c_int, C.c_int]
        lib.oracle_normal_op.argtypes = [ip, dp, dp, C.c_double, C.c_double, dp, dp, dp]
        lib.oracle_true_residual.argtypes = [ip, dp, dp, C.c_double, C.c_double, dp, dp]
        lib.oracle_true_residual.restype = C.c_double
        lib.oracle_cg.argtypes = [ip, dp, dp, C.c_double, C.c_double, dp, dp, C.c_double, C.c_int,
                                  ip, dp]
        lib.oracle_cg.restype = C.c_int
        lib.oracle_num_threads.restype = C.c_int
        lib.oracle_dslash_sites.argtypes = [ip, dp, dp, dp, C.POINTER(C.c_int64), C.c_long, dp]
        _LIB = lib
    return _LIB


def _dims(dims):
    d = (C.c_int * 4)(*[int(v) for v in dims])
    if any(v < 4 or v % 2 for v in d):
        raise ValueError(f"lattice extents must be even and >= 4: {tuple(dims)}")
    return d


def _ptr(a: np.ndarray):
    assert a.dtype == np.complex128 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _links(dims, U):
    U = np.ascontiguousarray(U, np.complex128)
    if U.shape != (int(np.prod(dims)), 4, 3, 3):
        raise ValueError(f"links must be [V,4,3,3], got {U.shape}")
    return U


def _vec(dims, v):
    v = np.ascontiguousarray(v, np.complex128)
    if v.shape != (int(np.prod(dims)), 3):
        raise ValueError(f"vector must be [V,3], got {v.shape}")
    return v


def num_threads() -> int:
    return int(_lib().oracle_num_threads())


def dslash(dims, fat, lng, vec, out_parity: int) -> np.ndarray:
    """D vec on the sites of ``out_parity`` (zero elsewhere); links phase-folded."""
    fat, lng, vec = _links(dims, fat), _links(dims, lng), _vec(dims, vec)
    out = np.empty_like(vec)
    _lib().oracle_dslash(_dims(dims), _ptr(fat), _ptr(lng), _ptr(vec), _ptr(out), int(out_parity))
    return out


def dslash_sites(dims, fat, lng, vec, sites) -> np.ndarray:
    """(D vec) at the given lexicographic sites only; returns [len(sites), 3]."""
    fat, lng, vec = _links(dims, fat), _links(dims, lng), _vec(dims, vec)
    sites = np.ascontiguousarray(sites, np.int64)
    out = np.empty((len(sites), 3), np.complex128)
    _lib().oracle_dslash_sites(_dims(dims), _ptr(fat), _ptr(lng), _ptr(vec),
                               sites.ctypes.data_as(C.POINTER(C.c_int64)), len(sites), _ptr(out))
    return out


def dslash_phased(dims, fat, lng, vec, out_parity: int, antiperiodic_t: bool = False) -> np.ndarray:
    """Same operator with the staggered phases / time boundary applied explicitly."""
    fat, lng, vec = _links(dims, fat), _links(dims, lng), _vec(dims, vec)
    out = np.empty_like(vec)
    _lib().oracle_dslash_phased(_dims(dims), _ptr(fat), _ptr(lng), _ptr(vec), _ptr(out),
                                int(out_parity), int(bool(antiperiodic_t)))
    return out


def normal_op(dims, fat, lng, mass: float, vec, sigma: float = 0.0) -> np.ndarray:
    """(4 m^2 + sigma - D_eo D_oe) vec on even sites; vec must vanish on odd sites."""
    fat, lng, vec = _links(dims, fat), _links(dims, lng), _vec(dims, vec)
    out = np.empty_like(vec)
    tmp = np.empty_like(vec)
    _lib().oracle_normal_op(_dims(dims), _ptr(fat), _ptr(lng), float(mass), float(sigma),
                            _ptr(vec), _ptr(out), _ptr(tmp))
    return out


def true_residual(dims, fat, lng, mass: float, b, x, sigma: float = 0.0) -> float:
    fat, lng, b, x = _links(dims, fat), _links(dims, lng), _vec(dims, b), _vec(dims, x)
    return float(_lib().oracle_true_residual(_dims(dims), _ptr(fat), _ptr(lng), float(mass),
                                             float(sigma), _ptr(b), _ptr(x)))


def cg(dims, fat, lng, mass: float, b, tol: float = 1e-10, max_iter: int = 100000,
       sigma: float = 0.0):
    """Plain FP64 CG on A + sigma from x = 0; stops on the true residual.

    Returns ``(x, status, iterations, true_relative_residual)``; status 0 is
    converged, 1 not converged, 2 breakdown.
    """
    fat, lng, b = _links(dims, fat), _links(dims, lng), _vec(dims, b)
    x = np.zeros_like(b)
    it = C.c_int(0)
    tr = C.c_double(0.0)
    st = _lib().oracle_cg(_dims(dims), _ptr(fat), _ptr(lng), float(mass), float(sigma), _ptr(b),
                          _ptr(x), float(tol), int(max_iter), C.byref(it), C.byref(tr))
    return x, int(st), int(it.value), float(tr.value)


def multishift_cg(dims, fat, lng, mass: float, shifts, b, tol: float = 1e-10,
                  max_iter: int = 100000):
    """x_k = (A + sigma_k)^{-1} b for every shift, as independent plain CGs: the
    definition of what a multi-shift solver must return."""
    out = []
    for s in shifts:
        out.append(cg(dims, fat, lng, mass, b, tol, max_iter, sigma=float(s)))
    return out
