"""Host-side conversion between site-major colour vectors and the library's
spinor buffers (the layouts of include/hisq.h).  numpy only; no arithmetic of
the operator happens here.

* ``to_planes(vec, parity_sites)``: [V, 3] full-lattice vector -> [3, Vh]
  values on the sites of one parity, in checkerboard order (h = lex >> 1);
* ``encode(planes, prec)`` / ``decode(raw, vh, prec)``: [3, Vh] complex <->
  the raw bytes of one buffer of precision ``"fp64" | "fp32" | "fp16s"``.
"""

from __future__ import annotations

import numpy as np


def parity_sites(dims, parity: int) -> np.ndarray:
    """Lexicographic indices of the sites of one parity (increasing, so that
    their position in the list is the checkerboard index h)."""
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    par = ((x + y + z + t) & 1).ravel()
    return np.nonzero(par == parity)[0]


def to_planes(vec_full: np.ndarray, sites: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(vec_full[sites].T)


def encode(planes: np.ndarray, prec: str) -> np.ndarray:
    vh = planes.shape[1]
    if prec == "fp64":
        return np.ascontiguousarray(planes.astype(np.complex128)).view(np.uint8).ravel()
    if prec == "fp32":
        c = planes.astype(np.complex64)
        a = np.ascontiguousarray(c[:2].T)
        b = np.ascontiguousarray(c[2])
        return np.concatenate([a.view(np.uint8).ravel(), b.view(np.uint8).ravel()])
    if prec == "fp16s":
        re = np.stack([planes.real, planes.imag], axis=-1).transpose(1, 0, 2).reshape(vh, 6)
        scale = np.abs(re).max(axis=1).astype(np.float32)
        inv = np.where(scale > 0, 1.0 / scale.astype(np.float64), 0.0)
        halves = (re * inv[:, None]).astype(np.float16)
        rec = np.empty((vh, 16), np.uint8)
        rec[:, :12] = halves.view(np.uint8).reshape(vh, 12)
        rec[:, 12:] = scale.view(np.uint8).reshape(vh, 4)
        return rec.ravel()
    raise ValueError(prec)


def decode(raw: np.ndarray, vh: int, prec: str) -> np.ndarray:
    raw = np.ascontiguousarray(raw).view(np.uint8)
    if prec == "fp64":
        return raw[: 48 * vh].view(np.complex128).reshape(3, vh).copy()
    if prec == "fp32":
        a = raw[: 16 * vh].view(np.complex64).reshape(vh, 2)
        b = raw[16 * vh: 24 * vh].view(np.complex64)
        return np.stack([a[:, 0], a[:, 1], b]).astype(np.complex128)
    if prec == "fp16s":
        rec = raw[: 16 * vh].reshape(vh, 16)
        h = np.ascontiguousarray(rec[:, :12]).view(np.float16).reshape(vh, 3, 2).astype(np.float64)
        s = np.ascontiguousarray(rec[:, 12:]).view(np.float32).reshape(vh).astype(np.float64)
        v = h * s[:, None, None]
        return (v[..., 0] + 1j * v[..., 1]).T.copy()
    raise ValueError(prec)
