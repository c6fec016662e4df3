"""Test-side conversion between the canonical full-lattice vectors of the
oracle ([V, 3] complex128) and the library's public spinor buffers
([3][Vh] colour-major planes of one parity; FP16S adds a per-site scale).

Written from the layout stated in include/hisq.h; shares no code with the
library.
"""

from __future__ import annotations

import numpy as np

import synth


def parity_sites(dims, parity: int) -> np.ndarray:
    """Lexicographic indices of the sites of one parity, in checkerboard order
    (h = lex >> 1 is increasing along them)."""
    return np.nonzero(synth.site_parity(dims) == parity)[0]


def to_cb(dims, vec_full: np.ndarray, parity: int) -> np.ndarray:
    """[V,3] -> [3, Vh] complex128 on the sites of `parity`."""
    s = parity_sites(dims, parity)
    assert np.array_equal(s >> 1, np.arange(len(s)))
    return np.ascontiguousarray(vec_full[s].T)


def from_cb(dims, cb: np.ndarray, parity: int) -> np.ndarray:
    V = synth.volume(dims)
    out = np.zeros((V, 3), np.complex128)
    out[parity_sites(dims, parity)] = cb.T
    return out


def encode(cb: np.ndarray, prec: str) -> np.ndarray:
    """[3, Vh] complex128 -> raw bytes (uint8) of one library spinor buffer."""
    vh = cb.shape[1]
    if prec == "fp64":
        return np.ascontiguousarray(cb.astype(np.complex128)).view(np.uint8).ravel()
    if prec == "fp32":
        c = cb.astype(np.complex64)
        plane_a = np.ascontiguousarray(c[:2].T)  # [Vh, 2] complex = (re0, im0, re1, im1)
        plane_b = np.ascontiguousarray(c[2])     # [Vh] complex
        return np.concatenate([plane_a.view(np.uint8).ravel(), plane_b.view(np.uint8).ravel()])
    if prec == "fp16s":
        re = np.stack([cb.real, cb.imag], axis=-1).transpose(1, 0, 2).reshape(vh, 6)  # per site
        scale = np.abs(re).max(axis=1).astype(np.float32)
        inv = np.where(scale > 0, 1.0 / scale.astype(np.float64), 0.0)
        halves = (re * inv[:, None]).astype(np.float16)
        rec = np.zeros((vh, 16), np.uint8)
        rec[:, :12] = halves.view(np.uint8).reshape(vh, 12)
        rec[:, 12:] = scale.view(np.uint8).reshape(vh, 4)
        return rec.ravel()
    raise ValueError(prec)


def decode(raw: np.ndarray, vh: int, prec: str) -> np.ndarray:
    """Raw bytes of one buffer -> [3, Vh] complex128."""
    raw = np.ascontiguousarray(raw).view(np.uint8)
    if prec == "fp64":
        return raw.view(np.complex128).reshape(3, vh).copy()
    if prec == "fp32":
        a = raw[: 16 * vh].view(np.complex64).reshape(vh, 2)
        b = raw[16 * vh: 24 * vh].view(np.complex64)
        return np.stack([a[:, 0], a[:, 1], b]).astype(np.complex128)
    if prec == "fp16s":
        rec = raw[: 16 * vh].reshape(vh, 16)
        halves = np.ascontiguousarray(rec[:, :12]).view(np.float16).reshape(vh, 3, 2).astype(np.float64)
        scale = np.ascontiguousarray(rec[:, 12:]).view(np.float32).reshape(vh).astype(np.float64)
        v = halves * scale[:, None, None]
        return (v[..., 0] + 1j * v[..., 1]).T.copy()
    raise ValueError(prec)


def spinor_nbytes(prec: str, vh: int) -> int:
    return {"fp64": 48, "fp32": 24, "fp16s": 16}[prec] * vh


def rel_l2(a, b) -> float:
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
