"""Save and restore preconditioner-network weights.

A checkpoint is two files: ``<path>.bin`` holds the complex weights as raw
little-endian complex128 in the library's order (layer by layer, each
[9 paths][C_out][C_in]), and ``<path>.json`` a header with the format version,
the channel counts, the number of weights, the lattice and whatever the caller
adds (seed, loss, training steps).  Gauge fields need no checkpoint: they are
reproducible from their seeds.
"""

from __future__ import annotations

import json
import os

import numpy as np

FORMAT = 1


def num_weights(channels) -> int:
    ch = [int(c) for c in channels]
    return sum(9 * a * b for a, b in zip(ch[:-1], ch[1:]))


def save(path: str, weights, channels, dims=None, **meta) -> None:
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.complex128).ravel())
    if w.size != num_weights(channels):
        raise ValueError(f"{w.size} weights do not match channels {tuple(channels)}")
    header = {"format": FORMAT, "dtype": "complex128-le", "channels": [int(c) for c in channels],
              "num_weights": int(w.size), "dims": None if dims is None else [int(d) for d in dims]}
    header.update(meta)
    tmp = path + ".bin.tmp"
    w.astype("<c16").tofile(tmp)
    os.replace(tmp, path + ".bin")
    with open(path + ".json", "w") as f:
        json.dump(header, f, indent=1, sort_keys=True)


def load(path: str):
    """Returns (weights complex128 array, header dict)."""
    with open(path + ".json") as f:
        header = json.load(f)
    if header.get("format") != FORMAT:
        raise ValueError(f"unsupported checkpoint format {header.get('format')}")
    w = np.fromfile(path + ".bin", dtype="<c16")
    if w.size != header["num_weights"] or w.size != num_weights(header["channels"]):
        raise ValueError("checkpoint size does not match its header")
    return w.astype(np.complex128), header
