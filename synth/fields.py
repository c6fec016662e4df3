"""Seeded synthetic gauge fields and sources in the canonical lexicographic layout.

Canonical layout (both sides of the parity tests read it):

* site index ``lex = x + Lx*(y + Ly*(z + Lz*t))``, direction mu = 0..3 <-> x,y,z,t;
* links: complex128 array ``[V, 4, 3, 3]``; ``U[s, mu]`` maps the colour vector at
  ``s + mu`` to ``s`` (row index = colour at ``s``);
* colour vectors: complex128 array ``[V, 3]`` over the full lattice, zero on the
  sites of the parity the vector does not live on.

Field recipe (the workloads of the benchmark configurations):

* thin links ``U = exp(i*eps*H)`` with ``H = sum_a h_a lambda_a / 2``,
  ``h_a ~ N(0, 1)`` and ``lambda_a`` the Gell-Mann matrices;
* fat links ``F = 0.6 U + 0.1 R`` with ``R`` Haar-random SU(3) (a general 3x3
  complex matrix, not unitary);
* Naik long links ``L_mu(x) = U_mu(x) U_mu(x+mu) U_mu(x+2mu)``;
* the staggered phases ``eta_mu(x)`` and the boundary signs are folded into F, L
  (and into the returned thin links), so the operator itself is sign free.

Random numbers come from numpy's PCG64 seeded with
``[2111, 10354, cfg_id, stream_id, t]``: one stream per purpose and per time
slice, so any slice can be regenerated alone and the result does not depend on
how many worker processes built it.
"""

from __future__ import annotations

import math
import mmap
import multiprocessing as mp
import os

import numpy as np

SEED_BASE = (2111, 10354)

STREAM_THIN = 0
STREAM_FAT = 1
STREAM_SRC = 2
STREAM_NN_INIT = 3
STREAM_NN_PAIRS = 4
STREAM_GAUGE_TF = 5

# Workloads: lattice shape, link randomness, quark mass, right-hand sides.
CONFIGS = {
    "c1": dict(dims=(8, 8, 8, 8), eps=0.3, mass=0.1, nrhs=1),
    "c2": dict(dims=(32, 32, 32, 8), eps=0.5, mass=0.01, nrhs=1),
    "c3": dict(dims=(48, 48, 48, 12), eps=0.5, mass=0.005, nrhs=16, nshift=12),
    "c4": dict(dims=(32, 32, 32, 8), eps=0.5, mass=0.005, nrhs=1, npairs=2048),
    "c5": dict(dims=(96, 96, 96, 24), eps=0.5, mass=0.002, nrhs=4),
}
CFG_IDS = {"c1": 0, "c2": 1, "c3": 2, "c4": 3, "c5": 4, "test": 99}


def _rng(cfg_id: int, stream: int, *extra: int) -> np.random.Generator:
    return np.random.default_rng([*SEED_BASE, int(cfg_id), int(stream), *map(int, extra)])


def volume(dims) -> int:
    return int(np.prod(dims))


def _check_dims(dims):
    if len(dims) != 4 or any(int(L) < 4 or int(L) % 2 for L in dims):
        raise ValueError(f"lattice extents must be even and >= 4, got {dims}")


def site_coords(dims) -> np.ndarray:
    """(V, 4) int64 coordinates (x, y, z, t) of every site in lexicographic order."""
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx),
                             indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel(), t.ravel()], axis=1)


def site_parity(dims) -> np.ndarray:
    return site_coords(dims).sum(axis=1) & 1


def staggered_eta(dims) -> np.ndarray:
    """(V, 4) staggered phases: eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y),
    eta_3 = (-1)^(x+y+z).  eta_mu does not depend on the mu coordinate."""
    c = site_coords(dims)
    cum = np.concatenate([np.zeros((c.shape[0], 1), np.int64), np.cumsum(c[:, :3], axis=1)], axis=1)
    return np.where(cum & 1, -1.0, 1.0)


def _gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7] = np.diag([1, 1, -2]) / math.sqrt(3)
    return lam


_LAMBDA = _gell_mann()


def su3_near_identity(rng: np.random.Generator, n: int, eps: float) -> np.ndarray:
    """n matrices exp(i*eps*H), H = sum_a h_a lambda_a / 2, h_a ~ N(0,1)."""
    h = rng.standard_normal((n, 8))
    H = np.einsum("na,aij->nij", h, _LAMBDA) * 0.5
    w, v = np.linalg.eigh(H)
    return np.einsum("nij,nj,nkj->nik", v, np.exp(1j * eps * w), v.conj())


def haar_su3(rng: np.random.Generator, n: int) -> np.ndarray:
    """n Haar-random SU(3) matrices: the first two columns are a Gram-Schmidt
    orthonormalised pair of complex Gaussian vectors (a uniform 2-frame), the
    third is fixed by unitarity and det = 1 (conjugated cross product)."""
    g = rng.standard_normal((n, 2, 3, 2))
    a = g[:, 0, :, 0] + 1j * g[:, 0, :, 1]
    b = g[:, 1, :, 0] + 1j * g[:, 1, :, 1]
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b -= a * np.sum(a.conj() * b, axis=1, keepdims=True)
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    c = np.cross(a, b).conj()
    return np.stack([a, b, c], axis=2)


def _slice_shape(dims):
    Lx, Ly, Lz, _ = dims
    return (Lz, Ly, Lx)


# ---------------------------------------------------------------- generation
_SHARED: dict = {}


def _thin_slice_into(t: int):
    d = _SHARED
    dims, cfg_id, eps = d["dims"], d["cfg_id"], d["eps"]
    Vs = volume(dims[:3])
    U = d["U"].reshape(dims[3], Vs, 4, 3, 3)
    U[t] = su3_near_identity(_rng(cfg_id, STREAM_THIN, t), Vs * 4, eps).reshape(Vs, 4, 3, 3)


def _derived_slice_into(t: int):
    """Fat, long and folded thin links of time slice t from the shared thin field."""
    d = _SHARED
    dims, cfg_id, apbc = d["dims"], d["cfg_id"], d["apbc"]
    Lx, Ly, Lz, Lt = dims
    Vs = Lx * Ly * Lz
    sh = _slice_shape(dims)
    U = d["U"].reshape(Lt, *sh, 4, 3, 3)
    F = d["F"].reshape(Lt, *sh, 4, 3, 3)
    L = d["L"].reshape(Lt, *sh, 4, 3, 3)
    T = d["T"].reshape(Lt, *sh, 4, 3, 3) if d["T"] is not None else None
    u0 = U[t]
    R = haar_su3(_rng(cfg_id, STREAM_FAT, t), Vs * 4).reshape(*sh, 4, 3, 3)
    f = 0.6 * u0 + 0.1 * R
    lng = np.empty_like(u0)
    for mu, axis in ((0, 2), (1, 1), (2, 0)):
        um = u0[..., mu, :, :]
        lng[..., mu, :, :] = um @ np.roll(um, -1, axis=axis) @ np.roll(um, -2, axis=axis)
    lng[..., 3, :, :] = u0[..., 3, :, :] @ U[(t + 1) % Lt][..., 3, :, :] @ U[(t + 2) % Lt][..., 3, :, :]
    # staggered phases for this slice; constant along their own direction
    z, y, x = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    eta = np.ones((*sh, 4))
    eta[..., 1] = 1 - 2 * (x & 1)
    eta[..., 2] = 1 - 2 * ((x + y) & 1)
    eta[..., 3] = 1 - 2 * ((x + y + z) & 1)
    if not d["fold"]:
        eta[:] = 1.0
    sF = eta.copy()
    sL = eta.copy()
    if apbc and d["fold"]:
        if t + 1 >= Lt:
            sF[..., 3] *= -1
        if t + 3 >= Lt:
            sL[..., 3] *= -1
    F[t] = f * sF[..., None, None]
    L[t] = lng * sL[..., None, None]
    if T is not None:
        T[t] = u0 * sF[..., None, None]


def _shared_array(shape, dtype=np.complex128):
    nbytes = int(np.prod(shape)) * np.dtype(dtype).itemsize
    buf = mmap.mmap(-1, max(nbytes, 1))
    return np.frombuffer(buf, dtype=dtype, count=int(np.prod(shape))).reshape(shape)


def _run(fn, items, workers):
    if workers <= 1 or len(items) <= 1:
        for i in items:
            fn(i)
        return
    ctx = mp.get_context("fork")
    pool = ctx.Pool(min(workers, len(items)))
    try:
        pool.map(fn, items, chunksize=1)
    except BaseException:
        pool.terminate()
        pool.join()
        raise
    # let the workers finish and exit by themselves: terminate() would end them
    # with SIGTERM, which a profiler's signal handler in the process reports as
    # an abort
    pool.close()
    pool.join()


def _gpu_initialised() -> bool:
    """True if this process has already set up the GPU through torch (forking
    worker processes from it is then avoided)."""
    import sys
    torch = sys.modules.get("torch")
    try:
        return bool(torch is not None and torch.cuda.is_initialized())
    except Exception:
        return False


def _memfd_array(shape, dtype=np.complex128):
    """(array, fd): an array in anonymous shared memory that a child process
    can map through the inherited file descriptor."""
    nbytes = max(int(np.prod(shape)) * np.dtype(dtype).itemsize, 1)
    fd = os.memfd_create("hisq_synth_links")
    os.ftruncate(fd, nbytes)
    buf = mmap.mmap(fd, nbytes)
    return np.frombuffer(buf, dtype=dtype, count=int(np.prod(shape))).reshape(shape), fd


def _in_child(kind, nout, V, **kw):
    """Run the generator `kind` ("thin" or "hisq") in a fresh Python interpreter
    (its own fork pool, no GPU state) that writes `nout` link fields into shared
    memory kept by this process.  Used once this process has initialised the
    GPU, where forking workers is avoided."""
    import json
    import subprocess
    import sys
    outs = [_memfd_array((V, 4, 3, 3)) for _ in range(nout)]
    fds = [fd for _, fd in outs]
    spec = json.dumps(dict(kind=kind, fds=fds, **kw))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, sys.argv[1]); "
            "from synth import fields; fields._child_main(sys.argv[2])")
    try:
        subprocess.run([sys.executable, "-c", code, root, spec], pass_fds=fds, check=True)
    finally:
        for fd in fds:
            os.close(fd)  # the mappings stay valid
    return tuple(a for a, _ in outs)


def _child_main(spec: str):
    import json
    d = json.loads(spec)
    dims = tuple(d["dims"])
    V = volume(dims)
    arrs = [np.frombuffer(mmap.mmap(fd, V * 4 * 9 * 16), dtype=np.complex128).reshape(V, 4, 3, 3)
            for fd in d["fds"]]
    if d["kind"] == "thin":
        thin_links(dims, d["cfg_id"], d["eps"], out=arrs[0])
    else:
        hisq_links(dims, d["cfg_id"], d["eps"], antiperiodic_t=d["apbc"], want_thin=len(arrs) == 3,
                   fold=d["fold"], out=arrs)


def _default_workers(V: int) -> int:
    if V < 200_000:
        return 1
    return max(1, min(16, os.cpu_count() or 1))


def thin_links(dims, cfg_id: int, eps: float, workers: int | None = None, out=None) -> np.ndarray:
    """Unfolded thin links U = exp(i eps H), shape (V, 4, 3, 3) (into `out` if given)."""
    _check_dims(dims)
    V = volume(dims)
    workers = _default_workers(V) if workers is None else workers
    if out is None and workers > 1 and _gpu_initialised():
        return _in_child("thin", 1, V, dims=list(dims), cfg_id=cfg_id, eps=eps)[0]
    if out is not None:
        U = out
    else:
        U = _shared_array((V, 4, 3, 3)) if workers > 1 else np.empty((V, 4, 3, 3), np.complex128)
    _SHARED.clear()
    _SHARED.update(dims=tuple(dims), cfg_id=cfg_id, eps=eps, U=U)
    try:
        _run(_thin_slice_into, list(range(dims[3])), workers)
    finally:
        _SHARED.clear()
    return U


def hisq_links(dims, cfg_id: int, eps: float, antiperiodic_t: bool = False,
               want_thin: bool = False, workers: int | None = None, fold: bool = True, out=None, thin=None):
    """Folded fat and Naik links of the benchmark recipe.

    Returns ``(fat, long)`` or ``(fat, long, thin)`` where ``thin`` is the thin
    field with the same phases and one-hop boundary signs folded in.  With
    ``fold=False`` no phase or boundary sign is applied (used to check the
    folding against an operator that applies them itself).  ``out``: arrays
    (shared with forked workers) to write the result into.  ``thin``: the
    unfolded thin links of these arguments (``thin_links``), if already made.

    Large lattices are built by a pool of forked worker processes.  Once this
    process has initialised the GPU, the pool runs in a fresh child interpreter
    instead, which writes into shared memory kept by this process.
    """
    _check_dims(dims)
    V = volume(dims)
    workers = _default_workers(V) if workers is None else workers
    if out is None and thin is None and workers > 1 and _gpu_initialised():
        return _in_child("hisq", 3 if want_thin else 2, V, dims=list(dims), cfg_id=cfg_id, eps=eps,
                         apbc=bool(antiperiodic_t), fold=bool(fold))
    U = thin if thin is not None else thin_links(dims, cfg_id, eps, workers)
    alloc = (lambda: _shared_array((V, 4, 3, 3))) if workers > 1 else \
        (lambda: np.empty((V, 4, 3, 3), np.complex128))
    if out is not None:
        F, L = out[0], out[1]
        T = out[2] if want_thin else None
    else:
        F, L = alloc(), alloc()
        T = alloc() if want_thin else None
    _SHARED.clear()
    _SHARED.update(dims=tuple(dims), cfg_id=cfg_id, apbc=bool(antiperiodic_t), U=U, F=F, L=L, T=T,
                   fold=bool(fold))
    try:
        _run(_derived_slice_into, list(range(dims[3])), workers)
    finally:
        _SHARED.clear()
    del U
    return (F, L, T) if want_thin else (F, L)


def hisq_links_and_thin(dims, cfg_id: int, eps: float):
    """(fat, long, unfolded thin) of the benchmark recipe, the thin links made once."""
    V = volume(dims)
    workers = _default_workers(V)
    U = thin_links(dims, cfg_id, eps, workers)
    F, L = hisq_links(dims, cfg_id, eps, workers=workers, thin=U)  # forked workers only read U
    return F, L, U


def free_links(dims, c1: float, c3: float, antiperiodic_t: bool = False):
    """Free field: F = c1 * eta * bc * 1, L = c3 * eta * bc3 * 1 (folded)."""
    _check_dims(dims)
    V = volume(dims)
    eta = staggered_eta(dims)
    t = site_coords(dims)[:, 3]
    sF = eta.copy()
    sL = eta.copy()
    if antiperiodic_t:
        sF[:, 3] *= np.where(t + 1 >= dims[3], -1.0, 1.0)
        sL[:, 3] *= np.where(t + 3 >= dims[3], -1.0, 1.0)
    eye = np.eye(3, dtype=np.complex128)
    F = (c1 * sF)[:, :, None, None] * eye
    L = (c3 * sL)[:, :, None, None] * eye
    assert F.shape == (V, 4, 3, 3)
    return F, L


def gaussian_source(dims, cfg_id: int, nrhs: int = 1, parity: int = 0,
                    stream: int = STREAM_SRC, index0: int = 0) -> np.ndarray:
    """(nrhs, V, 3) complex vectors, Re and Im ~ N(0,1) on sites of `parity`, 0 elsewhere."""
    V = volume(dims)
    mask = site_parity(dims) == parity
    out = np.zeros((nrhs, V, 3), np.complex128)
    for i in range(nrhs):
        g = _rng(cfg_id, stream, index0 + i).standard_normal((int(mask.sum()), 3, 2))
        out[i, mask] = g[..., 0] + 1j * g[..., 1]
    return out


def plane_wave(dims, n, colour, parity: int | None = 0, antiperiodic_t: bool = False) -> np.ndarray:
    """e^{i p.x} * colour on sites of `parity` (all sites if None).

    p_mu = 2 pi n_mu / L_mu, except p_t = (2 n_t + 1) pi / L_t when the time
    direction is antiperiodic.  Returns (V, 3) and the momentum vector p.
    """
    c = site_coords(dims)
    p = np.array([2 * math.pi * n[m] / dims[m] for m in range(4)])
    if antiperiodic_t:
        p[3] = (2 * n[3] + 1) * math.pi / dims[3]
    phase = np.exp(1j * (c @ p))
    v = phase[:, None] * np.asarray(colour, np.complex128)[None, :]
    if parity is not None:
        v[(c.sum(1) & 1) != parity] = 0
    return v, p


def random_gauge_transform(dims, cfg_id: int = 99) -> np.ndarray:
    """(V, 3, 3) Haar SU(3) matrices g(x)."""
    return haar_su3(_rng(cfg_id, STREAM_GAUGE_TF), volume(dims))


def shifted_ladder(n: int = 12, lo_exp: float = -4.0, hi_exp: float = 0.0) -> np.ndarray:
    """Log-spaced shifts 10^(lo + (hi-lo) k/(n-1)), k = 0..n-1, endpoints included."""
    if n == 1:
        return np.array([10.0 ** lo_exp])
    return 10.0 ** (lo_exp + (hi_exp - lo_exp) * np.arange(n) / (n - 1))
