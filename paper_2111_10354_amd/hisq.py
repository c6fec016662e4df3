"""Python binding of libhisq.so: argument marshalling only.

Every function here forwards to the C ABI declared in ``include/hisq.h`` with
the same name; all arithmetic runs in the library's HIP kernels.  Torch tensors
are used only as device buffers and for the current HIP stream.  If the
library has not been built, importing this module raises - there is no
fallback implementation.
"""

from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhisq.so")

PREC_FP64, PREC_FP32, PREC_FP16S = 0, 1, 2
PREC_FP16L = 3  # solver sloppy mode only: FP16 links applied to FP32 vectors
PREC_NAMES = {"fp64": PREC_FP64, "fp32": PREC_FP32, "fp16s": PREC_FP16S, "fp16l": PREC_FP16L}

OK, ERR_INVALID, ERR_HIP, ERR_OOM, ERR_UNSUPPORTED = 0, -1, -2, -3, -4
NOT_CONVERGED, BREAKDOWN, CONVERGED_AFTER_FALLBACK = 1, 2, 3


class HisqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hisq error {code}: {msg}")
        self.code = code


class SolverParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("sloppy_prec", C.c_int),
                ("ru_period", C.c_int), ("graph_chunk", C.c_int), ("warm_start", C.c_int),
                ("fallback", C.c_int), ("precond", C.c_void_p), ("ru_delta", C.c_double)]


class SolverStats(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", C.c_int), ("reliable_updates", C.c_int),
                ("fallback_used", C.c_int), ("true_residual", C.c_double), ("wall_ms", C.c_double),
                ("dslash_bytes", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2111_10354_amd/build.py "
                          "(or __graft_entry__.build()) first")
    lib = C.CDLL(LIB_PATH)
    vp, ip, dp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)
    sig = {
        "hisq_version": (C.c_int, []),
        "hisq_last_error": (C.c_char_p, []),
        "hisq_spinor_bytes": (C.c_size_t, [C.c_int, C.c_int64]),
        "hisq_gauge_create": (C.c_int, [C.POINTER(vp), ip, vp, vp, C.c_uint, vp]),
        "hisq_gauge_destroy": (C.c_int, [vp]),
        "hisq_gauge_device_bytes": (C.c_int, [vp, C.POINTER(C.c_size_t)]),
        "hisq_dslash_eo": (C.c_int, [vp, C.c_int, C.c_int, vp, vp, vp]),
        "hisq_dslash_multi_rhs": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, vp, vp, dp, vp, vp]),
        "hisq_dslash_multi_rhs_noalloc": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, vp, vp, dp, vp, vp]),
        "hisq_solver_params_default": (None, [C.POINTER(SolverParams)]),
        "hisq_cg_solve": (C.c_int, [vp, C.c_double, C.c_int, vp, vp, C.POINTER(SolverParams),
                                    C.POINTER(SolverStats), vp]),
        "hisq_multishift_cg": (C.c_int, [vp, C.c_double, C.c_int, dp, vp, vp, C.POINTER(SolverParams),
                                         C.POINTER(SolverStats), vp]),
        "hisq_multishift_cg_batched": (C.c_int, [vp, C.c_double, C.c_int, C.c_int, dp, vp, vp,
                                                 C.POINTER(SolverParams), C.POINTER(SolverStats), vp]),
        "hisq_precond_apply": (C.c_int, [vp, vp, vp, vp, vp]),
        "hisq_autotune": (C.c_int, [vp, C.c_int, C.c_int, C.c_char_p, vp]),
        "hisq_gauge_set_thin": (C.c_int, [vp, vp, vp]),
        "hisq_nn_create": (C.c_int, [C.POINTER(vp), vp, C.c_int, ip, dp, vp]),
        "hisq_nn_destroy": (C.c_int, [vp]),
        "hisq_nn_num_weights": (C.c_int, [vp, C.POINTER(C.c_size_t)]),
        "hisq_nn_get_weights": (C.c_int, [vp, dp, vp]),
        "hisq_nn_set_weights": (C.c_int, [vp, dp, vp]),
        "hisq_nn_loss_grad": (C.c_int, [vp, C.c_int, vp, vp, dp, dp, vp]),
        "hisq_nn_train_step": (C.c_int, [vp, C.c_int, vp, vp, C.c_double, dp, vp]),
        "hisq_dslash_shape": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int)]),
        "hisq_gauge_links_compressed": (C.c_int, [vp]),
        "hisq_rational_apply": (C.c_int, [vp, C.c_double, C.c_double, C.c_int, dp, dp, vp, vp,
                                          C.POINTER(SolverParams), C.POINTER(SolverStats), vp]),
        "hisq_rational_apply_batched": (C.c_int, [vp, C.c_double, C.c_int, C.c_double, C.c_int, dp, dp, vp, vp,
                                                  C.POINTER(SolverParams), C.POINTER(SolverStats), vp]),
        "hisq_zolotarev_inv_sqrt": (C.c_int, [C.c_double, C.c_double, C.c_int, dp, dp, dp, dp]),
        "hisq_rational_remez": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_int, dp, dp, dp, dp]),
        "hisq_spectral_bounds": (C.c_int, [vp, C.c_double, C.c_int, dp, dp, vp]),
        "hisq_smear_links": (C.c_int, [ip, vp, vp, vp, C.c_uint, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


LIB = _load()

# C ABI entry points declared in include/hisq.h (checked by the test-suite).
EXPORTS = ("hisq_version", "hisq_last_error", "hisq_spinor_bytes", "hisq_gauge_create",
           "hisq_gauge_destroy", "hisq_gauge_device_bytes", "hisq_dslash_eo", "hisq_dslash_multi_rhs",
           "hisq_solver_params_default", "hisq_cg_solve", "hisq_multishift_cg", "hisq_precond_apply",
           "hisq_autotune", "hisq_dslash_shape", "hisq_gauge_set_thin", "hisq_nn_create", "hisq_nn_destroy",
           "hisq_nn_num_weights", "hisq_nn_get_weights", "hisq_nn_set_weights", "hisq_nn_loss_grad",
           "hisq_nn_train_step", "hisq_gauge_links_compressed", "hisq_rational_apply",
           "hisq_zolotarev_inv_sqrt", "hisq_rational_remez", "hisq_spectral_bounds",
           "hisq_dslash_multi_rhs_noalloc", "hisq_smear_links", "hisq_multishift_cg_batched",
           "hisq_rational_apply_batched")

LINKS_FULL = 1 << 8  # hisq_gauge_create: store every link whole


def last_error() -> str:
    return (LIB.hisq_last_error() or b"").decode()


def _check(rc: int, allow_soft: bool = False) -> int:
    if rc < 0 or (rc > 0 and not allow_soft):
        raise HisqError(rc, last_error())
    return rc


def _prec(p) -> int:
    return PREC_NAMES[p] if isinstance(p, str) else int(p)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t) -> C.c_void_p:
    if t is None:
        return C.c_void_p(0)
    if not t.is_cuda:
        raise ValueError("device tensors are required")
    if not t.is_contiguous():
        raise ValueError("contiguous tensors are required")
    return C.c_void_p(t.data_ptr())


def _need(t, nbytes: int, what: str):
    """Raise before any launch when a buffer is smaller than what the call
    reads or writes (the C ABI sees only pointers)."""
    if t is None:
        return
    have = t.numel() * t.element_size()
    if have < nbytes:
        raise ValueError(f"{what}: {have} bytes, the call touches {nbytes}")


def version() -> int:
    return LIB.hisq_version()


def spinor_bytes(prec, vh: int) -> int:
    return int(LIB.hisq_spinor_bytes(_prec(prec), int(vh)))


def empty_spinor(prec, vh: int, nrhs: int = 1, device="cuda") -> torch.Tensor:
    """A raw device buffer of nrhs stacked spinors of the given precision."""
    return torch.empty(spinor_bytes(prec, vh) * nrhs, dtype=torch.uint8, device=device)


class Gauge:
    """Handle owning the packed link copies (see hisq_gauge_create)."""

    def __init__(self, dims, fat: torch.Tensor, lng: torch.Tensor, precs=("fp64", "fp32", "fp16s"),
                 stream=None, full_links: bool = False):
        self.dims = tuple(int(d) for d in dims)
        V = 1
        for d in self.dims:
            V *= d
        self.vh = V // 2
        for t in (fat, lng):
            if t.dtype not in (torch.complex128, torch.float64) or t.numel() * t.element_size() != V * 4 * 9 * 16:
                raise ValueError("links must be complex128 [V,4,3,3] device tensors")
        mask = 0
        for p in precs:
            mask |= 1 << _prec(p)
        if full_links:
            mask |= LINKS_FULL
        h = C.c_void_p()
        d = (C.c_int * 4)(*self.dims)
        _check(LIB.hisq_gauge_create(C.byref(h), d, _ptr(fat), _ptr(lng), mask, _stream(stream)))
        self.handle = h

    @property
    def compressed(self) -> bool:
        """True if the FP32 / FP16 long links are stored as two rows (see hisq_gauge_create)."""
        return self.comp_mode != 0

    @property
    def comp_mode(self) -> int:
        """0 long links whole, 1 two rows + determinant sign, 2 two rows + complex factor."""
        return int(_check(LIB.hisq_gauge_links_compressed(self.handle), allow_soft=True))

    def device_bytes(self) -> int:
        n = C.c_size_t()
        _check(LIB.hisq_gauge_device_bytes(self.handle, C.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "handle", None):
            LIB.hisq_gauge_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gauge_create(dims, fat, lng, precs=("fp64", "fp32", "fp16s"), stream=None) -> Gauge:
    return Gauge(dims, fat, lng, precs, stream)


def dslash_eo(g: Gauge, out_parity: int, prec, inp: torch.Tensor, out: torch.Tensor, stream=None):
    sb = spinor_bytes(prec, g.vh)
    _need(inp, sb, "in")
    _need(out, sb, "out")
    _check(LIB.hisq_dslash_eo(g.handle, int(out_parity), _prec(prec), _ptr(inp), _ptr(out), _stream(stream)))


def dslash_multi_rhs(g: Gauge, out_parity: int, prec, nrhs: int, inp, out, diag=None, y=None, stream=None):
    stack = spinor_bytes(prec, g.vh) * int(nrhs)
    for t, what in ((inp, "in"), (out, "out"), (y, "y")):
        _need(t, stack, what)
    dd = None
    if diag is not None:
        if len(diag) < nrhs:
            raise ValueError(f"diag: {len(diag)} values for {nrhs} right-hand sides")
        dd = (C.c_double * nrhs)(*[float(v) for v in diag])
    _check(LIB.hisq_dslash_multi_rhs(g.handle, int(out_parity), _prec(prec), int(nrhs), _ptr(inp), _ptr(out),
                                     dd, _ptr(y), _stream(stream)))


def dslash_multi_rhs_noalloc(g: Gauge, out_parity: int, prec, nrhs: int, inp, out, diag=None, y=None,
                             stream=None):
    """dslash_multi_rhs through the entry point that allocates no device memory."""
    stack = spinor_bytes(prec, g.vh) * int(nrhs)
    for t, what in ((inp, "in"), (out, "out"), (y, "y")):
        _need(t, stack, what)
    dd = None
    if diag is not None:
        if len(diag) < nrhs:
            raise ValueError(f"diag: {len(diag)} values for {nrhs} right-hand sides")
        dd = (C.c_double * nrhs)(*[float(v) for v in diag])
    _check(LIB.hisq_dslash_multi_rhs_noalloc(g.handle, int(out_parity), _prec(prec), int(nrhs), _ptr(inp),
                                             _ptr(out), dd, _ptr(y), _stream(stream)))


def solver_params(**kw) -> SolverParams:
    p = SolverParams()
    LIB.hisq_solver_params_default(C.byref(p))
    for k, v in kw.items():
        if k == "sloppy_prec":
            v = _prec(v)
        if k == "precond" and isinstance(v, Net):
            v = v.handle.value
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def cg_solve(g: Gauge, mass: float, nrhs: int, b, x, params: SolverParams | None = None, stream=None):
    """Returns (status, [stats dict per RHS])."""
    stack = spinor_bytes("fp64", g.vh) * int(nrhs)
    _need(b, stack, "b")
    _need(x, stack, "x")
    st = (SolverStats * nrhs)()
    rc = LIB.hisq_cg_solve(g.handle, float(mass), int(nrhs), _ptr(b), _ptr(x),
                           C.byref(params) if params is not None else None, st, _stream(stream))
    _check(rc, allow_soft=True)
    return rc, [s.as_dict() for s in st]


def multishift_cg(g: Gauge, mass: float, shifts, b, x, params: SolverParams | None = None, stream=None):
    n = len(shifts)
    sb = spinor_bytes("fp64", g.vh)
    _need(b, sb, "b")
    _need(x, sb * n, "x")
    sh = (C.c_double * n)(*[float(v) for v in shifts])
    st = (SolverStats * n)()
    rc = LIB.hisq_multishift_cg(g.handle, float(mass), n, sh, _ptr(b), _ptr(x),
                                C.byref(params) if params is not None else None, st, _stream(stream))
    _check(rc, allow_soft=True)
    return rc, [s.as_dict() for s in st]


def multishift_cg_batched(g: Gauge, mass: float, nsrc: int, shifts, b, x, params: SolverParams | None = None,
                          stream=None):
    """nsrc sources b [nsrc][spinor] with the same shifts, solved in lockstep;
    x [nsrc][nshift][spinor].  Returns (status, [stats per (source, shift)],
    source-major)."""
    n, m = len(shifts), int(nsrc)
    sb = spinor_bytes("fp64", g.vh)
    _need(b, sb * m, "b")
    _need(x, sb * n * m, "x")
    sh = (C.c_double * n)(*[float(v) for v in shifts])
    st = (SolverStats * (n * m))()
    rc = LIB.hisq_multishift_cg_batched(g.handle, float(mass), m, n, sh, _ptr(b), _ptr(x),
                                        C.byref(params) if params is not None else None, st, _stream(stream))
    _check(rc, allow_soft=True)
    return rc, [s.as_dict() for s in st]


def rational_apply_batched(g: Gauge, mass: float, nsrc: int, alpha0: float, alphas, shifts, b, out,
                           params: SolverParams | None = None, stream=None):
    """out_j = alpha0 b_j + sum_k alphas[k] (A + shifts[k])^-1 b_j for nsrc sources
    (stacks [nsrc][spinor]); returns (status, [stats per (source, term)])."""
    n, m = len(shifts), int(nsrc)
    if len(alphas) != n:
        raise ValueError("alphas and shifts differ in length")
    sb = spinor_bytes("fp64", g.vh)
    _need(b, sb * m, "b")
    _need(out, sb * m, "out")
    al = (C.c_double * max(n, 1))(*[float(v) for v in alphas])
    sh = (C.c_double * max(n, 1))(*[float(v) for v in shifts])
    st = (SolverStats * max(n * m, 1))()
    rc = LIB.hisq_rational_apply_batched(g.handle, float(mass), m, float(alpha0), n, al, sh, _ptr(b), _ptr(out),
                                         C.byref(params) if params is not None else None, st, _stream(stream))
    _check(rc, allow_soft=True)
    return rc, [s.as_dict() for s in st[:n * m]]


def rational_apply(g: Gauge, mass: float, alpha0: float, alphas, shifts, b, out,
                   params: SolverParams | None = None, stream=None):
    """out = alpha0 b + sum_k alphas[k] (A + shifts[k])^-1 b; returns (status, [stats per term])."""
    n = len(shifts)
    if len(alphas) != n:
        raise ValueError("alphas and shifts differ in length")
    sb = spinor_bytes("fp64", g.vh)
    _need(b, sb, "b")
    _need(out, sb, "out")
    al = (C.c_double * max(n, 1))(*[float(v) for v in alphas])
    sh = (C.c_double * max(n, 1))(*[float(v) for v in shifts])
    st = (SolverStats * max(n, 1))()
    rc = LIB.hisq_rational_apply(g.handle, float(mass), float(alpha0), n, al, sh, _ptr(b), _ptr(out),
                                 C.byref(params) if params is not None else None, st, _stream(stream))
    _check(rc, allow_soft=True)
    return rc, [s.as_dict() for s in st[:n]]


def zolotarev_inv_sqrt(lmin: float, lmax: float, npole: int):
    """(alpha0, alphas, shifts, delta): x^(-1/2) ~ alpha0 + sum_k alphas[k] / (x + shifts[k]) on
    [lmin, lmax] with maximal relative error delta (host only)."""
    a0, dl = C.c_double(0.0), C.c_double(0.0)
    al, sh = (C.c_double * npole)(), (C.c_double * npole)()
    _check(LIB.hisq_zolotarev_inv_sqrt(float(lmin), float(lmax), int(npole), C.byref(a0), al, sh, C.byref(dl)))
    return a0.value, list(al), list(sh), dl.value


def rational_remez(power: float, lmin: float, lmax: float, npole: int):
    """(alpha0, alphas, shifts, delta): minimax relative approximation
    x^power ~ alpha0 + sum_k alphas[k] / (x + shifts[k]) on [lmin, lmax] (host only)."""
    a0, dl = C.c_double(0.0), C.c_double(0.0)
    n = max(int(npole), 1)
    al, sh = (C.c_double * n)(), (C.c_double * n)()
    _check(LIB.hisq_rational_remez(float(power), float(lmin), float(lmax), int(npole), C.byref(a0), al, sh,
                                   C.byref(dl)))
    return a0.value, list(al), list(sh), dl.value


def spectral_bounds(g: Gauge, mass: float, iters: int = 100, stream=None):
    """(4 m^2, Rayleigh-quotient estimate of the largest eigenvalue of A)."""
    lo, hi = C.c_double(0.0), C.c_double(0.0)
    _check(LIB.hisq_spectral_bounds(g.handle, float(mass), int(iters), C.byref(lo), C.byref(hi), _stream(stream)))
    return lo.value, hi.value


def autotune(g: Gauge, prec, nrhs: int, cache_path: str | None = None, stream=None):
    """Time and install the best Dslash launch shapes for solves in `prec` with `nrhs` RHS."""
    _check(LIB.hisq_autotune(g.handle, _prec(prec), int(nrhs),
                             cache_path.encode() if cache_path else None, _stream(stream)))


def dslash_shape(g: Gauge, prec, nrhs: int, epilogue: int = 0):
    """(tile, block, order) currently used for this Dslash form."""
    out = (C.c_int * 3)()
    _check(LIB.hisq_dslash_shape(g.handle, _prec(prec), int(nrhs), int(epilogue), out))
    return tuple(out)


SMEAR_ANTIPERIODIC_T = 1


def smear_links(dims, thin, fat, lng, antiperiodic_t: bool = False, stream=None):
    """HISQ fat and Naik links (phases folded) from thin links: complex128 [V,4,3,3]
    device tensors, fat and lng written."""
    V = 1
    for d in dims:
        V *= int(d)
    for t, what in ((thin, "thin"), (fat, "fat"), (lng, "lng")):
        _need(t, V * 4 * 9 * 16, what)
    d = (C.c_int * 4)(*[int(v) for v in dims])
    _check(LIB.hisq_smear_links(d, _ptr(thin), _ptr(fat), _ptr(lng),
                                SMEAR_ANTIPERIODIC_T if antiperiodic_t else 0, _stream(stream)))


def gauge_set_thin(g: Gauge, thin: torch.Tensor, stream=None):
    """Thin links (complex128 [V,4,3,3] device tensor, phases folded) for the network."""
    _need(thin, 2 * g.vh * 4 * 9 * 16, "thin")
    _check(LIB.hisq_gauge_set_thin(g.handle, _ptr(thin), _stream(stream)))


class Net:
    """Preconditioner network (see hisq_nn_create); weights as a flat complex128 numpy array."""

    def __init__(self, g: Gauge, channels, weights=None, stream=None):
        import numpy as np
        self.channels = tuple(int(c) for c in channels)
        self.vh = g.vh
        nl = len(self.channels) - 1
        ch = (C.c_int * (nl + 1))(*self.channels)
        w = None
        if weights is not None:
            wa = np.ascontiguousarray(np.asarray(weights, np.complex128).ravel())
            w = wa.view(np.float64).ctypes.data_as(C.POINTER(C.c_double))
        h = C.c_void_p()
        _check(LIB.hisq_nn_create(C.byref(h), g.handle, nl, ch, w, _stream(stream)))
        self.handle = h
        n = C.c_size_t()
        _check(LIB.hisq_nn_num_weights(h, C.byref(n)))
        self.n = n.value

    def get_weights(self, stream=None):
        import numpy as np
        out = np.zeros(self.n, np.complex128)
        _check(LIB.hisq_nn_get_weights(self.handle, out.view(np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                                       _stream(stream)))
        return out

    def set_weights(self, weights, stream=None):
        import numpy as np
        wa = np.ascontiguousarray(np.asarray(weights, np.complex128).ravel())
        assert wa.size == self.n
        _check(LIB.hisq_nn_set_weights(self.handle, wa.view(np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                                       _stream(stream)))

    def _pairs(self, batch, av, v):
        stack = spinor_bytes("fp32", self.vh) * int(batch)
        _need(av, stack, "av")
        _need(v, stack, "v")

    def loss_grad(self, batch, av, v, want_grad=True, stream=None):
        import numpy as np
        self._pairs(batch, av, v)
        loss = C.c_double()
        grad = np.zeros(self.n, np.complex128) if want_grad else None
        gp = grad.view(np.float64).ctypes.data_as(C.POINTER(C.c_double)) if want_grad else None
        _check(LIB.hisq_nn_loss_grad(self.handle, int(batch), _ptr(av), _ptr(v), C.byref(loss), gp, _stream(stream)))
        return loss.value, grad

    def train_step(self, batch, av, v, lr, stream=None):
        self._pairs(batch, av, v)
        loss = C.c_double()
        _check(LIB.hisq_nn_train_step(self.handle, int(batch), _ptr(av), _ptr(v), float(lr), C.byref(loss),
                                      _stream(stream)))
        return loss.value

    def close(self):
        if getattr(self, "handle", None):
            LIB.hisq_nn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def precond_apply(g: Gauge, net: Net, inp, out, stream=None):
    sb = spinor_bytes("fp32", g.vh)
    _need(inp, sb, "in")
    _need(out, sb, "out")
    _check(LIB.hisq_precond_apply(g.handle, net.handle, _ptr(inp), _ptr(out), _stream(stream)))
