"""Host-only checks of the C ABI: the library loads, exports every function
include/hisq.h declares, and rejects bad arguments before touching the GPU."""

import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hisq.h")
LIB = os.path.join(ROOT, "paper_2111_10354_amd", "libhisq.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hisq_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libhisq.so is not built (run __graft_entry__.build())")
    return C.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "hisq_dslash_eo" in names and "hisq_cg_solve" in names
    for required in ("hisq_dslash_eo", "hisq_dslash_multi_rhs", "hisq_cg_solve", "hisq_multishift_cg",
                     "hisq_precond_apply"):
        assert required in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_export():
    from paper_2111_10354_amd import hisq
    assert set(hisq.EXPORTS) == set(declared_functions())
    for n in declared_functions():
        assert hasattr(hisq.LIB, n)


def test_library_version_matches_the_header(lib):
    text = open(HEADER).read()
    want = int(re.search(r"#define HISQ_VERSION (\d+)", text).group(1))
    assert lib.hisq_version() == want


def test_spinor_bytes(lib):
    f = lib.hisq_spinor_bytes
    f.restype = C.c_size_t
    f.argtypes = [C.c_int, C.c_int64]
    assert f(0, 10) == 480 and f(1, 10) == 240 and f(2, 10) == 160
    assert f(7, 10) == 0


def test_params_default(lib):
    from paper_2111_10354_amd import hisq
    p = hisq.solver_params()
    assert p.tol == 1e-10 and p.max_iter == 100000 and p.ru_period == 100
    assert p.sloppy_prec == hisq.PREC_FP64 and p.fallback == 1 and p.ru_delta == 0.1


def test_invalid_arguments_rejected_without_gpu():
    from paper_2111_10354_amd import hisq
    L = hisq.LIB
    h = C.c_void_p()
    dummy = C.c_void_p(0x1000)
    for dims in [(4, 4, 5, 4), (2, 4, 4, 4), (4, 4, 4, 0)]:
        d = (C.c_int * 4)(*dims)
        assert L.hisq_gauge_create(C.byref(h), d, dummy, dummy, 7, None) == hisq.ERR_INVALID
    d = (C.c_int * 4)(4, 4, 4, 4)
    assert L.hisq_gauge_create(C.byref(h), d, None, dummy, 7, None) == hisq.ERR_INVALID
    assert L.hisq_gauge_create(C.byref(h), d, dummy, dummy, 0, None) == hisq.ERR_INVALID
    assert L.hisq_gauge_create(C.byref(h), d, dummy, dummy, 8, None) == hisq.ERR_INVALID
    big = (C.c_int * 4)(1024, 1024, 1024, 4)
    assert L.hisq_gauge_create(C.byref(h), big, dummy, dummy, 1, None) == hisq.ERR_INVALID
    assert "2^31" in hisq.last_error()
    assert L.hisq_dslash_eo(None, 0, 0, dummy, dummy, None) == hisq.ERR_INVALID
    assert L.hisq_dslash_multi_rhs(None, 0, 0, 1, dummy, dummy, None, None, None) == hisq.ERR_INVALID
    assert L.hisq_cg_solve(None, 0.1, 1, dummy, dummy, None, None, None) == hisq.ERR_INVALID
    assert L.hisq_precond_apply(None, None, dummy, dummy, None) == hisq.ERR_INVALID
    a0 = C.c_double()
    al, sh = (C.c_double * 4)(), (C.c_double * 4)()
    assert L.hisq_rational_remez(0.25, 1e-3, 1.0, 4, None, al, sh, None) == hisq.ERR_INVALID
    assert L.hisq_rational_remez(0.0, 1e-3, 1.0, 4, C.byref(a0), al, sh, None) == hisq.ERR_INVALID
    assert L.hisq_rational_remez(0.25, 1e-3, 1.0, 4, C.byref(a0), al, al, None) == hisq.ERR_INVALID
    assert "overlap" in hisq.last_error()
    assert L.hisq_zolotarev_inv_sqrt(1e-3, 1.0, 4, C.byref(a0), None, sh, None) == hisq.ERR_INVALID
    assert L.hisq_zolotarev_inv_sqrt(1e-3, 1.0, 4, C.byref(a0), al, al, None) == hisq.ERR_INVALID
    assert L.hisq_rational_remez(0.25, 1e-3, 1.0, 4, C.byref(a0), al, sh, None) == hisq.OK
    assert L.hisq_gauge_destroy(None) == hisq.OK


def test_header_layout_constants_match_binding():
    from paper_2111_10354_amd import hisq
    text = open(HEADER).read()
    consts = dict(re.findall(r"#define (HISQ_[A-Z0-9_]+) (-?\d+)\b", text))
    assert int(consts["HISQ_PREC_FP64"]) == hisq.PREC_FP64
    assert int(consts["HISQ_PREC_FP32"]) == hisq.PREC_FP32
    assert int(consts["HISQ_PREC_FP16S"]) == hisq.PREC_FP16S
    assert int(consts["HISQ_ERR_INVALID"]) == hisq.ERR_INVALID
    assert int(consts["HISQ_NOT_CONVERGED"]) == hisq.NOT_CONVERGED


@pytest.mark.parametrize("struct,cls", [("hisq_solver_params", "SolverParams"),
                                        ("hisq_solver_stats", "SolverStats")])
def test_struct_layout_matches_the_c_compiler(tmp_path, struct, cls):
    """The ctypes mirrors of the host structs have the size and field offsets that
    a C compiler gives the header's declarations."""
    import shutil
    import subprocess
    from paper_2111_10354_amd import hisq
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    py = getattr(hisq, cls)
    names = [f for f, _ in py._fields_]
    src = tmp_path / "layout.c"
    body = "".join(f'    printf("%zu\\n", offsetof({struct}, {n}));\n' for n in names)
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"hisq.h\"\n"
                   f"int main(void) {{\n    printf(\"%zu\\n\", sizeof({struct}));\n{body}    return 0;\n}}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got[0] == C.sizeof(py)
    assert got[1:] == [getattr(py, n).offset for n in names]


def test_layout_helpers_roundtrip():
    import sys
    sys.path.insert(0, os.path.dirname(__file__))
    import layout
    import synth
    dims = (4, 6, 4, 4)
    v = synth.gaussian_source(dims, 99, 1, parity=1)[0]
    cb = layout.to_cb(dims, v, 1)
    assert np.array_equal(layout.from_cb(dims, cb, 1), v)
    vh = cb.shape[1]
    for prec, tol in (("fp64", 0), ("fp32", 1e-7), ("fp16s", 2 ** -11)):
        back = layout.decode(layout.encode(cb, prec), vh, prec)
        err = np.abs(back - cb)
        scale = np.maximum(np.abs(cb.real), np.abs(cb.imag)).max(axis=0)
        assert np.all(err <= tol * scale[None, :] * 1.5 + 1e-300)


def test_misaligned_spinors_rejected_before_any_gpu_work():
    from paper_2111_10354_amd import hisq
    fake_handle = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    rc = hisq.LIB.hisq_dslash_eo(fake_handle, 0, 1, C.c_void_p(0x10008), C.c_void_p(0x20000), None)
    assert rc == hisq.ERR_INVALID and "aligned" in hisq.last_error()


def test_no_bit_cast_of_vector_elements_in_device_code():
    """hipcc (ROCm 7.2) compiles __builtin_bit_cast(T, v.w) / (T, v[i]) of an
    ext_vector element as if it read element 0; the kernels bind the element to
    a scalar first.  Guard against the pattern coming back."""
    import glob
    pat = re.compile(r"__builtin_bit_cast\(\s*[\w ]+,\s*[\w]+(\.[xyzw]\b|\[)")
    bad = []
    for path in glob.glob(os.path.join(ROOT, "paper_2111_10354_amd", "csrc", "*")):
        for i, line in enumerate(open(path), 1):
            if pat.search(line):
                bad.append(f"{os.path.basename(path)}:{i}: {line.strip()}")
    assert not bad, bad


def test_bench_traffic_is_keyed_on_sources_layout_and_shape():
    """The counter traffic that bench.py reports belongs to one kernel source
    hash, link layout and launch shape; any other combination reports None."""
    import json
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "dslash_fp32_96x96x96x24.traffic.json")))
    dims = (96, 96, 96, 24)
    shape = tuple(rec["launch_shape"])
    got = bench.counter_traffic(dims, rec["long_links_compressed"], shape)
    import hashlib
    csrc = os.path.join(ROOT, "paper_2111_10354_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, n), "rb").read() for n in ("dslash.hip", "hisq_internal.h", "pack.hip"))
    if hashlib.sha256(src).hexdigest() == rec["kernel_sources_sha256"]:
        assert got == pytest.approx(rec["traffic_bytes_per_launch"] / 1e9)
    else:  # kernel changed since the counters were taken: no traffic claimed
        assert got is None
    assert bench.counter_traffic(dims, rec["long_links_compressed"], (shape[0], shape[1], shape[2] + 1)) is None
    assert bench.counter_traffic(dims, not rec["long_links_compressed"], shape) is None
    assert bench.counter_traffic((48, 48, 48, 12), False, shape) is None


def test_coefficient_scalar_outputs_must_not_alias_the_arrays():
    """alpha0 and delta are written before (and read back after) the arrays:
    any of them inside alpha or shift, or delta on alpha0, is refused."""
    from paper_2111_10354_amd import hisq
    L = hisq.LIB
    n = 4
    for fn, args in ((L.hisq_zolotarev_inv_sqrt, (1e-3, 1.0)), (L.hisq_rational_remez, (0.25, 1e-3, 1.0))):
        al, sh = (C.c_double * n)(), (C.c_double * n)()
        a0, dl = C.c_double(), C.c_double()
        elem = lambda arr, i: C.cast(C.byref(arr, 8 * i), C.POINTER(C.c_double))  # noqa: E731
        for bad in ((elem(al, 2), al, sh, C.byref(dl)),      # alpha0 inside alpha
                    (elem(sh, 0), al, sh, C.byref(dl)),      # alpha0 inside shift
                    (C.byref(a0), al, sh, elem(al, 3)),      # delta inside alpha
                    (C.byref(a0), al, sh, elem(sh, 1)),      # delta inside shift
                    (C.byref(a0), al, sh, C.byref(a0))):     # delta on alpha0
            assert fn(*args, n, *bad) == hisq.ERR_INVALID
            assert "overlap" in hisq.last_error()
        assert fn(*args, n, C.byref(a0), al, sh, C.byref(dl)) == hisq.OK
        assert dl.value > 0 and all(v > 0 for v in sh)
        # neighbours in one buffer are not overlaps: delta | alpha[n] | alpha0 | shift[n]
        buf = (C.c_double * (2 * n + 2))()
        assert fn(*args, n, elem(buf, n + 1), elem(buf, 1), elem(buf, n + 2), elem(buf, 0)) == hisq.OK, \
            hisq.last_error()
        assert buf[0] == pytest.approx(dl.value) and list(buf[n + 2:]) == pytest.approx(list(sh))


def test_binding_rejects_undersized_buffers_before_any_call():
    """The C ABI sees only pointers: the binding compares every buffer with the
    bytes the call touches and raises before anything reaches the library (the
    handle here is a stand-in that the library never sees)."""
    import torch
    from paper_2111_10354_amd import hisq
    g = hisq.Gauge.__new__(hisq.Gauge)
    g.dims, g.vh, g.handle = (8, 8, 8, 8), 2048, None
    one32 = torch.empty(hisq.spinor_bytes("fp32", g.vh), dtype=torch.uint8)
    one64 = torch.empty(hisq.spinor_bytes("fp64", g.vh), dtype=torch.uint8)
    short = one32[:-16]
    calls = [
        lambda: hisq.dslash_eo(g, 0, "fp32", short, one32),
        lambda: hisq.dslash_eo(g, 0, "fp32", one32, short),
        lambda: hisq.dslash_eo(g, 0, "fp64", one32, one64),           # fp32-sized input for fp64
        lambda: hisq.dslash_multi_rhs(g, 0, "fp32", 4, one32, one32),  # a 1-RHS buffer with nrhs = 4
        lambda: hisq.dslash_multi_rhs(g, 0, "fp32", 1, one32, one32, diag=[1.0], y=short),
        lambda: hisq.cg_solve(g, 0.1, 2, one64, one64),
        lambda: hisq.multishift_cg(g, 0.1, [0.0, 0.1], one64, one64),  # x holds one of two shifts
        lambda: hisq.rational_apply(g, 0.1, 1.0, [1.0], [0.1], one32, one64),
        lambda: hisq.precond_apply(g, None, one32[:-8], one32),
        lambda: hisq.gauge_set_thin(g, one64),
        lambda: hisq.multishift_cg_batched(g, 0.1, 2, [0.0, 0.1], one64, one64),   # b holds one of two sources
        lambda: hisq.multishift_cg_batched(g, 0.1, 1, [0.0, 0.1], one64, one64),   # x holds one of two shifts
        lambda: hisq.rational_apply_batched(g, 0.1, 2, 1.0, [1.0], [0.1], one64, one64),
    ]
    # CPU tensors: the size check must fire before the device check would
    for i, call in enumerate(calls):
        with pytest.raises(ValueError, match="the call touches"):
            call()


def test_c_abi_check_program_builds(tmp_path):
    """tests/capi_c_check.cpp (run on the GPU by test_gpu_capi_c.py) compiles
    and links against the library and the C oracle from the header alone."""
    import shutil
    import sys
    if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not available")
    sys.path.insert(0, ROOT)
    import __graft_entry__ as entry
    exe = entry.build_capi_check(str(tmp_path / "capi_c_check"))
    assert os.path.exists(exe)
