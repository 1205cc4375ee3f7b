"""C-ABI checks that need no GPU: the library loads, exports every function
include/lenshpc.h declares, and its host-only helpers agree with the oracle."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lenshpc.h")
LIB = os.path.join(ROOT, "paper_2004_06352_amd", "_native", "liblenshpc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lens_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} missing: run python -m paper_2004_06352_amd.build")
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("lens_grad_map", "lens_hessian_map", "lens_chi2_batch", "lens_find_images",
                 "lens_table_from_physical", "lens_ctx_create", "lens_ctx_destroy"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2004_06352_amd import binding
    assert sorted(binding.EXPORTS) == declared_functions()


def test_abi_version(lib):
    lib.lens_abi_version.restype = C.c_int32
    text = open(HEADER).read()
    v = int(re.search(r"#define LENSHPC_ABI_VERSION (\d+)", text).group(1))
    assert lib.lens_abi_version() == v


def _call_d(fn, *args):
    out = C.c_double()
    st = fn(*args, C.byref(out))
    return st, out.value


def test_host_distance_ratio_matches_oracle(lib, oracle):
    fn = lib.lens_dlsds
    fn.argtypes = [C.c_double] * 4 + [C.POINTER(C.c_double)]
    fn.restype = C.c_int32
    for zl, zs in [(0.4, 1.0), (0.4, 2.0), (0.4, 6.0), (0.1, 0.11), (0.0, 3.0)]:
        for om, ol in [(0.3, 0.7), (1.0, 0.0)]:
            st, v = _call_d(fn, zl, zs, om, ol)
            assert st == 0
            assert v == pytest.approx(oracle.dlsds(zl, zs, om, ol), rel=1e-12, abs=1e-15)
    assert _call_d(fn, 2.0, 1.0, 0.3, 0.7)[0] == -1
    assert _call_d(fn, 0.4, 2.0, 0.3, 0.6)[0] == -1
    assert _call_d(fn, 0.4, float("nan"), 0.3, 0.7)[0] == -1


def test_host_time_delay_scale_matches_oracle(lib, oracle):
    fn = lib.lens_time_delay_scale
    fn.argtypes = [C.c_double] * 5 + [C.POINTER(C.c_double)]
    fn.restype = C.c_int32
    for zl, zs in [(0.2, 1.0), (0.4, 2.0), (0.5, 6.0)]:
        for h0, om, ol in [(70.0, 0.3, 0.7), (67.0, 1.0, 0.0)]:
            v = C.c_double()
            assert fn(zl, zs, h0, om, ol, C.byref(v)) == 0
            assert v.value == pytest.approx(oracle.time_delay_scale(zl, zs, h0, om, ol), rel=1e-12)
    v = C.c_double()
    assert fn(0.0, 1.0, 70.0, 0.3, 0.7, C.byref(v)) == -1  # zl must be > 0


def test_host_parameter_conversions_match_oracle(lib, oracle):
    fb = lib.lens_b0_from_sigma
    fb.argtypes = [C.c_double, C.c_int32, C.POINTER(C.c_double)]
    fb.restype = C.c_int32
    fe = lib.lens_eps_from_e
    fe.argtypes = [C.c_double, C.POINTER(C.c_double)]
    fe.restype = C.c_int32
    for s in [0.0, 50.0, 180.0, 1000.0]:
        for conv in (0, 1):
            st, v = _call_d(fb, s, conv)
            assert st == 0 and v == pytest.approx(oracle.b0_from_sigma([s], conv)[0], rel=1e-14)
    assert _call_d(fb, -1.0, 0)[0] == -1
    assert _call_d(fb, 10.0, 2)[0] == -1
    for e in [0.0, 1e-9, 0.3, 0.5, 0.99]:
        st, v = _call_d(fe, e)
        assert st == 0 and v == pytest.approx(oracle.eps_from_e([e])[0], rel=1e-14, abs=1e-300)
    assert _call_d(fe, 1.0)[0] == -1
    assert _call_d(fe, -0.1)[0] == -1


def test_null_arguments_are_rejected_without_a_device(lib):
    lib.lens_ctx_create.argtypes = [C.c_int32, C.c_uint64, C.c_uint32, C.c_void_p]
    lib.lens_ctx_create.restype = C.c_int32
    assert lib.lens_ctx_create(0, 1 << 20, 0, None) == -1
    lib.lens_grad_map.restype = C.c_int32
    lib.lens_grad_map.argtypes = [C.c_void_p] * 3 + [C.c_double, C.c_int32] + [C.c_void_p] * 3
    assert lib.lens_grad_map(None, None, None, 1.0, 0, None, None, None) == -1
    lib.lens_last_error.restype = C.c_char_p
    assert len(lib.lens_last_error()) > 0
