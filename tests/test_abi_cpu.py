"""CPU-side checks of the C ABI: the shared library loads and exports every
function that include/gwl.h declares.  No GPU call is made."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gwl.h")
LIB = os.path.join(ROOT, "paper_2310_20103_amd", "_lib", "libgwl.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(gwl_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["gwl_setup", "gwl_sigma_c", "gwl_lanczos_pairs", "gwl_sigma_from_coeffs",
                     "gwl_poisson", "gwl_apply_c", "gwl_apply_d", "gwl_coupling",
                     "gwl_set_option", "gwl_query", "gwl_last_error", "gwl_destroy",
                     "gwl_default_options"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgwl.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    h = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(h, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgwl.so not built")
def test_host_only_calls():
    """Calls that touch no device: defaults, last error, null handling."""
    from paper_2310_20103_amd import binding as B
    L = B.lib()
    op = B._Options()
    L.gwl_default_options(ctypes.byref(op))
    assert op.poly_degree == 7 and op.reorth == 2 and op.precision == 0 and op.kernel_scale == 1.0
    out = ctypes.c_double()
    assert L.gwl_query(None, B.KEY_N_VC, ctypes.byref(out)) == B.GWL_EINVAL
    assert b"null context" in L.gwl_last_error()
    L.gwl_destroy(None)


def _header_enum(prefix):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return {m.group(1): int(m.group(2))
            for m in re.finditer(r"\b" + prefix + r"([A-Z0-9_]+)\s*=\s*(-?\d+)", text)}


def test_binding_constants_match_header():
    """Every option key and status code the binding names has the value the
    header gives it (ctypes passes them as plain ints)."""
    from paper_2310_20103_amd import binding as B
    keys = _header_enum("GWL_KEY_")
    bound = {n[len("KEY_"):]: v for n, v in vars(B).items()
             if n.startswith("KEY_") and isinstance(v, int)}
    assert bound, "no option keys in the binding"
    for name, value in bound.items():
        assert keys.get(name) == value, name
    for name, (ms, cnt, vec) in {"GEMM1": B.KEY_PROF["gemm1"], "GEMM2": B.KEY_PROF["gemm2"],
                                 "FFT": B.KEY_PROF["fft"]}.items():
        assert (keys["PROF_MS_" + name], keys["PROF_N_" + name], keys["PROF_VEC_" + name]) == \
            (ms, cnt, vec)
    codes = _header_enum("GWL_E")
    for name in ("INVAL", "NOMEM", "DEVICE", "NUMERIC", "STATE", "UNSUPPORTED"):
        assert getattr(B, "GWL_E" + name) == codes[name], name
    assert B.GWL_OK == 0
    prec = _header_enum("GWL_")
    assert (B.FP64, B.MIXED_F16, B.MIXED_BF16X3, B.MIXED_FP32) == (
        prec["FP64"], prec["MIXED_F16"], prec["MIXED_BF16X3"], prec["MIXED_FP32"])
    assert B.REORTH == {"none": prec["REORTH_NONE"], "local": prec["REORTH_LOCAL"],
                        "full": prec["REORTH_FULL"]}
