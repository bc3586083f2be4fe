"""The C-ABI library loads, exports every function include/cloverqcd.h declares,
and rejects invalid arguments before any device work (runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_0910_0262_amd import capi

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "cloverqcd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qcd_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["qcd_create", "qcd_destroy", "qcd_load_gauge", "qcd_build_clover", "qcd_load_clover",
                 "qcd_apply", "qcd_solve", "qcd_action_force", "qcd_hmd_step", "qcd_last_error"]:
        assert must in names


def test_header_is_plain_c():
    """The boundary header compiles as C99 and as C++17 on its own (no GPU, no HIP types)."""
    import shutil
    import subprocess

    for compiler, std in (("gcc", "c99"), ("g++", "c++17")):
        exe = shutil.which(compiler)
        if exe is None:
            pytest.skip(f"{compiler} not found")
        lang = "c" if compiler == "gcc" else "c++"
        res = subprocess.run([exe, "-fsyntax-only", "-Wall", "-Werror", f"-std={std}", "-x", lang, HEADER],
                             capture_output=True, text=True)
        assert res.returncode == 0, res.stderr


def test_options_match_the_header():
    text = open(HEADER).read()
    for name in ("QCD_OPT_LINK_RECON", "QCD_OPT_MIXED_CLOVER", "QCD_OPT_BLOCK", "QCD_OPT_GRAPH",
                 "QCD_OPT_SMALL_GRID", "QCD_OPT_MIXED_STALL", "QCD_OPT_COMPACT_CLOVER",
                 "QCD_OPT_X_CYCLE"):
        m = re.search(rf"\b{name}\s*=\s*(\d+)", text)
        assert m and int(m.group(1)) == getattr(capi, name), name


def test_library_exports_every_declared_symbol():
    lib = capi.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in capi.SIGNATURES, name


def test_version():
    assert capi.qcd_version() >> 16 == 1


@pytest.mark.parametrize("dims", [(3, 4, 4, 4), (4, 4, 4, 5), (0, 4, 4, 4), (4, -2, 4, 4), (1, 2, 2, 2)])
def test_create_rejects_bad_shapes(dims):
    lib = capi.lib()
    out = ctypes.c_void_p(123)
    d = (ctypes.c_int * 4)(*dims)
    assert lib.qcd_create(d, 0, 0, ctypes.byref(out)) == capi.QCD_EINVAL
    assert out.value is None
    assert "even" in capi.last_error()


@pytest.mark.parametrize("dims", [(64, 64, 64, 684), (2, 2, 2, 1 << 28)])
def test_create_rejects_too_large_volume(dims):
    """V/2 (rounded up to a multiple of 64) x 48 must stay below 2^32 (the
    kernels address a binary16 spinor element with a 32-bit byte offset):
    64^3 x 684 is just past that bound; rejected before any device call."""
    vh = (dims[0] * dims[1] * dims[2] * dims[3] // 2 + 63) // 64 * 64
    assert vh * 48 >= 1 << 32
    lib = capi.lib()
    out = ctypes.c_void_p(123)
    d = (ctypes.c_int * 4)(*dims)
    assert lib.qcd_create(d, 0, 0, ctypes.byref(out)) == capi.QCD_EINVAL
    assert out.value is None
    assert "too large" in capi.last_error()


def test_null_arguments_are_rejected():
    lib = capi.lib()
    d = (ctypes.c_int * 4)(4, 4, 4, 4)
    assert lib.qcd_create(d, 0, 0, None) == capi.QCD_EINVAL
    assert lib.qcd_create(None, 0, 0, ctypes.byref(ctypes.c_void_p())) == capi.QCD_EINVAL
    assert lib.qcd_destroy(None) == capi.QCD_OK
    for fn, args in [("qcd_set_params", (None, 0.1, 1.0, -1)), ("qcd_build_clover", (None,)),
                     ("qcd_load_gauge", (None, None)), ("qcd_apply", (None, 2, 0, None, None)),
                     ("qcd_solve", (None, None, None, None, None)),
                     ("qcd_action_force", (None, None, None, None, None, None, None, None)),
                     ("qcd_hmd_step", (None, 0.1, None, None, None, None, None, None)),
                     ("qcd_encode_half", (None, 1, None, None, None)),
                     ("qcd_stream_copy", (None, None, None, 16))]:
        assert getattr(lib, fn)(*args) == capi.QCD_EINVAL, fn
        assert capi.last_error() == "null context"


def test_error_message_is_thread_local_and_stable():
    lib = capi.lib()
    d = (ctypes.c_int * 4)(4, 4, 4, 7)
    lib.qcd_create(d, 0, 0, ctypes.byref(ctypes.c_void_p()))
    msg = capi.last_error()
    assert "got 7" in msg
    err = capi.QCDError(capi.QCD_EINVAL, msg)
    assert err.status == "QCD_EINVAL" and "got 7" in str(err)
