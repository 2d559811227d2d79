"""The C ABI: header compiles as plain C, the built library loads and exports every declared entry
point, and the Python binding declares them all (CPU only; no compute calls)."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ngd.h")
LIB = os.path.join(ROOT, "paper_2505_11638_amd", "libngd.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ngd_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_four_hot_path_calls():
    names = declared_functions()
    for n in ("ngd_residual_jacobian", "ngd_gramian_matvec", "ngd_nystrom_sketch", "ngd_pcg_solve"):
        assert n in names


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_header_is_plain_c99(tmp_path):
    c = tmp_path / "t.c"
    c.write_text('#include "ngd.h"\nint main(void) { ngd_pcg_info i; (void)i; return (int)NGD_OK; }\n')
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-I", os.path.dirname(HEADER), str(c)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


@pytest.mark.skipif(not os.path.exists(LIB), reason="libngd.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libngd.so not built")
def test_binding_declares_every_symbol_and_validates_on_host():
    from paper_2505_11638_amd import _lib
    assert set(declared_functions()) == set(_lib.SIGNATURES)
    lib = _lib.load()
    # argument errors are detected on the host, before any device work
    assert lib.ngd_problem_create(None, None) == _lib.NGD_ERR_INVALID
    assert b"NULL" in lib.ngd_last_error()
    assert lib.ngd_num_params(None) == -1
    h = ctypes.c_void_p()
    widths = (ctypes.c_int32 * 3)(2, 8, 2)   # output width must be 1
    desc = _lib.ProblemDesc(2, widths, 0, 1, 10, 1, 1, 1, 1, 1, 4)
    assert lib.ngd_problem_create(ctypes.byref(desc), ctypes.byref(h)) == _lib.NGD_ERR_INVALID
    assert b"output width" in lib.ngd_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libngd.so not built")
def test_navier_stokes_descriptor_checks_on_host():
    """Navier-Stokes handles (Section 5.1.3): velocity network 2 -> ... -> 2, hidden widths <= 64,
    viscosity > 0; each violation is refused before any device work."""
    from paper_2505_11638_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    ns = _lib.NGD_PDE_NAVIER_STOKES
    for widths, nu, msg in [((2, 8, 1), 0.025, b"2 outputs"), ((3, 8, 2), 0.025, b"2 inputs"),
                            ((2, 65, 2), 0.025, b"<= 64"), ((2, 8, 2), 0.0, b"viscosity"),
                            ((2, 2), 0.025, b"hidden layer")]:
        w = (ctypes.c_int32 * len(widths))(*widths)
        desc = _lib.ProblemDesc(len(widths) - 1, w, ns, 1, 10, 1, 1, 1, 1, 1, 4, nu)
        assert lib.ngd_problem_create(ctypes.byref(desc), ctypes.byref(h)) == _lib.NGD_ERR_INVALID
        assert msg in lib.ngd_last_error(), (widths, lib.ngd_last_error())
