"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def libpath():
    from paper_1711_00336_amd import lbdem
    if not os.path.exists(lbdem.LIB_PATH):
        from paper_1711_00336_amd import build
        build.build()
    return lbdem.LIB_PATH


def test_library_loads_and_exports_header_symbols(libpath):
    from paper_1711_00336_amd import lbdem
    L = ctypes.CDLL(libpath)
    names = lbdem.exported_symbols()
    assert "lbdem_create" in names and "lbdem_step" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert set(names) <= exported


def test_params_default_and_validation_without_gpu(libpath):
    from paper_1711_00336_amd import lbdem
    P = lbdem.lbdem_params()
    assert lbdem.lib().lbdem_params_default(ctypes.byref(P)) == lbdem.OK
    assert P.n_int == 10 and abs(P.c_am - 0.5) < 1e-15 and abs(P.h_min - 1e-5) < 1e-20
    assert abs(P.e_n - 0.88) < 1e-15 and abs(P.mu_c - 0.25) < 1e-15
    # host-side validation rejects tau <= 1/2 before touching the device
    P.tau = 0.5
    h = ctypes.c_void_p()
    st = lbdem.lib().lbdem_create(ctypes.byref(P), None, ctypes.byref(h))
    assert st == lbdem.E_INVALID and not h.value
    assert b"tau" in lbdem.lib().lbdem_last_error(None)


def test_header_is_plain_c(libpath):
    """The header compiles as C99 with no C++ or HIP types."""
    src = os.path.join(ROOT, "include", "lbdem.h")
    r = subprocess.run(["gcc", "-std=c99", "-fsyntax-only", "-Wall", "-Werror", "-x", "c", src],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
