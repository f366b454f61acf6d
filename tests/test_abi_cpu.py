"""C ABI checks that need no GPU: the library loads, exports every declared
entry point, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tdse.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tdse_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1201_6062_amd import _capi
    return _capi.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("tdse_create", "tdse_propagate", "tdse_adjoint", "tdse_destroy",
                 "tdse_group_create", "tdse_group_propagate", "tdse_tune", "tdse_hmul"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    from paper_1201_6062_amd import _capi
    names = declared_functions()
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_capi.SIGNATURES), "binding and header disagree"


def test_abi_version(lib):
    assert lib.tdse_abi_version() == 1
    assert lib.tdse_last_error() is not None


def _err(lib):
    return lib.tdse_last_error().decode()


def test_create_rejects_invalid_arguments(lib):
    h = ctypes.c_void_p()
    bogus = ctypes.c_void_p(64)
    cases = [
        ((None, bogus, bogus, 3, 50, 1, None), "out is NULL"),
        ((ctypes.byref(h), None, bogus, 3, 50, 1, None), "energies is NULL"),
        ((ctypes.byref(h), bogus, bogus, -1, 50, 1, None), "lmax"),
        ((ctypes.byref(h), bogus, bogus, 3, 0, 1, None), "n must"),
        ((ctypes.byref(h), bogus, bogus, 3, 50, 0, None), "batch"),
        ((ctypes.byref(h), bogus, None, 3, 50, 1, None), "dipole is NULL"),
        ((ctypes.byref(h), bogus, bogus, 2 ** 30, 2 ** 20, 1, None), "too large"),
    ]
    for args, frag in cases:
        assert lib.tdse_create(*args) == 1, frag
        assert frag in _err(lib)
    assert h.value is None


def test_propagate_rejects_invalid_arguments(lib):
    nul = None
    cases = [
        ((nul, 0, 0, 0.1, 10, nul, nul, nul, nul, 0, nul), "plan is NULL"),
    ]
    for args, frag in cases:
        assert lib.tdse_propagate(*args) == 1
        assert frag in _err(lib)
    # method / order / dt / nsteps / checkpoint interval, on a fake plan handle:
    # these are rejected before the handle is used
    fake = ctypes.c_void_p(16)
    for args, frag in [
        ((fake, 7, 0, 0.1, 10, nul, nul, nul, nul, 0, nul), "unknown method"),
        ((fake, 1, 0, 0.1, 10, nul, nul, nul, nul, 0, nul), "taylor_order"),
        ((fake, 1, 33, 0.1, 10, nul, nul, nul, nul, 0, nul), "taylor_order"),
        ((fake, 0, 0, 0.0, 10, nul, nul, nul, nul, 0, nul), "dt must"),
        ((fake, 0, 0, float("nan"), 10, nul, nul, nul, nul, 0, nul), "dt must"),
        ((fake, 0, 0, float("inf"), 10, nul, nul, nul, nul, 0, nul), "dt must"),
        ((fake, 0, 0, 0.1, -1, nul, nul, nul, nul, 0, nul), "nsteps"),
        ((fake, 0, 0, 0.1, 10, nul, nul, nul, ctypes.c_void_p(64), 0, nul), "ckpt_every"),
    ]:
        assert lib.tdse_propagate(*args) == 1, frag
        assert frag in _err(lib), (frag, _err(lib))


def test_stability_and_adaptive_argument_errors(lib):
    import ctypes as ct
    th, bd = ct.c_double(0.0), ct.c_double(0.0)
    assert lib.tdse_check_stability(None, 0, 0, 0.1, 0.0, ct.byref(th), ct.byref(bd)) == 1
    assert "plan is NULL" in _err(lib)
    fake = ct.c_void_p(16)  # rejected before the handle is used
    assert lib.tdse_check_stability(fake, 9, 0, 0.1, 0.0, None, None) == 1
    assert lib.tdse_check_stability(fake, 0, 0, -1.0, 0.0, None, None) == 1
    n = ct.c_int64(0)
    assert lib.tdse_propagate_adaptive(None, 1.0, 0.1, 1e-8, 1e-6, 10, None, None, None, None, None,
                                       ct.byref(n), None) == 1
    assert "plan is NULL" in _err(lib)


def test_adjoint_and_group_argument_errors(lib):
    assert lib.tdse_adjoint(None, 0, 0, 0.1, 10, None, None, None, 64, None, None, None, None) == 1
    assert "plan is NULL" in _err(lib)
    assert lib.tdse_destroy(None) == 0
    assert lib.tdse_group_destroy(None) == 0


@pytest.mark.parametrize("sanitize", [False, True])
def test_host_logic_native(tmp_path, sanitize):
    """Argument rules, the Sec. 4.1 work split, the tile order and the
    stability bounds, compiled host-only with g++; once plain and once under
    AddressSanitizer and UndefinedBehaviorSanitizer."""
    import subprocess
    csrc = os.path.join(ROOT, "paper_1201_6062_amd", "csrc")
    exe = str(tmp_path / "host_logic")
    flags = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"] \
        if sanitize else []
    subprocess.check_call(["g++", "-std=c++17", "-O1", *flags, "-I", csrc, "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "native", "host_logic.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
