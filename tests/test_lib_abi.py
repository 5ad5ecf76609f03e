"""CPU checks of the C-ABI library: it loads and exports every symbol the
header declares; host-side argument checks need no GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pi.h")
LIB = os.path.join(ROOT, "paper_2406_16091_amd", "libpi.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pi_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("pi_bin", "pi_interact", "pi_ctx_create", "pi_sync"):
        assert must in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libpi.so is not built (run __graft_entry__.build())")
    import torch  # noqa: F401  (the binding shares torch's HIP runtime)
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"declared in pi.h but not exported: {missing}"


def test_binding_covers_every_declared_symbol():
    from paper_2406_16091_amd import pi
    assert sorted(pi.EXPORTS) == declared_functions()


def test_status_strings(lib):
    lib.pi_status_str.restype = ctypes.c_char_p
    lib.pi_status_str.argtypes = [ctypes.c_int32]
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        s = lib.pi_status_str(code).decode()
        assert s.startswith("PI_")
    assert lib.pi_status_str(123).decode() == "unknown pi_status"


def test_null_argument_checks_need_no_device(lib):
    P = ctypes.c_void_p
    lib.pi_ctx_create.argtypes = [ctypes.c_int32, ctypes.POINTER(P)]
    lib.pi_ctx_create.restype = ctypes.c_int32
    assert lib.pi_ctx_create(0, None) == -1
    lib.pi_bin.restype = ctypes.c_int32
    lib.pi_bin.argtypes = [P, P, P, P, P, P, ctypes.c_int64, P, P]
    assert lib.pi_bin(None, None, None, None, None, None, 0, None, None) == -1
    lib.pi_interact.restype = ctypes.c_int32
    lib.pi_interact.argtypes = [P] * 10
    assert lib.pi_interact(*([None] * 10)) == -1
    lib.pi_ctx_destroy.restype = ctypes.c_int32
    lib.pi_ctx_destroy.argtypes = [P]
    assert lib.pi_ctx_destroy(None) == -1
