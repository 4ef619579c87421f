"""CPU-side checks of the C ABI: the built library loads, exports every symbol
that include/ntd.h declares, and rejects invalid arguments before touching the
GPU.  No kernel is launched here."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ntd.h")
LIB = os.path.join(ROOT, "paper_1909_09771_amd", "libntd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ntd_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        import paper_1909_09771_amd.build as b
        b.build()
    lib = ctypes.CDLL(LIB)
    lib.ntd_workspace_bytes.restype = ctypes.c_size_t
    lib.ntd_workspace_bytes.argtypes = [ctypes.c_int] * 5
    lib.ntd_strerror.restype = ctypes.c_char_p
    P = ctypes.c_void_p
    lib.ntd_setup.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int,
                              ctypes.c_int, ctypes.c_int, P, ctypes.c_size_t, P, ctypes.POINTER(P)]
    return lib


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ntd_setup", "ntd_apply_precond", "ntd_spmv", "ntd_pcg_solve", "ntd_dot",
                     "ntd_destroy", "ntd_workspace_bytes", "ntd_strerror"):
        assert required in names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_workspace_bytes(L):
    assert L.ntd_workspace_bytes(0, 4, 4, 0, 0) == 0
    assert L.ntd_workspace_bytes(4, 4, 4, 7, 0) == 0
    assert L.ntd_workspace_bytes(4, 4, 4, 0, 5) == 0
    assert L.ntd_workspace_bytes(2048, 1, 1, 0, 0) == 0       # beyond the longest line
    a = L.ntd_workspace_bytes(32, 32, 32, 0, 0)
    b = L.ntd_workspace_bytes(32, 32, 32, 1, 0)
    c = L.ntd_workspace_bytes(32, 32, 32, 1, 1)
    assert a > 14 * 8 * 32 ** 3 and b > 14 * 8 * 32 ** 3       # 14 FP64 vectors + packed factors
    assert b < a                                               # packed factors in float
    assert c >= b + 4 * 8 * 32 ** 3                            # ILU(0) diagonal, inverse, 2 vectors
    assert L.ntd_workspace_bytes(1024, 2, 2, 1, 0) > 0


def test_strerror(L):
    for code in range(7):
        assert len(L.ntd_strerror(code)) > 0
    assert L.ntd_strerror(99) == b"unknown status"


@pytest.mark.parametrize("bc,size", [((1, 1, 1, 1, 1, 1), 4),   # all Neumann: singular
                                     ((0, 2, 0, 0, 0, 0), 4),   # bad face type
                                     ((0, 0, 0, 0, 0, 0), 0)])  # bad size
def test_setup_rejects_invalid_arguments_without_gpu(L, bc, size):
    out = ctypes.c_void_p(123)
    bc_arr = (ctypes.c_int * 6)(*bc)
    fake = ctypes.c_void_p(4096)  # never dereferenced: validation fails first
    st = L.ntd_setup(size, 4, 4, fake, bc_arr, None, 0, 0, 0, fake, 1 << 30, None, ctypes.byref(out))
    assert st == 1 and out.value is None


def test_setup_rejects_small_or_misaligned_workspace(L):
    out = ctypes.c_void_p()
    bc_arr = (ctypes.c_int * 6)(0, 0, 0, 0, 0, 0)
    fake = ctypes.c_void_p(4096)
    need = L.ntd_workspace_bytes(8, 8, 8, 0, 0)
    assert L.ntd_setup(8, 8, 8, fake, bc_arr, None, 0, 0, 0, fake, need - 1, None, ctypes.byref(out)) == 1
    assert L.ntd_setup(8, 8, 8, fake, bc_arr, None, 0, 0, 0, ctypes.c_void_p(4096 + 8), need, None,
                       ctypes.byref(out)) == 1
    assert L.ntd_setup(8, 8, 8, fake, bc_arr, None, 0, 5, 0, fake, need, None, ctypes.byref(out)) == 1
    assert L.ntd_setup(8, 8, 8, fake, bc_arr, None, 0, 0, 3, fake, need, None, ctypes.byref(out)) == 1
