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


def _dims(*sizes):
    flat = [v for s in sizes for v in s]
    return (ctypes.c_int * len(flat))(*flat)


def test_batch_workspace_bytes(L):
    f = L.ntd_batch_workspace_bytes
    f.restype = ctypes.c_size_t
    f.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int]
    two = _dims((32, 32, 32), (40, 36, 20))
    assert f(0, two, 1, 1) == 0                      # no systems
    assert f(2, two, 0, 1) == 0                      # no right-hand side
    assert f(2, two, 17, 1) == 0                     # beyond NTD_BATCH_MAX_RHS
    assert f(2, two, 1, 9) == 0                      # bad precision
    assert f(1, _dims((513, 2, 2)), 1, 1) == 0       # beyond NTD_BATCH_MAX_NX
    assert f(1, _dims((0, 2, 2)), 1, 1) == 0
    one, four = f(2, two, 1, 1), f(2, two, 4, 1)
    n = 32 ** 3 + 40 * 36 * 20
    assert one > 0 and four >= one + 3 * 4 * 8 * n   # r, z, p, q per extra right-hand side
    assert f(2, two, 1, 0) > one                     # FP64 records and packed vectors


def test_batch_setup_rejects_invalid_arguments_without_gpu(L):
    P = ctypes.c_void_p
    s = L.ntd_batch_setup
    s.restype = ctypes.c_int
    s.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(P),
                  ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int, ctypes.c_int, P,
                  ctypes.c_size_t, P, ctypes.POINTER(P)]
    L.ntd_batch_workspace_bytes.restype = ctypes.c_size_t
    L.ntd_batch_workspace_bytes.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                            ctypes.c_int, ctypes.c_int]
    dims = _dims((8, 8, 8), (12, 6, 4))
    need = L.ntd_batch_workspace_bytes(2, dims, 2, 1)
    kap = (P * 2)(4096, 8192)  # never dereferenced: validation fails first
    bc = (ctypes.c_int * 12)(*([0] * 12))
    ws = P(1 << 20)
    out = P(123)
    assert s(2, dims, kap, bc, 2, 1, 0, ws, need - 1, None, ctypes.byref(out)) == 1
    assert out.value is None
    assert s(2, dims, kap, bc, 2, 1, 0, P((1 << 20) + 8), need, None, ctypes.byref(out)) == 1
    assert s(2, dims, kap, bc, 2, 1, 7, ws, need, None, ctypes.byref(out)) == 1       # schur
    assert s(2, dims, (P * 2)(4096, None), bc, 2, 1, 0, ws, need, None, ctypes.byref(out)) == 1
    assert s(2, dims, kap, bc, 0, 1, 0, ws, need, None, ctypes.byref(out)) == 1       # nrhs
    for name in ("ntd_batch_apply", "ntd_batch_pcg_solve", "ntd_batch_apply_profile"):
        getattr(L, name).restype = ctypes.c_int
    L.ntd_batch_apply.argtypes = [P, P, P, P]
    assert L.ntd_batch_apply(None, None, None, None) == 1


def test_cnn_validation_before_any_launch(L):
    P, I, Z = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    L.ntd_cnn_workspace_bytes.restype = Z
    L.ntd_cnn_workspace_bytes.argtypes = [I, I, I]
    assert L.ntd_cnn_workspace_bytes(0, 4, 4) == 0
    assert L.ntd_cnn_workspace_bytes(1024, 1024, 512) == 0         # beyond 2^28 voxels
    n = 32 ** 3
    assert L.ntd_cnn_workspace_bytes(32, 32, 32) >= 168 * n
    L.ntd_cnn_predict.argtypes = [I, I, I, P, P, P, P, P, Z, P]
    L.ntd_cnn_predict.restype = I
    assert L.ntd_cnn_predict(4, 4, 4, None, None, None, None, None, 0, None) == 1
    L.ntd_cnn_loss_grad.argtypes = [I, I, I, P, P, P, P, P, P, Z, P]
    L.ntd_cnn_loss_grad.restype = I
    assert L.ntd_cnn_loss_grad(0, 4, 4, None, None, None, None, None, None, 0, None) == 1
    L.ntd_cnn_adam.argtypes = [P, P, P, P, I, ctypes.c_float, P]
    L.ntd_cnn_adam.restype = I
    buf = ctypes.create_string_buffer(16)
    assert L.ntd_cnn_adam(buf, buf, buf, buf, 0, 0.01, None) == 1     # step counts from 1
    assert L.ntd_cnn_adam(buf, buf, buf, buf, 1, -1.0, None) == 1     # lr > 0


def test_symmetric_smoother_workspace(L):
    n = 16
    none_ = L.ntd_workspace_bytes(n, n, n, 1, 0)
    ilu = L.ntd_workspace_bytes(n, n, n, 1, 1)
    sym = L.ntd_workspace_bytes(n, n, n, 1, 2)
    assert sym == ilu > none_                 # same ILU(0) arrays, tv used as the third stage's residual
    assert L.ntd_workspace_bytes(n, n, n, 1, 3) == 0


@pytest.mark.parametrize("prec,smoother", [(0, 0), (1, 0), (1, 1), (1, 2)])
def test_storage_is_linear_in_the_unknowns(L, prec, smoother):
    """The factorization and its workspace take O(N) storage (Sec. 2.3).  At a
    fixed line length, doubling the number of planes doubles the bytes (fixed
    tables aside).  Over cubes the bytes per unknown never grow: each line
    record also holds a fixed per-lane part (scan multipliers, twist row), an
    O(N / nx) term."""
    a = L.ntd_workspace_bytes(128, 128, 64, prec, smoother)
    b = L.ntd_workspace_bytes(128, 128, 128, prec, smoother)
    c = L.ntd_workspace_bytes(128, 128, 256, prec, smoother)
    assert abs(b / a - 2.0) <= 0.01 and abs(c / b - 2.0) <= 0.01
    per = [L.ntd_workspace_bytes(n, n, n, prec, smoother) / n ** 3 for n in (32, 64, 128, 256)]
    assert all(x >= y for x, y in zip(per, per[1:])) and per[-1] <= 260


def test_dot_noalloc_rejects_bad_arguments_on_the_host(L):
    """Argument checks happen before any HIP call, so they run without a GPU."""
    P = ctypes.c_void_p
    L.ntd_dot_noalloc.argtypes = [P, P, ctypes.c_longlong, P, P]
    L.ntd_dot_noalloc.restype = ctypes.c_int
    buf = ctypes.create_string_buffer(64)
    p = ctypes.cast(buf, P)
    assert L.ntd_dot_noalloc(None, p, 4, p, None) == 1
    assert L.ntd_dot_noalloc(p, None, 4, p, None) == 1
    assert L.ntd_dot_noalloc(p, p, 4, None, None) == 1
    assert L.ntd_dot_noalloc(p, p, -1, p, None) == 1
    assert L.ntd_dot_noalloc(p, p, (1 << 50) + 1, p, None) == 1
