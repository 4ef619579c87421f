"""FP64 CPU oracle of the nested twisted filtering preconditioner (arXiv:1909.09771).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg use this package; the GPU library never imports, links or runs
it, and the two share no code.  The arithmetic lives in `ntd_oracle.c` (plain
C99, single thread, built with -ffp-contract=off); this module only marshals
numpy arrays into it.

Arrays are C-contiguous float64 numpy arrays of shape (nz, ny, nx) (x fastest).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ntd_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None

OK, EINVAL, ENOMEM, ENOTSPD, EBREAKDOWN, ENOCONV = 0, 1, 2, 3, 4, 5
MODES = {"newton": 0, "paper_literal": 1, "diag": 2}


def build(force: bool = True) -> str:
    """Compile liborc.so next to its source (gcc -O3 for x86-64-v3, i.e. AVX2,
    which every host here has; no FP contraction, so no FMA is formed)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-std=c99", "-ffp-contract=off",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i, d, l = ctypes.c_int, ctypes.c_double, ctypes.c_long
        lib.orc_assemble.argtypes = [i, i, i, P, P, P, P, P, P]
        lib.orc_assemble.restype = i
        lib.orc_spmv.argtypes = [i, i, i, P, P, P, P, P, P]
        lib.orc_spmv.restype = None
        lib.orc_dot.argtypes = [l, P, P]
        lib.orc_dot.restype = d
        lib.orc_setup.argtypes = [i, i, i, P, P, P, P, P, i, P, P, P, P, P, P]
        lib.orc_setup.restype = i
        lib.orc_apply.argtypes = [i, i, i, P, P, P, P, P, P]
        lib.orc_apply.restype = i
        lib.orc_plane_solve.argtypes = [i, i, i, P, P, P, i, P, P]
        lib.orc_plane_solve.restype = i
        lib.orc_line_solve.argtypes = [i, P, P, P, P]
        lib.orc_line_solve.restype = None
        lib.orc_line_pivots.argtypes = [i, P, P, P]
        lib.orc_line_pivots.restype = i
        lib.orc_pcg.argtypes = [i, i, i, P, P, P, P, P, P, P, P, i, P, P, d, i,
                                ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double), P]
        lib.orc_pcg_combo.argtypes = [i, i, i, P, P, P, P, P, P, P, P, i, i, P, P, d, i,
                                      ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_double), P]
        lib.orc_pcg_combo.restype = i
        lib.orc_sym_combo_apply.argtypes = [i, i, i, P, P, P, P, P, P, P, P, i, P, P]
        lib.orc_sym_combo_apply.restype = i
        lib.orc_ilu0.argtypes = [i, i, i, P, P, P, P, i, P]
        lib.orc_ilu0.restype = i
        lib.orc_ilu0_apply.argtypes = [i, i, i, P, P, P, P, i, P, P]
        lib.orc_ilu0_apply.restype = None
        lib.orc_combo_apply.argtypes = [i, i, i, P, P, P, P, P, P, P, P, i, P, P]
        lib.orc_combo_apply.restype = i
        lib.orc_pcg.restype = i
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__("%s failed with status %d" % (what, status))
        self.status = status


def assemble(kappa, bc):
    """Bands (d, ax, ay, az) of the 7-point matrix A for kappa of shape (nz, ny, nx)."""
    kappa = _f64(kappa)
    nz, ny, nx = kappa.shape
    bc = np.ascontiguousarray(bc, dtype=np.int32)
    out = [np.empty_like(kappa) for _ in range(4)]
    st = _L().orc_assemble(nx, ny, nz, _ptr(kappa), _ptr(bc), *[_ptr(a) for a in out])
    if st != OK:
        raise OracleError(st, "orc_assemble")
    return tuple(out)


def spmv(bands, x):
    d, ax, ay, az = [_f64(a) for a in bands]
    nz, ny, nx = d.shape
    x = _f64(x).reshape(d.shape)
    y = np.empty_like(d)
    _L().orc_spmv(nx, ny, nz, _ptr(d), _ptr(ax), _ptr(ay), _ptr(az), _ptr(x), _ptr(y))
    return y


def dot(x, y):
    x, y = _f64(x).ravel(), _f64(y).ravel()
    return float(_L().orc_dot(x.size, _ptr(x), _ptr(y)))


def setup(bands, t=None, mode="newton", raise_on_error=True):
    """Factor B.  Returns dict with e1, M (pivots), f2, g3 (= az), dT, dP, xP and status."""
    d, ax, ay, az = [_f64(a) for a in bands]
    nz, ny, nx = d.shape
    tt = None if t is None else _f64(t).reshape(d.shape)
    outs = {k: np.empty_like(d) for k in ("e1", "M", "f2", "dT", "dP", "xP")}
    st = _L().orc_setup(nx, ny, nz, _ptr(d), _ptr(ax), _ptr(ay), _ptr(az), _ptr(tt), MODES[mode],
                        _ptr(outs["e1"]), _ptr(outs["M"]), _ptr(outs["f2"]),
                        _ptr(outs["dT"]), _ptr(outs["dP"]), _ptr(outs["xP"]))
    if st != OK and raise_on_error:
        raise OracleError(st, "orc_setup")
    outs["g3"] = az
    outs["status"] = st
    return outs


def apply(F, r):
    """z = B^{-1} r with the factors F returned by setup()."""
    e1 = F["e1"]
    nz, ny, nx = e1.shape
    r = _f64(r).reshape(e1.shape)
    z = np.empty_like(e1)
    st = _L().orc_apply(nx, ny, nz, _ptr(e1), _ptr(F["M"]), _ptr(F["f2"]), _ptr(F["g3"]),
                        _ptr(r), _ptr(z))
    if st != OK:
        raise OracleError(st, "orc_apply")
    return z


def plane_solve(F, k, y):
    """x = Pt_k^{-1} y (level-2 solve with plane k's factors); y has shape (ny, nx)."""
    e1 = F["e1"]
    nz, ny, nx = e1.shape
    y = _f64(y).reshape(ny, nx)
    x = np.empty_like(y)
    st = _L().orc_plane_solve(nx, ny, nz, _ptr(e1), _ptr(F["M"]), _ptr(F["f2"]), int(k),
                              _ptr(y), _ptr(x))
    if st != OK:
        raise OracleError(st, "orc_plane_solve")
    return x


def line_pivots(d, e):
    d, e = _f64(d), _f64(e)
    M = np.empty_like(d)
    st = _L().orc_line_pivots(d.size, _ptr(d), _ptr(e), _ptr(M))
    return M, st


def line_solve(e, M, y):
    e, M, y = _f64(e), _f64(M), _f64(y)
    x = np.empty_like(y)
    _L().orc_line_solve(y.size, _ptr(e), _ptr(M), _ptr(y), _ptr(x))
    return x


def ilu0(bands, nblocks=2, raise_on_error=True):
    """Diagonal dt of ILU(0) of blkD(A) (nblocks = 2, split at M = floor(N/2)) or of A."""
    d, ax, ay, az = [_f64(a) for a in bands]
    nz, ny, nx = d.shape
    dt = np.empty_like(d)
    st = _L().orc_ilu0(nx, ny, nz, _ptr(d), _ptr(ax), _ptr(ay), _ptr(az), int(nblocks), _ptr(dt))
    if st != OK and raise_on_error:
        raise OracleError(st, "orc_ilu0")
    return dt, st


def ilu0_apply(bands, dt, r, nblocks=2):
    d, ax, ay, az = [_f64(a) for a in bands]
    nz, ny, nx = d.shape
    r = _f64(r).reshape(d.shape)
    z = np.empty_like(d)
    _L().orc_ilu0_apply(nx, ny, nz, _ptr(ax), _ptr(ay), _ptr(az), _ptr(_f64(dt)), int(nblocks),
                        _ptr(r), _ptr(z))
    return z


def combo_apply(bands, F, dt, r, nblocks=2):
    """z = B^{-1} r + B_ILU^{-1} r - B^{-1} A B_ILU^{-1} r (eq. com)."""
    d, ax, ay, az = [_f64(a) for a in bands]
    nz, ny, nx = d.shape
    r = _f64(r).reshape(d.shape)
    z = np.empty_like(d)
    st = _L().orc_combo_apply(nx, ny, nz, _ptr(d), _ptr(ax), _ptr(ay), _ptr(az), _ptr(F["e1"]),
                              _ptr(F["M"]), _ptr(F["f2"]), _ptr(_f64(dt)), int(nblocks), _ptr(r),
                              _ptr(z))
    if st != OK:
        raise OracleError(st, "orc_combo_apply")
    return z


def sym_combo_apply(bands, F, dt, r, nblocks=2):
    """The symmetric combination: z1 = B_ILU^{-1} r, z2 = z1 + B^{-1}(r - A z1),
    z = z2 + B_ILU^{-1}(r - A z2) -- the three steps in order, each one an oracle
    routine (not from the paper: eq. com's combination is not symmetric)."""
    r = _f64(r)
    z1 = ilu0_apply(bands, dt, r, nblocks)
    z2 = z1 + apply(F, r - spmv(bands, z1))
    return z2 + ilu0_apply(bands, dt, r - spmv(bands, z2), nblocks)


def sym_combo_apply_c(bands, F, dt, r, nblocks=2):
    """The symmetric combination's three steps in the C oracle (orc_sym_combo_apply)."""
    d, ax, ay, az = [_f64(a) for a in bands]
    nz, ny, nx = d.shape
    r = _f64(r).reshape(d.shape)
    z = np.empty_like(d)
    st = _L().orc_sym_combo_apply(nx, ny, nz, _ptr(d), _ptr(ax), _ptr(ay), _ptr(az),
                                  _ptr(F["e1"]), _ptr(F["M"]), _ptr(F["f2"]), _ptr(_f64(dt)),
                                  int(nblocks), _ptr(r), _ptr(z))
    if st != OK:
        raise OracleError(st, "orc_sym_combo_apply")
    return z


def pcg_with(bands, precond, b, tol=1e-8, maxit=200):
    """Preconditioned CG (x0 = 0) with any preconditioner function z = precond(r),
    stopping on the recursive residual and confirming with the true one, and
    breaking down when p'Ap or r'z is not positive (the rules of orc_pcg);
    returns (x, iters, true relres, status)."""
    b = _f64(b)
    bn = np.sqrt(dot(b, b))
    x = np.zeros_like(b)
    if bn == 0.0:
        return x, 0, 0.0, OK
    r = b.copy()
    z = precond(r)
    p = z.copy()
    rho = dot(r, z)
    if not (rho > 0.0) or not np.isfinite(rho):
        return x, 0, 1.0, EBREAKDOWN
    for it in range(1, maxit + 1):
        q = spmv(bands, p)
        pq = dot(p, q)
        if not (pq > 0.0) or not np.isfinite(pq):
            return x, it - 1, np.sqrt(dot(b - spmv(bands, x), b - spmv(bands, x))) / bn, EBREAKDOWN
        alpha = rho / pq
        x += alpha * p
        r -= alpha * q
        if np.sqrt(dot(r, r)) / bn <= tol:
            res = b - spmv(bands, x)
            tr = np.sqrt(dot(res, res)) / bn
            if tr <= tol:
                return x, it, tr, OK
        z = precond(r)
        rho_new = dot(r, z)
        if not (rho_new > 0.0) or not np.isfinite(rho_new):
            res = b - spmv(bands, x)
            return x, it, np.sqrt(dot(res, res)) / bn, EBREAKDOWN
        p = z + (rho_new / rho) * p
        rho = rho_new
    res = b - spmv(bands, x)
    return x, maxit, np.sqrt(dot(res, res)) / bn, ENOCONV


COMBOS = {"none": 0, "ilu0": 1, "ilu0sym": 2}


def pcg(bands, F, b, tol=1e-8, maxit=200, dt=None, nblocks=2, smoother=None):
    """PCG with B (dt None), with the combination of eq. com (dt given), or with
    the symmetric combination (smoother="ilu0sym", dt given); returns (x, iters,
    true relres, status, residual history)."""
    d, ax, ay, az = [_f64(a) for a in bands]
    nz, ny, nx = d.shape
    b = _f64(b).reshape(d.shape)
    x = np.empty_like(d)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    hist = np.zeros(maxit + 1)
    dtp = None if dt is None else _f64(dt)
    combo = COMBOS[smoother] if smoother is not None else (0 if dt is None else 1)
    st = _L().orc_pcg_combo(nx, ny, nz, _ptr(d), _ptr(ax), _ptr(ay), _ptr(az), _ptr(F["e1"]),
                            _ptr(F["M"]), _ptr(F["f2"]), _ptr(dtp), int(nblocks), int(combo),
                            _ptr(b), _ptr(x), float(tol), int(maxit), ctypes.byref(it),
                            ctypes.byref(rr), _ptr(hist))
    return x, it.value, rr.value, st, hist[: it.value]
