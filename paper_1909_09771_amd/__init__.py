"""MI355X (gfx950) library for the nested, twisted frequency-filtering
preconditioned conjugate gradient method of arXiv:1909.09771.

This module is argument marshalling only: every step (assembly, factorization,
preconditioner apply, SpMV, reductions, PCG) runs in the HIP kernels of
libntd.so behind the C ABI of include/ntd.h.  PyTorch provides device memory
and the current HIP stream.  There is no CPU fallback: if libntd.so is missing
or no GPU is present the calls raise.

Grid vectors are float64 CUDA tensors of shape (nz, ny, nx), C-contiguous.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libntd.so")

OK, EINVAL, ENOMEM, ENOTSPD, EBREAKDOWN, ENOCONV, EHIP = range(7)
PREC = {"fp64": 0, "mixed": 1}
SCHUR = {"newton": 0, "diag": 1}
SMOOTHER = {"none": 0, "ilu0": 1, "ilu0sym": 2}
EXPORTS = {"d": 0, "ax": 1, "ay": 2, "az": 3, "e1": 4, "minv": 5, "f2": 6, "dT": 7, "dP": 8,
           "xP": 9, "dt": 10}
MAX_NX = 1024
# ntd_progress_fn: (iteration, relres, ctx)
PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_int, ctypes.c_double, ctypes.c_void_p)

_lib = None


class NTDError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__("%s: %s (status %d)" % (what, strerror(status), status))
        self.status = status


def lib() -> ctypes.CDLL:
    """Load libntd.so (built in-tree by build.py); raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libntd.so is not built: run paper_1909_09771_amd/build.py "
                               "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(LIB_PATH)
        P, I, D, Z = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        L.ntd_workspace_bytes.argtypes = [I, I, I, I, I]
        L.ntd_workspace_bytes.restype = Z
        L.ntd_setup.argtypes = [I, I, I, P, P, P, I, I, I, P, Z, P, ctypes.POINTER(P)]
        L.ntd_setup.restype = I
        for name in ("ntd_apply_precond", "ntd_apply_ntd", "ntd_apply_ilu0"):
            getattr(L, name).argtypes = [P, P, P, P]
            getattr(L, name).restype = I
        L.ntd_apply_profile.argtypes = [P, P, P, ctypes.POINTER(ctypes.c_float), P]
        L.ntd_apply_profile.restype = I
        L.ntd_spmv.argtypes = [P, P, P, P]
        L.ntd_spmv.restype = I
        L.ntd_dot.argtypes = [P, P, P, ctypes.POINTER(D), P]
        L.ntd_dot.restype = I
        L.ntd_dot_noalloc.argtypes = [P, P, ctypes.c_longlong, P, P]
        L.ntd_dot_noalloc.restype = I
        L.ntd_pcg_solve.argtypes = [P, P, P, D, I, ctypes.POINTER(I), ctypes.POINTER(D), P]
        L.ntd_pcg_solve.restype = I
        L.ntd_pcg_solve_history.argtypes = [P, P, P, D, I, ctypes.POINTER(I), ctypes.POINTER(D),
                                            ctypes.POINTER(D), P]
        L.ntd_pcg_solve_history.restype = I
        L.ntd_pcg_solve_progress.argtypes = [P, P, P, D, I, ctypes.POINTER(I),
                                             ctypes.POINTER(D), P, I, PROGRESS_FN, P, P]
        L.ntd_pcg_solve_progress.restype = I
        L.ntd_filter_target.argtypes = [P, P, I, D, I, D, P, ctypes.POINTER(I),
                                        ctypes.POINTER(D), P]
        L.ntd_filter_target.restype = I
        L.ntd_vec_normalize.argtypes = [P, ctypes.c_longlong, D, P, ctypes.POINTER(D), P]
        L.ntd_vec_normalize.restype = I
        L.ntd_export.argtypes = [P, I, P, P]
        L.ntd_export.restype = I
        L.ntd_load_factors.argtypes = [P, P, P, P, P]
        L.ntd_load_factors.restype = I
        L.ntd_footprint_bytes.argtypes = [P]
        L.ntd_footprint_bytes.restype = Z
        L.ntd_destroy.argtypes = [P]
        L.ntd_destroy.restype = I
        L.ntd_strerror.argtypes = [I]
        L.ntd_strerror.restype = ctypes.c_char_p
        PP = ctypes.POINTER(P)
        L.ntd_batch_workspace_bytes.argtypes = [I, ctypes.POINTER(I), I, I]
        L.ntd_batch_workspace_bytes.restype = Z
        L.ntd_batch_setup.argtypes = [I, ctypes.POINTER(I), PP, ctypes.POINTER(I), I, I, I, P, Z, P,
                                      ctypes.POINTER(P)]
        L.ntd_batch_setup.restype = I
        L.ntd_batch_apply.argtypes = [P, PP, PP, P]
        L.ntd_batch_apply.restype = I
        L.ntd_batch_apply_profile.argtypes = [P, PP, PP, ctypes.POINTER(ctypes.c_float), P]
        L.ntd_batch_apply_profile.restype = I
        L.ntd_batch_pcg_solve.argtypes = [P, PP, PP, D, I, I, ctypes.POINTER(I), ctypes.POINTER(D),
                                          ctypes.POINTER(I), P]
        L.ntd_batch_pcg_solve.restype = I
        L.ntd_batch_tune.argtypes = [P, ctypes.POINTER(I), P]
        L.ntd_batch_tune.restype = I
        L.ntd_batch_set_sweep_group.argtypes = [P, I]
        L.ntd_batch_set_sweep_group.restype = I
        L.ntd_batch_tune_sweeps.argtypes = [P, ctypes.POINTER(I), P]
        L.ntd_batch_set_plane_lds.argtypes = [P, I, ctypes.POINTER(I)]
        L.ntd_batch_set_plane_lds.restype = I
        L.ntd_batch_tune_sweeps.restype = I
        L.ntd_batch_solve_stats.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(D),
                                            ctypes.POINTER(D)]
        L.ntd_batch_solve_stats.restype = I
        L.ntd_batch_footprint_bytes.argtypes = [P]
        L.ntd_batch_footprint_bytes.restype = Z
        L.ntd_batch_destroy.argtypes = [P]
        L.ntd_batch_destroy.restype = I
        L.ntd_cnn_workspace_bytes.argtypes = [I, I, I]
        L.ntd_cnn_workspace_bytes.restype = Z
        L.ntd_cnn_predict.argtypes = [I, I, I, P, P, P, P, P, Z, P]
        L.ntd_cnn_predict.restype = I
        L.ntd_cnn_loss_grad.argtypes = [I, I, I, P, P, P, P, ctypes.POINTER(D), P, Z, P]
        L.ntd_cnn_loss_grad.restype = I
        L.ntd_cnn_adam.argtypes = [P, P, P, P, I, ctypes.c_float, P]
        L.ntd_cnn_adam.restype = I
        _lib = L
    return _lib


def vec_normalize(v: torch.Tensor, floor: float = -2.0) -> float:
    """v <- max(v / (its entry of largest magnitude), floor) in place on the
    device (ntd_vec_normalize); floor <= -1 leaves it unclipped.  Returns the
    scale applied."""
    if not (v.is_cuda and v.dtype == torch.float64 and v.is_contiguous()):
        raise ValueError("v must be a contiguous float64 CUDA tensor")
    part = torch.empty(2048, dtype=torch.float64, device=v.device)
    sc = ctypes.c_double(0.0)
    st = lib().ntd_vec_normalize(_dptr(v), v.numel(), float(floor), _dptr(part), ctypes.byref(sc),
                                 _stream_ptr(v.device))
    if st != OK:
        raise NTDError(st, "ntd_vec_normalize")
    return sc.value


def strerror(status: int) -> str:
    return lib().ntd_strerror(int(status)).decode()


def workspace_bytes(nx: int, ny: int, nz: int, prec: str = "mixed", smoother: str = "none") -> int:
    return int(lib().ntd_workspace_bytes(nx, ny, nz, PREC[prec], SMOOTHER[smoother]))


def _stream_ptr(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _check_vec(t: torch.Tensor, shape, device, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError("%s must be a contiguous float64 tensor of shape %s" % (name, shape))
    if t.device != device:
        raise ValueError("%s is on %s, the solver on %s" % (name, t.device, device))


class Solver:
    """A factored preconditioner B for one grid, kappa field, boundary set and filter.

    kappa: float64 CUDA tensor (nz, ny, nx), > 0.  bc: six ints (x-, x+, y-, y+,
    z-, z+), 0 = Dirichlet, 1 = Neumann.  t: optional filter vector (> 0), default
    ones.  prec: "fp64" or "mixed".  schur: "newton" or "diag".  smoother: "none"
    or "ilu0" (the combination preconditioner of the paper's experiments).
    """

    def __init__(self, kappa: torch.Tensor, bc, t: torch.Tensor | None = None,
                 prec: str = "mixed", schur: str = "diag", smoother: str = "none"):
        if kappa.dim() != 3:
            raise ValueError("kappa must have shape (nz, ny, nx)")
        self.shape = tuple(kappa.shape)
        self.device = kappa.device
        nz, ny, nx = self.shape
        _check_vec(kappa, self.shape, self.device, "kappa")
        if t is not None:
            _check_vec(t, self.shape, self.device, "t")
        self.prec, self.schur, self.smoother = prec, schur, smoother
        L = lib()
        nbytes = int(L.ntd_workspace_bytes(nx, ny, nz, PREC[prec], SMOOTHER[smoother]))
        if nbytes == 0:
            raise NTDError(EINVAL, "ntd_workspace_bytes(%d, %d, %d)" % (nx, ny, nz))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        bc_arr = (ctypes.c_int * 6)(*[int(v) for v in bc])
        h = ctypes.c_void_p()
        st = L.ntd_setup(nx, ny, nz, _dptr(kappa), bc_arr, _dptr(t) if t is not None else None,
                         PREC[prec], SCHUR[schur], SMOOTHER[smoother], _dptr(self.workspace),
                         nbytes,
                         _stream_ptr(self.device), ctypes.byref(h))
        if st != OK:
            raise NTDError(st, "ntd_setup")
        self._h = h

    # -- the hot path -------------------------------------------------------
    def _apply_with(self, name: str, r: torch.Tensor, out: torch.Tensor | None):
        _check_vec(r, self.shape, self.device, "r")
        z = torch.empty_like(r) if out is None else out
        _check_vec(z, self.shape, self.device, "out")
        st = getattr(lib(), name)(self._h, _dptr(r), _dptr(z), _stream_ptr(self.device))
        if st != OK:
            raise NTDError(st, name)
        return z

    def apply(self, r: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """z = (preconditioner)^{-1} r: B^{-1} r, or the combination with ILU(0)."""
        return self._apply_with("ntd_apply_precond", r, out)

    def apply_ntd(self, r: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """z = B^{-1} r (the nested twisted sweeps alone)."""
        return self._apply_with("ntd_apply_ntd", r, out)

    def apply_ilu0(self, r: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """z = B_ILU^{-1} r (block-diagonal ILU(0) alone; needs smoother="ilu0")."""
        return self._apply_with("ntd_apply_ilu0", r, out)

    def apply_profile(self, r: torch.Tensor, out: torch.Tensor):
        """The preconditioner as PCG launches it (synchronous); returns the
        durations in ms of the lower level-3 sweep, the twist plane, the upper
        level-3 sweep and the smoother part before them (without a smoother,
        the gap between two back-to-back events)."""
        _check_vec(r, self.shape, self.device, "r")
        _check_vec(out, self.shape, self.device, "out")
        ms = (ctypes.c_float * 4)()
        st = lib().ntd_apply_profile(self._h, _dptr(r), _dptr(out), ms, _stream_ptr(self.device))
        if st != OK:
            raise NTDError(st, "ntd_apply_profile")
        return tuple(float(v) for v in ms)

    def spmv(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        _check_vec(x, self.shape, self.device, "x")
        y = torch.empty_like(x) if out is None else out
        _check_vec(y, self.shape, self.device, "out")
        st = lib().ntd_spmv(self._h, _dptr(x), _dptr(y), _stream_ptr(self.device))
        if st != OK:
            raise NTDError(st, "ntd_spmv")
        return y

    def dot(self, x: torch.Tensor, y: torch.Tensor) -> float:
        _check_vec(x, self.shape, self.device, "x")
        _check_vec(y, self.shape, self.device, "y")
        res = ctypes.c_double(0.0)
        st = lib().ntd_dot(self._h, _dptr(x), _dptr(y), ctypes.byref(res),
                           _stream_ptr(self.device))
        if st != OK:
            raise NTDError(st, "ntd_dot")
        return res.value

    def pcg(self, b: torch.Tensor, tol: float = 1e-8, maxit: int = 200,
            x: torch.Tensor | None = None, progress=None, every: int = 100):
        """Solve A x = b; returns (x, iterations, true relative residual, status).
        status is OK, ENOCONV or EBREAKDOWN; other failures raise.  progress,
        if given, is called as progress(iteration, relres) after every
        `every`-th iteration (ntd_pcg_solve_progress)."""
        _check_vec(b, self.shape, self.device, "b")
        x = torch.empty_like(b) if x is None else x
        _check_vec(x, self.shape, self.device, "x")
        it = ctypes.c_int(0)
        rr = ctypes.c_double(0.0)
        if progress is None:
            st = lib().ntd_pcg_solve(self._h, _dptr(b), _dptr(x), float(tol), int(maxit),
                                     ctypes.byref(it), ctypes.byref(rr), _stream_ptr(self.device))
        else:
            cb = PROGRESS_FN(lambda i, r, _ctx: progress(i, r))
            st = lib().ntd_pcg_solve_progress(self._h, _dptr(b), _dptr(x), float(tol), int(maxit),
                                              ctypes.byref(it), ctypes.byref(rr), None,
                                              int(every), cb, None, _stream_ptr(self.device))
        if st not in (OK, ENOCONV, EBREAKDOWN):
            raise NTDError(st, "ntd_pcg_solve")
        return x, it.value, rr.value, st

    def pcg_history(self, b: torch.Tensor, tol: float = 1e-8, maxit: int = 200,
                    x: torch.Tensor | None = None, progress=None, every: int = 100):
        """As pcg, plus the recursive relative residual after every iteration:
        returns (x, iterations, true relative residual, status, history)."""
        _check_vec(b, self.shape, self.device, "b")
        x = torch.empty_like(b) if x is None else x
        _check_vec(x, self.shape, self.device, "x")
        it = ctypes.c_int(0)
        rr = ctypes.c_double(0.0)
        hist = (ctypes.c_double * max(int(maxit), 1))()
        if progress is None:
            st = lib().ntd_pcg_solve_history(self._h, _dptr(b), _dptr(x), float(tol), int(maxit),
                                             ctypes.byref(it), ctypes.byref(rr), hist,
                                             _stream_ptr(self.device))
        else:
            cb = PROGRESS_FN(lambda i, r, _ctx: progress(i, r))
            st = lib().ntd_pcg_solve_progress(self._h, _dptr(b), _dptr(x), float(tol), int(maxit),
                                              ctypes.byref(it), ctypes.byref(rr), hist,
                                              int(every), cb, None, _stream_ptr(self.device))
        if st not in (OK, ENOCONV, EBREAKDOWN):
            raise NTDError(st, "ntd_pcg_solve_history")
        return x, it.value, rr.value, st, list(hist[: it.value])

    def filter_target(self, v0: torch.Tensor | None = None, outer: int = 20,
                      inner_tol: float = 1e-10, inner_maxit: int = 5000, floor: float = 1e-3):
        """The smallest-eigenvalue eigenvector of B^{-1}A by inverse iteration
        (ntd_filter_target), clipped below at floor; returns (t, inner CG steps,
        eigenvalue estimate)."""
        v = torch.ones(self.shape, dtype=torch.float64, device=self.device) if v0 is None \
            else v0.clone()
        _check_vec(v, self.shape, self.device, "v0")
        work = torch.empty((7,) + tuple(self.shape), dtype=torch.float64, device=self.device)
        it = ctypes.c_int(0)
        lam = ctypes.c_double(0.0)
        st = lib().ntd_filter_target(self._h, _dptr(v), int(outer), float(inner_tol),
                                     int(inner_maxit), float(floor), _dptr(work),
                                     ctypes.byref(it), ctypes.byref(lam), _stream_ptr(self.device))
        if st != OK:
            raise NTDError(st, "ntd_filter_target")
        return v, it.value, lam.value

    # -- inspection ---------------------------------------------------------
    def export(self, which: str) -> torch.Tensor:
        out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        st = lib().ntd_export(self._h, EXPORTS[which], _dptr(out), _stream_ptr(self.device))
        if st != OK:
            raise NTDError(st, "ntd_export")
        return out

    def load_factors(self, e1: torch.Tensor, pivots: torch.Tensor, f2: torch.Tensor):
        for n, v in (("e1", e1), ("pivots", pivots), ("f2", f2)):
            _check_vec(v, self.shape, self.device, n)
        st = lib().ntd_load_factors(self._h, _dptr(e1), _dptr(pivots), _dptr(f2),
                                    _stream_ptr(self.device))
        if st != OK:
            raise NTDError(st, "ntd_load_factors")

    @property
    def footprint_bytes(self) -> int:
        return int(lib().ntd_footprint_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().ntd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


BATCH_GRAPH = 1


def _ptr_array(tensors):
    return (ctypes.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])


class Batch:
    """Many independent systems, nrhs right-hand sides each, preconditioned with
    B (no smoother) and solved together: every batched launch covers all
    systems and right-hand sides.

    kappas: list of float64 CUDA tensors (nz, ny, nx), one per system (sizes may
    differ; nx <= 512).  bcs: one six-int face list per system, or a single list
    for all.  Entry e = s * nrhs + q is right-hand side q of system s; the
    methods take and return flat lists of [N_s] tensors in that order.
    """

    def __init__(self, kappas, bcs, nrhs: int = 1, prec: str = "mixed", schur: str = "diag"):
        if len(kappas) == 0:
            raise ValueError("a batch needs at least one system")
        self.device = kappas[0].device
        self.shapes = [tuple(k.shape) for k in kappas]
        for k, sh in zip(kappas, self.shapes):
            if k.dim() != 3:
                raise ValueError("kappa must have shape (nz, ny, nx)")
            _check_vec(k, sh, self.device, "kappa")
        if len(bcs) > 0 and not hasattr(bcs[0], "__len__"):  # one face list for all
            bcs = [bcs] * len(kappas)
        if len(bcs) != len(kappas):
            raise ValueError("one face list per system")
        self.count, self.nrhs, self.prec, self.schur = len(kappas), int(nrhs), prec, schur
        dims = []
        for (nz, ny, nx) in self.shapes:
            dims += [nx, ny, nz]
        self._dims = (ctypes.c_int * len(dims))(*dims)
        L = lib()
        nbytes = int(L.ntd_batch_workspace_bytes(self.count, self._dims, self.nrhs, PREC[prec]))
        if nbytes == 0:
            raise NTDError(EINVAL, "ntd_batch_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        bc_flat = [int(v) for bc in bcs for v in bc]
        bc_arr = (ctypes.c_int * len(bc_flat))(*bc_flat)
        self._kappas = list(kappas)  # kept alive only through setup
        h = ctypes.c_void_p()
        st = L.ntd_batch_setup(self.count, self._dims, _ptr_array(self._kappas), bc_arr, self.nrhs,
                               PREC[prec], SCHUR[schur], _dptr(self.workspace), nbytes,
                               _stream_ptr(self.device), ctypes.byref(h))
        self._kappas = None
        if st != OK:
            raise NTDError(st, "ntd_batch_setup")
        self._h = h

    @property
    def entries(self) -> int:
        return self.count * self.nrhs

    def entry_shape(self, e: int):
        return self.shapes[e // self.nrhs]

    def _check_list(self, vecs, name):
        if len(vecs) != self.entries:
            raise ValueError("%s: expected %d vectors (systems x rhs)" % (name, self.entries))
        for e, v in enumerate(vecs):
            _check_vec(v, self.entry_shape(e), self.device, "%s[%d]" % (name, e))

    def empty_like_entries(self):
        return [torch.empty(self.entry_shape(e), dtype=torch.float64, device=self.device)
                for e in range(self.entries)]

    def apply(self, rs, zs=None):
        """z[e] = B_s^{-1} r[e] for every entry."""
        self._check_list(rs, "r")
        zs = self.empty_like_entries() if zs is None else zs
        self._check_list(zs, "z")
        st = lib().ntd_batch_apply(self._h, _ptr_array(rs), _ptr_array(zs),
                                   _stream_ptr(self.device))
        if st != OK:
            raise NTDError(st, "ntd_batch_apply")
        return zs

    def apply_profile(self, rs, zs):
        """As apply, synchronous; returns the event-timed durations (ms) of the
        lower sweep, the twist planes, the upper sweep and the rest."""
        self._check_list(rs, "r")
        self._check_list(zs, "z")
        ms = (ctypes.c_float * 4)()
        st = lib().ntd_batch_apply_profile(self._h, _ptr_array(rs), _ptr_array(zs), ms,
                                           _stream_ptr(self.device))
        if st != OK:
            raise NTDError(st, "ntd_batch_apply_profile")
        return tuple(float(v) for v in ms)

    def pcg(self, bs, tol: float = 1e-8, maxit: int = 1000, graph: bool = True, xs=None):
        """PCG for every entry; returns (xs, iters, relres, status) with per-entry lists."""
        self._check_list(bs, "b")
        xs = self.empty_like_entries() if xs is None else xs
        self._check_list(xs, "x")
        n = self.entries
        it = (ctypes.c_int * n)()
        rr = (ctypes.c_double * n)()
        stv = (ctypes.c_int * n)()
        st = lib().ntd_batch_pcg_solve(self._h, _ptr_array(bs), _ptr_array(xs), float(tol),
                                       int(maxit), BATCH_GRAPH if graph else 0, it, rr, stv,
                                       _stream_ptr(self.device))
        if st != OK:
            raise NTDError(st, "ntd_batch_pcg_solve")
        return xs, list(it), list(rr), list(stv)

    def tune(self) -> int:
        """Autotune the workgroups per entry of the bandwidth kernels (ntd_batch_tune);
        returns the choice."""
        gx = ctypes.c_int(0)
        st = lib().ntd_batch_tune(self._h, ctypes.byref(gx), _stream_ptr(self.device))
        if st != OK:
            raise NTDError(st, "ntd_batch_tune")
        return gx.value

    def set_sweep_group(self, nr: int):
        """Right-hand sides per wavefront pair in the line sweeps (1, 2 or 4;
        ntd_batch_set_sweep_group)."""
        st = lib().ntd_batch_set_sweep_group(self._h, int(nr))
        if st != OK:
            raise NTDError(st, "ntd_batch_set_sweep_group")

    def set_plane_lds(self, on: bool) -> bool:
        """Plane buffers of the line sweeps in LDS (True, the default) or in
        device memory (ntd_batch_set_plane_lds); returns whether the sweeps
        will use LDS buffers (every workgroup of a sweep resident at once with
        its buffers, at the current sweep group)."""
        used = ctypes.c_int(0)
        st = lib().ntd_batch_set_plane_lds(self._h, 1 if on else 0, ctypes.byref(used))
        if st != OK:
            raise NTDError(st, "ntd_batch_set_plane_lds")
        return bool(used.value)

    def solve_stats(self):
        """(passes, gap_ms, solve_ms) of the last pcg: host checks, the stream's
        idle time between runs of iterations, and the iterations' total time."""
        n, g, t = ctypes.c_int(0), ctypes.c_double(0.0), ctypes.c_double(0.0)
        st = lib().ntd_batch_solve_stats(self._h, ctypes.byref(n), ctypes.byref(g),
                                         ctypes.byref(t))
        if st != OK:
            raise NTDError(st, "ntd_batch_solve_stats")
        return n.value, g.value, t.value

    def tune_sweeps(self) -> int:
        """Autotune the right-hand sides per wavefront pair of the line sweeps
        (ntd_batch_tune_sweeps); returns the choice."""
        nr = ctypes.c_int(0)
        st = lib().ntd_batch_tune_sweeps(self._h, ctypes.byref(nr), _stream_ptr(self.device))
        if st != OK:
            raise NTDError(st, "ntd_batch_tune_sweeps")
        return nr.value

    @property
    def footprint_bytes(self) -> int:
        return int(lib().ntd_batch_footprint_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().ntd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


CNN_NPARAMS = 14737


class FilterNet:
    """The learned filter vector's network (ntd_cnn_* in include/ntd.h): kappa ->
    t > 0, four 3x3x3 convolution layers 1-16-16-16-1 on the matrix cores.

    params: float32 array-like of CNN_NPARAMS values (per layer W[cout][tap][cin]
    then b[cout]).  The parameters and the Adam moments live on `device`; a
    workspace is kept per grid shape.
    """

    def __init__(self, params, device="cuda:0"):
        self.device = torch.device(device)
        p = torch.as_tensor(params, dtype=torch.float32).reshape(-1)
        if p.numel() != CNN_NPARAMS:
            raise ValueError("expected %d parameters, got %d" % (CNN_NPARAMS, p.numel()))
        self.params = p.to(self.device).contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.step = 0
        self._ws = {}

    def _workspace(self, shape):
        nz, ny, nx = shape
        ws = self._ws.get(shape)
        if ws is None:
            nbytes = int(lib().ntd_cnn_workspace_bytes(nx, ny, nz))
            if nbytes == 0:
                raise NTDError(EINVAL, "ntd_cnn_workspace_bytes")
            ws = self._ws[shape] = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return ws

    def release_workspaces(self):
        self._ws = {}

    def predict(self, kappa: torch.Tensor, t: torch.Tensor | None = None,
                y: torch.Tensor | None = None) -> torch.Tensor:
        """t (float64, shape of kappa) for one field; y optionally receives the
        output before the softplus (float32)."""
        if kappa.dim() != 3:
            raise ValueError("kappa must have shape (nz, ny, nx)")
        shape = tuple(kappa.shape)
        _check_vec(kappa, shape, self.device, "kappa")
        if t is None:
            t = torch.empty_like(kappa)
        _check_vec(t, shape, self.device, "t")
        if y is not None and (y.dtype != torch.float32 or tuple(y.shape) != shape
                              or not y.is_contiguous() or y.device != self.device):
            raise ValueError("y must be a contiguous float32 tensor of shape %s" % (shape,))
        ws = self._workspace(shape)
        nz, ny, nx = shape
        st = lib().ntd_cnn_predict(nx, ny, nz, _dptr(kappa), _dptr(self.params), _dptr(t),
                                   _dptr(y) if y is not None else None, _dptr(ws), ws.numel(),
                                   _stream_ptr(self.device))
        if st != OK:
            raise NTDError(st, "ntd_cnn_predict")
        return t

    def loss_grad(self, kappa: torch.Tensor, target: torch.Tensor, grad: torch.Tensor | None = None):
        """(loss, grad): mean (t - target)^2 and its gradient (float32 [CNN_NPARAMS])."""
        shape = tuple(kappa.shape)
        _check_vec(kappa, shape, self.device, "kappa")
        _check_vec(target, shape, self.device, "target")
        grad = self.grad if grad is None else grad
        ws = self._workspace(shape)
        nz, ny, nx = shape
        loss = ctypes.c_double()
        st = lib().ntd_cnn_loss_grad(nx, ny, nz, _dptr(kappa), _dptr(target), _dptr(self.params),
                                     _dptr(grad), ctypes.byref(loss), _dptr(ws), ws.numel(),
                                     _stream_ptr(self.device))
        if st != OK:
            raise NTDError(st, "ntd_cnn_loss_grad")
        return loss.value, grad

    def adam_step(self, grad: torch.Tensor, lr: float):
        self.step += 1
        st = lib().ntd_cnn_adam(_dptr(self.params), _dptr(self.m), _dptr(self.v), _dptr(grad),
                                self.step, float(lr), _stream_ptr(self.device))
        if st != OK:
            raise NTDError(st, "ntd_cnn_adam")

    def train_step(self, kappa: torch.Tensor, target: torch.Tensor, lr: float) -> float:
        loss, g = self.loss_grad(kappa, target)
        self.adam_step(g, lr)
        return loss
