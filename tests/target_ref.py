"""Dense reference of the filter-vector target for tiny grids, built on the
oracle's preconditioner (test infrastructure)."""
from __future__ import annotations

import numpy as np


def filter_target(kappa, bc, schur, outer, floor, v0=None):
    """Inverse iteration on B^{-1}A written out densely: B^{-1} from the
    oracle's apply (columns = applies to unit vectors), A from the oracle's
    bands; v <- y / (entry of y of largest magnitude), y = A^{-1} B v, from
    v = 1; returns (max(v, floor), the last v'Av / y'Av, A, B^{-1})."""
    import oracle as O
    bands = O.assemble(kappa, bc)
    F = O.setup(bands, mode=schur)
    N = kappa.size
    E = np.eye(N)
    Binv = np.stack([O.apply(F, E[j].reshape(kappa.shape)).ravel() for j in range(N)], axis=1)
    A = np.stack([O.spmv(bands, E[j].reshape(kappa.shape)).ravel() for j in range(N)], axis=1)
    B = np.linalg.inv(Binv)
    v = np.ones(N) if v0 is None else np.asarray(v0, dtype=np.float64).ravel().copy()
    lam = None
    for _ in range(outer):
        y = np.linalg.solve(A, B @ v)
        lam = (v @ A @ v) / (y @ A @ v)
        v = y / y[np.argmax(np.abs(y))]
    return np.maximum(v, floor).reshape(kappa.shape), lam, A, Binv
