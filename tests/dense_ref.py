"""Independent dense helpers for pinning the oracle on tiny grids.

Nothing here calls the oracle's arithmetic: matrices are assembled face by face
with numpy fancy indexing and solved with numpy/scipy dense routines.  Used only
by the tests.
"""
from __future__ import annotations

import numpy as np

DIRICHLET = 0


def assemble_dense(kappa, bc):
    """Dense 7-point matrix, built face by face (interior faces get the harmonic
    mean of the two node values, Dirichlet boundary faces add the node value to
    the diagonal, Neumann faces nothing)."""
    kappa = np.asarray(kappa, dtype=np.float64)
    N = kappa.size
    idx = np.arange(N).reshape(kappa.shape)
    A = np.zeros((N, N))
    # axis 2 = x (faces 0, 1), axis 1 = y (faces 2, 3), axis 0 = z (faces 4, 5)
    for axis, (f_lo, f_hi) in ((2, (0, 1)), (1, (2, 3)), (0, (4, 5))):
        n = kappa.shape[axis]
        if n > 1:
            k1 = np.take(kappa, np.arange(n - 1), axis=axis).ravel()
            k2 = np.take(kappa, np.arange(1, n), axis=axis).ravel()
            i1 = np.take(idx, np.arange(n - 1), axis=axis).ravel()
            i2 = np.take(idx, np.arange(1, n), axis=axis).ravel()
            c = 2.0 * k1 * k2 / (k1 + k2)
            np.add.at(A, (i1, i1), c)
            np.add.at(A, (i2, i2), c)
            np.add.at(A, (i1, i2), -c)
            np.add.at(A, (i2, i1), -c)
        for face, sl in ((f_lo, 0), (f_hi, n - 1)):
            if bc[face] == DIRICHLET:
                ii = np.take(idx, [sl], axis=axis).ravel()
                kk = np.take(kappa, [sl], axis=axis).ravel()
                np.add.at(A, (ii, ii), kk)
    return A


def bands_from_dense(A, shape):
    """(d, ax, ay, az) of a dense 7-point matrix on a grid of shape (nz, ny, nx)."""
    nz, ny, nx = shape
    N = nx * ny * nz
    d = np.diag(A).copy()
    ax = np.zeros(N); ay = np.zeros(N); az = np.zeros(N)
    p = np.arange(N)
    i, j, k = p % nx, (p // nx) % ny, p // (nx * ny)
    m = i < nx - 1; ax[m] = A[p[m], p[m] + 1]
    m = j < ny - 1; ay[m] = A[p[m], p[m] + nx]
    m = k < nz - 1; az[m] = A[p[m], p[m] + nx * ny]
    return tuple(a.reshape(shape) for a in (d, ax, ay, az))


def dense_from_bands(bands):
    d, ax, ay, az = [np.asarray(a).ravel() for a in bands]
    nz, ny, nx = np.asarray(bands[0]).shape
    N = d.size
    A = np.diag(d)
    for off, a in ((1, ax), (nx, ay), (nx * ny, az)):
        if off < N:
            v = a[: N - off]
            A += np.diag(v, off) + np.diag(v, -off)
    return A


def plane_matrix(dP, xP, yP):
    """Dense 5-point plane matrix from its diagonal, x-band and y-band (ny, nx)."""
    ny, nx = dP.shape
    n = nx * ny
    P = np.diag(dP.ravel())
    xv, yv = xP.ravel(), yP.ravel()
    if n > 1:
        P += np.diag(xv[: n - 1], 1) + np.diag(xv[: n - 1], -1)
    if nx < n:
        P += np.diag(yv[: n - nx], nx) + np.diag(yv[: n - nx], -nx)
    return P


def tridiag(d, e):
    n = len(d)
    T = np.diag(np.asarray(d, dtype=np.float64))
    if n > 1:
        T += np.diag(e[: n - 1], 1) + np.diag(e[: n - 1], -1)
    return T
