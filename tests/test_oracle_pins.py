"""Pins of the FP64 CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle (oracle/ntd_oracle.c) against something other than
itself: closed forms, brute force with independent dense linear algebra,
invariants of the method (filter property B t = A t, SPD, covariance), the
dependency structure that the twist position implies, and special cases in which
the preconditioner must reduce to an exact solve.  No GPU is used.
"""
from __future__ import annotations

import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import workloads as W
from tests import dense_ref as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_kappa(shape, seed, contrast=3.0):
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(-contrast, contrast, size=shape)


def dense_Binv(F, shape):
    """The oracle's B^{-1} as a dense matrix (columns = applies to unit vectors)."""
    N = int(np.prod(shape))
    M = np.zeros((N, N))
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        M[:, c] = O.apply(F, e.reshape(shape)).ravel()
    return M


# --------------------------------------------------------------------------
# O1: assembly of A and the SpMV
# --------------------------------------------------------------------------

def test_assemble_constant_kappa_is_textbook_laplacian():
    shape = (4, 5, 6)
    d, ax, ay, az = O.assemble(np.ones(shape), W.BC_ALL_DIRICHLET)
    assert np.all(d == 6.0)
    nz, ny, nx = shape
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    k = np.arange(nz)[:, None, None]
    assert np.array_equal(ax, np.broadcast_to(np.where(i < nx - 1, -1.0, 0.0), shape))
    assert np.array_equal(ay, np.broadcast_to(np.where(j < ny - 1, -1.0, 0.0), shape))
    assert np.array_equal(az, np.broadcast_to(np.where(k < nz - 1, -1.0, 0.0), shape))


@pytest.mark.parametrize("shape,bc", [((3, 4, 5), [0, 1, 1, 0, 1, 0]),
                                      ((5, 2, 3), [1, 1, 0, 1, 1, 1]),
                                      ((1, 1, 7), [0, 0, 1, 1, 1, 1]),
                                      ((2, 6, 1), [1, 1, 1, 0, 0, 1])])
def test_assemble_matches_face_by_face_dense_assembly(shape, bc):
    kappa = rand_kappa(shape, 11)
    bands = O.assemble(kappa, np.array(bc, dtype=np.int32))
    A = R.assemble_dense(kappa, bc)
    ref = R.bands_from_dense(A, shape)
    for got, want in zip(bands, ref):
        np.testing.assert_allclose(got, want, rtol=1e-15, atol=0)  # diagonal: 6 terms summed in another order
    np.testing.assert_allclose(R.dense_from_bands(bands), A, rtol=1e-15, atol=0)


def test_rowsum_counts_dirichlet_faces():
    shape = (3, 4, 5)
    bc = np.array([0, 1, 0, 0, 1, 0], dtype=np.int32)
    bands = O.assemble(np.full(shape, 2.5), bc)
    s = O.spmv(bands, np.ones(shape))
    nz, ny, nx = shape
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    k = np.arange(nz)[:, None, None]
    dirichlet = (bc == 0).astype(int)
    faces = ((i == 0) * dirichlet[0] + (i == nx - 1) * dirichlet[1] + (j == 0) * dirichlet[2]
             + (j == ny - 1) * dirichlet[3] + (k == 0) * dirichlet[4] + (k == nz - 1) * dirichlet[5])
    np.testing.assert_allclose(s, 2.5 * np.broadcast_to(faces, shape), atol=1e-14)


def test_laplacian_eigenpairs_closed_form():
    """kappa = 1, Dirichlet everywhere: sin-product eigenvectors with eigenvalues
    sum_d (2 - 2 cos(pi m_d/(n_d + 1)))."""
    nz, ny, nx = 5, 6, 7
    bands = O.assemble(np.ones((nz, ny, nx)), W.BC_ALL_DIRICHLET)
    for (mx, my, mz) in [(1, 1, 1), (3, 2, 5), (7, 6, 4)]:
        vx = np.sin(np.pi * mx * np.arange(1, nx + 1) / (nx + 1))
        vy = np.sin(np.pi * my * np.arange(1, ny + 1) / (ny + 1))
        vz = np.sin(np.pi * mz * np.arange(1, nz + 1) / (nz + 1))
        v = vz[:, None, None] * vy[None, :, None] * vx[None, None, :]
        lam = sum(2 - 2 * np.cos(np.pi * m / (n + 1)) for m, n in ((mx, nx), (my, ny), (mz, nz)))
        np.testing.assert_allclose(O.spmv(bands, v), lam * v, atol=1e-13)


def test_spmv_matches_dense_and_is_symmetric():
    shape = (4, 5, 6)
    kappa = rand_kappa(shape, 3)
    bc = np.array([0, 1, 1, 0, 0, 1], dtype=np.int32)
    bands = O.assemble(kappa, bc)
    A = R.assemble_dense(kappa, bc)
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal(shape), rng.standard_normal(shape)
    np.testing.assert_allclose(O.spmv(bands, x).ravel(), A @ x.ravel(), rtol=1e-13, atol=1e-12)
    a = float(np.sum(x * O.spmv(bands, y)))
    b = float(np.sum(y * O.spmv(bands, x)))
    assert abs(a - b) <= 1e-12 * abs(a)


def test_dot_is_correctly_rounded_sum():
    rng = np.random.default_rng(9)
    x = rng.standard_normal(10007) * 10.0 ** rng.integers(-8, 8, 10007)
    y = rng.standard_normal(10007)
    exact = math.fsum((x * y).tolist())
    assert abs(O.dot(x, y) - exact) <= 2e-16 * abs(exact) + 1e-300


# --------------------------------------------------------------------------
# O2: the level-1 twisted tridiagonal solve is exact
# --------------------------------------------------------------------------

def test_twist_index_golden():
    rows = [tuple(int(v) for v in ln.split()) for ln in open(os.path.join(GOLDEN, "twist_index.txt"))
            if ln.strip() and not ln.startswith("#")]
    for nb, j in rows:
        # pivots of a line of length nb: the twist row is the only one whose pivot
        # takes both neighbours; detect it by perturbing the ends.
        if nb > 600:
            continue
        d = np.full(nb, 2.0)              # 1-D Laplacian: a change travels the whole line
        e = np.full(max(nb - 1, 0), -1.0)
        M0, st = O.line_pivots(d, e)
        assert st == 0
        d1 = d.copy(); d1[0] += 1.0
        d2 = d.copy(); d2[-1] += 1.0
        M1, _ = O.line_pivots(d1, e)
        M2, _ = O.line_pivots(d2, e)
        # a change at row 0 reaches rows 0..j, a change at the last row reaches j..nb-1
        changed_first = np.nonzero(M1 != M0)[0]
        changed_last = np.nonzero(M2 != M0)[0]
        assert changed_first.max() == j
        assert changed_last.min() == j


@pytest.mark.parametrize("n", list(range(1, 10)) + [16, 33])
def test_line_solve_1d_laplacian_closed_form(n):
    """-u'' = 1 with u = 0 at both ends, unit spacing: x_i = (i+1)(n-i)/2.  On an
    n x 1 x 1 grid with Neumann y/z faces the whole preconditioner is the exact
    line solve."""
    bc = np.array([0, 0, 1, 1, 1, 1], dtype=np.int32)
    bands = O.assemble(np.ones((1, 1, n)), bc)
    F = O.setup(bands)
    x = O.apply(F, np.ones((1, 1, n))).ravel()
    i = np.arange(n)
    np.testing.assert_allclose(x, (i + 1) * (n - i) / 2.0, rtol=1e-14)


@pytest.mark.parametrize("n", [2, 5, 8, 31, 64, 101])
def test_line_solve_random_spd_tridiagonal(n):
    rng = np.random.default_rng(n)
    e = -rng.uniform(0.1, 1.0, n - 1)
    d = rng.uniform(0.0, 0.5, n)
    d[:-1] += -e
    d[1:] += -e
    d += 1e-3
    M, st = O.line_pivots(d, np.append(e, 0.0))
    assert st == 0 and np.all(M > 0)
    y = rng.standard_normal(n)
    x = O.line_solve(np.append(e, 0.0), M, y)
    np.testing.assert_allclose(R.tridiag(d, e) @ x, y, atol=1e-12 * np.abs(y).max() * 10)
    np.testing.assert_allclose(x, np.linalg.solve(R.tridiag(d, e), y), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("mode", ["newton", "diag"])
@pytest.mark.parametrize("shape", [(1, 1, 9), (1, 8, 1), (7, 1, 1), (1, 1, 1), (2, 1, 1), (1, 1, 2)])
def test_one_dimensional_grids_give_exact_solve(shape, mode):
    """With one non-trivial axis every Schur block is a scalar, beta is its exact
    inverse, and B = A: the apply must equal a dense solve."""
    bc = np.array([0, 1, 1, 0, 0, 1], dtype=np.int32)
    kappa = rand_kappa(shape, 21)
    bands = O.assemble(kappa, bc)
    F = O.setup(bands, mode=mode)
    r = np.random.default_rng(2).standard_normal(shape)
    A = R.assemble_dense(kappa, bc)
    np.testing.assert_allclose(O.apply(F, r).ravel(), np.linalg.solve(A, r.ravel()),
                               rtol=1e-11, atol=1e-12 * np.abs(np.linalg.solve(A, r.ravel())).max())


# --------------------------------------------------------------------------
# O3/O4: the setup recurrences
# --------------------------------------------------------------------------

FILTER_SHAPES = [(5, 6, 7), (4, 3, 2), (8, 8, 8), (1, 6, 5), (6, 1, 4), (3, 5, 1), (2, 2, 2)]


@pytest.mark.parametrize("mode", ["newton", "diag"])
@pytest.mark.parametrize("shape", FILTER_SHAPES)
def test_filter_property(shape, mode):
    """B t = A t (eq. filter): B^{-1}(A t) = t to rounding, for a general t > 0."""
    kappa = rand_kappa(shape, 31, contrast=2.0)
    bc = np.array([0, 0, 0, 0, 0, 0], dtype=np.int32)
    bands = O.assemble(kappa, bc)
    t = W.filter_random(shape[2], shape[1], shape[0], 4) if mode == "newton" else np.ones(shape)
    F = O.setup(bands, t, mode=mode)
    z = O.apply(F, O.spmv(bands, t))
    assert np.abs(z - t).max() <= 1e-11 * np.abs(t).max()


def test_paper_literal_filter_exact_on_planes_only():
    """Without the level-3 compensation the filter holds for a single plane
    (level 2 is filter-exact because the line solve is exact) but not in 3D."""
    kappa2 = rand_kappa((1, 6, 7), 41)
    b2 = O.assemble(kappa2, W.BC_ALL_DIRICHLET)
    F2 = O.setup(b2, mode="paper_literal")
    t2 = np.ones((1, 6, 7))
    assert np.abs(O.apply(F2, O.spmv(b2, t2)) - t2).max() < 1e-12
    kappa3 = rand_kappa((5, 6, 7), 41)
    b3 = O.assemble(kappa3, W.BC_ALL_DIRICHLET)
    F3 = O.setup(b3, mode="paper_literal")
    t3 = np.ones((5, 6, 7))
    assert np.abs(O.apply(F3, O.spmv(b3, t3)) - t3).max() > 1e-6


@pytest.mark.parametrize("mode", ["newton", "diag", "paper_literal"])
@pytest.mark.parametrize("shape", [(3, 4, 5), (4, 4, 4), (2, 5, 3)])
def test_B_is_symmetric_positive_definite(shape, mode):
    kappa = rand_kappa(shape, 51, contrast=2.0)
    bands = O.assemble(kappa, W.BC_Z0_DIRICHLET)
    F = O.setup(bands, mode=mode)
    Bi = dense_Binv(F, shape)
    assert np.abs(Bi - Bi.T).max() <= 1e-12 * np.abs(Bi).max()
    sla.cholesky(0.5 * (Bi + Bi.T))          # raises if not positive definite
    A = R.assemble_dense(kappa, W.BC_Z0_DIRICHLET)
    B = np.linalg.inv(Bi)
    # B - A is block diagonal over planes (level-3 twisted factorization)
    nz, ny, nx = shape
    nxy = nx * ny
    E = B - A
    for k in range(nz):
        for kk in range(nz):
            if k != kk:
                assert np.abs(E[k * nxy:(k + 1) * nxy, kk * nxy:(kk + 1) * nxy]).max() < 1e-9 * np.abs(A).max()


def _contrast_fields(n, c, seed):
    rng = np.random.default_rng(seed)
    return {"subcubes": W.kappa_subcubes(n, n, n, seed, cubes=2, log10_lo=0.0, log10_hi=c),
            "random": 10.0 ** rng.uniform(0.0, c, (n, n, n)),
            "spheres": W.kappa_spheres(n, n, n, seed, count=6, r_lo=0.1, r_hi=0.25,
                                       inside=10.0 ** c)}


@pytest.mark.parametrize("mode", ["newton", "diag", "paper_literal"])
@pytest.mark.parametrize("n", [6, 8])
@pytest.mark.parametrize("contrast", [3, 6])
def test_B_is_spd_at_high_contrast(contrast, n, mode):
    """B stays symmetric positive definite on fields of contrast 1e3 and 1e6
    (subcubes, random per-node kappa, spheres).  The spectrum of B^{-1}A is
    one-sided as the Schur blocks imply: the diagonal block b lies above
    P^{-1} (B <= A, lambda >= 1); the Newton block 2b - bPb lies below it
    (B >= A, lambda <= 1) up to the level-3 filter compensation, which moves
    the largest eigenvalue above 1 by at most about 1e-4 on these fields."""
    for kind, kappa in _contrast_fields(n, contrast, 11).items():
        bands = O.assemble(kappa, W.BC_ALL_DIRICHLET)
        F = O.setup(bands, mode=mode)
        Bi = dense_Binv(F, kappa.shape)
        assert np.abs(Bi - Bi.T).max() <= 1e-12 * np.abs(Bi).max(), kind
        Lc = sla.cholesky(0.5 * (Bi + Bi.T), lower=True)  # raises if not positive definite
        if mode == "paper_literal":
            continue
        A = R.assemble_dense(kappa, W.BC_ALL_DIRICHLET)
        lam = np.linalg.eigvalsh(Lc.T @ A @ Lc)   # the spectrum of B^{-1} A, symmetrically
        if mode == "newton":
            assert lam.min() > 0.0 and lam.max() <= 1.0 + 1e-3, (kind, lam.min(), lam.max())
        else:
            assert lam.min() >= 1.0 - 1e-9, (kind, lam.min(), lam.max())


def _newton_identity(P, beta, X):
    """I - P X == (I - P beta)^2 for X = 2 beta - beta P beta (one Newton-Schulz
    step toward P^{-1} from the diagonal beta), written without X's formula."""
    I = np.eye(P.shape[0])
    return I - P @ X, (I - P @ np.diag(beta)) @ (I - P @ np.diag(beta))


@pytest.mark.parametrize("mode", ["newton", "diag"])
def test_level2_schur_update_identity(mode):
    """T_m = (line block of P) - phi Y phi with, for Newton, I - T_nb Y = (I - T_nb g)^2 and
    g = diag(T_nb^{-1} v ./ v), v = phi .* t_m; for diag, Y = g.  Checked on every
    non-twist line of a single plane, with dense numpy solves."""
    shape = (1, 7, 6)
    kappa = rand_kappa(shape, 61)
    bands = O.assemble(kappa, W.BC_ALL_DIRICHLET)
    t = W.filter_random(6, 7, 1, 8)
    F = O.setup(bands, t, mode=mode)
    nx, ny = 6, 7
    jt = (ny - 1) // 2
    d, ax, ay, _ = bands
    for m in range(ny):
        if m == jt:
            continue
        nb = m - 1 if m < jt else m + 1
        if nb < 0 or nb >= ny:
            # chain ends are the untouched line blocks of P
            np.testing.assert_array_equal(F["dT"][0, m], F["dP"][0, m])
            continue
        Tn = R.tridiag(F["dT"][0, nb], F["e1"][0, nb])
        phi = F["f2"][0, min(m, nb)]
        v = phi * t[0, m]
        g = np.linalg.solve(Tn, v) / v
        Tm = R.tridiag(F["dT"][0, m], F["e1"][0, m])
        Pm = R.tridiag(F["dP"][0, m], F["xP"][0, m])
        Y = (Pm - Tm) / np.outer(phi, phi)
        if mode == "diag":
            np.testing.assert_allclose(Y, np.diag(g), atol=1e-12 * np.abs(g).max())
        else:
            lhs, rhs = _newton_identity(Tn, g, Y)
            np.testing.assert_allclose(lhs, rhs, atol=1e-11)


@pytest.mark.parametrize("mode", ["newton", "diag"])
def test_level3_schur_update_identity(mode):
    """On 1 x ny x nz grids the plane solve is exact, the compensation vanishes and
    P_k = D^_k - psi X psi with I - P_nb X = (I - P_nb b)^2 (Newton) or X = b (diag),
    b = diag(P_nb^{-1} w ./ w), w = psi .* t_k, all with dense numpy solves."""
    shape = (7, 5, 1)
    nz, ny, nx = shape
    kappa = rand_kappa(shape, 71)
    bands = O.assemble(kappa, W.BC_ALL_DIRICHLET)
    t = W.filter_random(nx, ny, nz, 9)
    F = O.setup(bands, t, mode=mode)
    d, ax, ay, az = bands
    jt = (nz - 1) // 2
    for k in range(nz):
        if k == jt:
            continue
        nb = k - 1 if k < jt else k + 1
        Dk = R.plane_matrix(d[k], ax[k], ay[k])
        Pk = R.plane_matrix(F["dP"][k], F["xP"][k], F["f2"][k])
        if nb < 0 or nb >= nz:
            np.testing.assert_array_equal(Pk, Dk)
            continue
        Pn = R.plane_matrix(F["dP"][nb], F["xP"][nb], F["f2"][nb])
        psi = az[min(k, nb)].ravel()
        w = psi * t[k].ravel()
        b = np.linalg.solve(Pn, w) / w
        X = (Dk - Pk) / np.outer(psi, psi)
        if mode == "diag":
            np.testing.assert_allclose(X, np.diag(b), atol=1e-12 * np.abs(b).max())
        else:
            lhs, rhs = _newton_identity(Pn, b, X)
            np.testing.assert_allclose(lhs, rhs, atol=1e-11)


@pytest.mark.parametrize("level", [1, 2, 3])
@pytest.mark.parametrize("nb", [4, 5])
def test_twist_dependency_cone(level, nb):
    """With the twist at j = floor((nb-1)/2), a change of the first block's
    diagonal can only reach blocks 0..j, and a change of the last block's only
    blocks j..nb-1 (Algs 2 and 5: the two halves meet at the twist block)."""
    shape = {1: (1, 1, nb), 2: (1, nb, 3), 3: (nb, 3, 2)}[level]
    axis = {1: 2, 2: 1, 3: 0}[level]
    kappa = rand_kappa(shape, 81, contrast=1.0)
    bands = O.assemble(kappa, W.BC_ALL_DIRICHLET)
    j = (nb - 1) // 2
    F0 = O.setup(bands)
    for end in (0, nb - 1):
        d = bands[0].copy()
        sl = [slice(None)] * 3
        sl[axis] = end
        d[tuple(sl)] += 0.7
        F1 = O.setup((d,) + tuple(bands[1:]))
        changed = set()
        for key in ("M", "e1", "f2", "dT"):
            diff = np.abs(F1[key] - F0[key]) > 0
            for q in range(nb):
                s2 = [slice(None)] * 3
                s2[axis] = q
                if diff[tuple(s2)].any():
                    changed.add(q)
        reach = set(range(0, j + 1)) if end == 0 else set(range(j, nb))
        assert changed <= reach, (end, changed, reach)
        assert end in changed and j in changed


def test_scale_invariance_in_t():
    """B depends on the direction of t only (every use of t is a ratio)."""
    shape = (4, 5, 6)
    bands = O.assemble(rand_kappa(shape, 91), W.BC_Z0_DIRICHLET)
    t = W.filter_random(6, 5, 4, 10)
    r = np.random.default_rng(3).standard_normal(shape)
    z1 = O.apply(O.setup(bands, t), r)
    z2 = O.apply(O.setup(bands, 37.5 * t), r)
    np.testing.assert_allclose(z2, z1, rtol=1e-12, atol=1e-12 * np.abs(z1).max())


@pytest.mark.parametrize("mode", ["newton", "diag"])
def test_diagonal_covariance(mode):
    """A' = S A S, t' = S^{-1} t  =>  B' = S B S, i.e. B'^{-1} r = S^{-1} B^{-1} S^{-1} r."""
    shape = (4, 5, 6)
    bands = O.assemble(rand_kappa(shape, 101), W.BC_ALL_DIRICHLET)
    rng = np.random.default_rng(4)
    s = rng.uniform(0.3, 3.0, shape)
    sf = s.ravel()
    nz, ny, nx = shape
    d, ax, ay, az = [a.ravel() for a in bands]
    N = sf.size

    def sh(a, off):
        out = np.zeros(N)
        out[: N - off] = sf[off:]
        return out
    bands2 = tuple(a.reshape(shape) for a in (d * sf * sf, ax * sf * sh(ax, 1), ay * sf * sh(ay, nx),
                                                az * sf * sh(az, nx * ny)))
    t = W.filter_random(nx, ny, nz, 11)
    r = rng.standard_normal(shape)
    z = O.apply(O.setup(bands, t, mode=mode), r / s) / s
    z2 = O.apply(O.setup(bands2, t / s, mode=mode), r)
    np.testing.assert_allclose(z2, z, rtol=1e-11, atol=1e-12 * np.abs(z).max())


def test_setup_reports_non_spd():
    shape = (3, 3, 3)
    d, ax, ay, az = O.assemble(np.ones(shape), W.BC_ALL_DIRICHLET)
    d = d.copy()
    d[1, 1, 1] = -5.0
    F = O.setup((d, ax, ay, az), raise_on_error=False)
    assert F["status"] == O.ENOTSPD


# --------------------------------------------------------------------------
# O7: PCG
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mode", ["newton", "diag"])
def test_pcg_filter_rhs_converges_in_one_step(mode):
    """b = A t: the first preconditioned residual is t, so one CG step is exact."""
    shape = (6, 7, 8)
    bands = O.assemble(rand_kappa(shape, 111), W.BC_Z0_DIRICHLET)
    t = W.filter_random(8, 7, 6, 12) if mode == "newton" else np.ones(shape)
    F = O.setup(bands, t, mode=mode)
    b = O.spmv(bands, t)
    x, it, rr, st, _ = O.pcg(bands, F, b, 1e-10, 10)
    assert st == 0 and it == 1
    np.testing.assert_allclose(x, t, rtol=1e-11)


def test_pcg_matches_dense_cholesky():
    shape = (6, 6, 6)
    kappa = W.kappa_subcubes(6, 6, 6, 201, cubes=2)
    bc = W.BC_Z0_DIRICHLET
    bands = O.assemble(kappa, bc)
    F = O.setup(bands, mode="diag")
    b = W.rhs_uniform(6, 6, 6, 202)
    x, it, rr, st, _ = O.pcg(bands, F, b, 1e-12, 200)
    assert st == 0 and rr <= 1e-12
    A = R.assemble_dense(kappa, bc)
    xr = sla.cho_solve(sla.cho_factor(A), b.ravel())
    cond = np.linalg.cond(A)
    assert np.linalg.norm(x.ravel() - xr) <= 10 * cond * 1e-12 * np.linalg.norm(xr)


def test_pcg_manufactured_solution():
    shape = (8, 7, 9)
    kappa = rand_kappa(shape, 121, contrast=1.5)
    bands = O.assemble(kappa, W.BC_ALL_DIRICHLET)
    xs = np.random.default_rng(13).standard_normal(shape)
    b = O.spmv(bands, xs)
    F = O.setup(bands, mode="diag")
    x, it, rr, st, hist = O.pcg(bands, F, b, 1e-10, 300)
    assert st == 0 and rr <= 1e-10
    cond = np.linalg.cond(R.assemble_dense(kappa, W.BC_ALL_DIRICHLET))
    assert np.linalg.norm(x - xs) <= cond * 1e-10 * np.linalg.norm(xs)


def test_pcg_reports_no_convergence():
    shape = (6, 6, 6)
    bands = O.assemble(W.kappa_subcubes(6, 6, 6, 5, cubes=2), W.BC_Z0_DIRICHLET)
    F = O.setup(bands, mode="diag")
    x, it, rr, st, _ = O.pcg(bands, F, W.rhs_uniform(6, 6, 6, 1), 1e-14, 2)
    assert st == O.ENOCONV and it == 2


def _identity_factors(shape, sign):
    """Factors of B = sign * I on a single plane (no line or plane couplings,
    every pivot = sign)."""
    z = np.zeros(shape)
    return {"e1": z, "M": np.full(shape, float(sign)), "f2": z, "g3": z}


def test_pcg_breaks_down_on_a_negative_definite_preconditioner():
    """B = -I gives r.z = -|r|^2 < 0 at once: CG cannot take a step, so the
    oracle stops with EBREAKDOWN before the first product with A, x = 0."""
    shape = (1, 5, 7)
    bands = O.assemble(rand_kappa(shape, 171), W.BC_ALL_DIRICHLET)
    b = W.rhs_uniform(7, 5, 1, 172)
    x, it, rr, st, _ = O.pcg(bands, _identity_factors(shape, -1.0), b, 1e-8, 50)
    assert st == O.EBREAKDOWN and it == 0 and np.all(x == 0.0) and rr == 1.0
    x, it, rr, st = O.pcg_with(bands, lambda r: -r, b, 1e-8, 50)
    assert st == O.EBREAKDOWN and it == 0 and np.all(x == 0.0)


def test_pcg_breaks_down_on_a_negative_definite_matrix():
    """With A negative definite and B = I, p.Ap = -p'(-A)p < 0 in the first
    step: EBREAKDOWN before any update, x = 0."""
    shape = (1, 5, 7)
    d, ax, ay, az = O.assemble(rand_kappa(shape, 173), W.BC_ALL_DIRICHLET)
    neg = (-d, -ax, -ay, -az)
    b = W.rhs_uniform(7, 5, 1, 174)
    x, it, rr, st, _ = O.pcg(neg, _identity_factors(shape, 1.0), b, 1e-8, 50)
    assert st == O.EBREAKDOWN and it == 0 and np.all(x == 0.0)
    x, it, rr, st = O.pcg_with(neg, lambda r: r.copy(), b, 1e-8, 50)
    assert st == O.EBREAKDOWN and it == 0


def test_pcg_breaks_down_when_rz_turns_negative():
    """A preconditioner that is positive on the first residual and negative on
    the second: z = s(k) r with s = +1 for the first call, -1 after.  Step 1
    is the steepest-descent step; then r.z < 0 and the oracle stops with
    EBREAKDOWN after exactly one iteration, x = that step's iterate."""
    shape = (2, 4, 5)
    bands = O.assemble(rand_kappa(shape, 175), W.BC_ALL_DIRICHLET)
    b = W.rhs_uniform(5, 4, 2, 176)
    calls = []

    def flip(r):
        calls.append(1)
        return r.copy() if len(calls) == 1 else -r
    x, it, rr, st = O.pcg_with(bands, flip, b, 1e-12, 50)
    assert st == O.EBREAKDOWN and it == 1
    Ab = O.spmv(bands, b)
    alpha = np.dot(b.ravel(), b.ravel()) / np.dot(b.ravel(), Ab.ravel())
    np.testing.assert_allclose(x, alpha * b, rtol=1e-13)


# --------------------------------------------------------------------------
# ILU(0) smoother and the combination preconditioner (Sec. 3, eq. com)
# --------------------------------------------------------------------------

def _dense_ilu(bands, dt, nblocks):
    """B_ILU = (Dt + L) Dt^{-1} (Dt + U) formed densely from the oracle's dt and
    the kept strict parts of A (couplings across row M = floor(N/2) dropped)."""
    A = R.dense_from_bands(bands)
    N = A.shape[0]
    M = N // 2
    At = A.copy()
    if nblocks == 2:
        At[:M, M:] = 0.0
        At[M:, :M] = 0.0
    L = np.tril(At, -1)
    D = np.diag(dt.ravel())
    return (D + L) @ np.linalg.inv(D) @ (D + L.T), At


@pytest.mark.parametrize("nblocks", [1, 2])
@pytest.mark.parametrize("shape", [(3, 4, 5), (5, 3, 2), (1, 5, 7), (2, 3, 3)])
def test_ilu0_matches_matrix_on_its_pattern(shape, nblocks):
    """The defining property of ILU(0): L D^{-1} U reproduces the (block-diagonal)
    matrix on every position of its sparsity pattern; fill appears only outside."""
    bands = O.assemble(rand_kappa(shape, 131), W.BC_Z0_DIRICHLET)
    dt, st = O.ilu0(bands, nblocks)
    assert st == 0 and np.all(dt > 0)
    B, At = _dense_ilu(bands, dt, nblocks)
    pattern = At != 0
    np.testing.assert_allclose(B[pattern], At[pattern], rtol=1e-12, atol=1e-12 * np.abs(At).max())
    if nblocks == 2:
        M = At.shape[0] // 2
        assert np.abs(B[:M, M:]).max() == 0.0 and np.abs(B[M:, :M]).max() == 0.0
    z = O.ilu0_apply(bands, dt, np.ones(shape), nblocks)
    np.testing.assert_allclose(B @ z.ravel(), np.ones(At.shape[0]), rtol=1e-10, atol=1e-10)


def test_ilu0_is_exact_on_a_line():
    """A tridiagonal matrix has no ILU(0) fill: one block gives B_ILU = A."""
    bc = np.array([0, 0, 1, 1, 1, 1], dtype=np.int32)
    kappa = rand_kappa((1, 1, 11), 141)
    bands = O.assemble(kappa, bc)
    dt, _ = O.ilu0(bands, 1)
    r = np.random.default_rng(5).standard_normal((1, 1, 11))
    A = R.assemble_dense(kappa, bc)
    np.testing.assert_allclose(O.ilu0_apply(bands, dt, r, 1).ravel(), np.linalg.solve(A, r.ravel()),
                               rtol=1e-11)


@pytest.mark.parametrize("mode", ["newton", "diag"])
def test_combination_error_propagation(mode):
    """eq. com is equivalent to I - Bc^{-1} A = (I - B^{-1} A)(I - B_ILU^{-1} A)."""
    shape = (3, 4, 4)
    kappa = rand_kappa(shape, 151, contrast=2.0)
    bands = O.assemble(kappa, W.BC_ALL_DIRICHLET)
    F = O.setup(bands, mode=mode)
    dt, _ = O.ilu0(bands, 2)
    A = R.assemble_dense(kappa, W.BC_ALL_DIRICHLET)
    N = A.shape[0]
    Bc = np.zeros((N, N))
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        Bc[:, c] = O.combo_apply(bands, F, dt, e.reshape(shape)).ravel()
    Bi = dense_Binv(F, shape)
    Bilu, _ = _dense_ilu(bands, dt, 2)
    I = np.eye(N)
    lhs = I - Bc @ A
    rhs = (I - Bi @ A) @ (I - np.linalg.solve(Bilu, A))
    np.testing.assert_allclose(lhs, rhs, atol=1e-10)


def test_pcg_with_combination_matches_dense_solve():
    shape = (8, 7, 6)
    kappa = W.kappa_subcubes(6, 7, 8, 161, cubes=2)
    bands = O.assemble(kappa, W.BC_Z0_DIRICHLET)
    F = O.setup(bands, mode="newton")
    dt, _ = O.ilu0(bands, 2)
    b = W.rhs_uniform(6, 7, 8, 162)
    x, it, rr, st, _ = O.pcg(bands, F, b, 1e-11, 300, dt=dt)
    assert st == 0 and rr <= 1e-11
    A = R.assemble_dense(kappa, W.BC_Z0_DIRICHLET)
    xr = np.linalg.solve(A, b.ravel())
    assert np.linalg.norm(x.ravel() - xr) <= 10 * np.linalg.cond(A) * 1e-11 * np.linalg.norm(xr)
