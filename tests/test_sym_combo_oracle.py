"""Pins of the symmetric ILU(0)-B-ILU(0) combination in the oracle
(oracle.sym_combo_apply) and of the generic oracle PCG (oracle.pcg_with).

M^{-1} = z1 -> z2 -> z expands to C (2 B_ILU - A) C + (I - C A) B^{-1} (I - A C)
with C = B_ILU^{-1}: built here from dense matrices (columns of the oracle's
B^{-1} and B_ILU^{-1}, A from the bands), not by composing the three steps.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
import workloads as W


def dense_ops(kappa, bc, mode):
    bands = O.assemble(kappa, bc)
    F = O.setup(bands, mode=mode)
    dt, st = O.ilu0(bands)
    assert st == 0
    N = kappa.size
    E = np.eye(N)
    shape = kappa.shape
    cols = lambda f: np.stack([f(E[j].reshape(shape)).ravel() for j in range(N)], axis=1)
    A = cols(lambda v: O.spmv(bands, v))
    Binv = cols(lambda v: O.apply(F, v))
    Cinv = cols(lambda v: O.ilu0_apply(bands, dt, v))
    M = cols(lambda v: O.sym_combo_apply(bands, F, dt, v))
    return bands, F, dt, A, Binv, Cinv, M


FIELDS = [("spheres", W.kappa_spheres(5, 4, 6, 301, count=6, r_lo=0.15, r_hi=0.3)),
          ("subcubes", W.kappa_subcubes(5, 4, 6, 77, cubes=2))]


@pytest.mark.parametrize("mode", ["newton", "diag"])
@pytest.mark.parametrize("name,kappa", FIELDS)
def test_sym_combo_closed_form_symmetry_and_spd(name, kappa, mode):
    bc = W.BC_ALL_DIRICHLET
    _, _, _, A, Binv, C, M = dense_ops(kappa, bc, mode)
    I = np.eye(A.shape[0])
    BI = np.linalg.inv(C)
    want = C @ (2 * BI - A) @ C + (I - C @ A) @ Binv @ (I - A @ C)
    assert np.abs(M - want).max() <= 1e-10 * np.abs(want).max()
    assert np.abs(M - M.T).max() <= 1e-10 * np.abs(M).max()       # B, B_ILU, A symmetric
    assert np.abs(C - C.T).max() <= 1e-10 * np.abs(C).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0.0


def test_pcg_with_matches_a_dense_solve():
    kappa = FIELDS[0][1]
    bands, F, dt, A, _, _, _ = dense_ops(kappa, W.BC_ALL_DIRICHLET, "diag")
    b = W.rhs_uniform(*kappa.shape[::-1], 5)
    x, it, rr, st = O.pcg_with(bands, lambda r: O.sym_combo_apply(bands, F, dt, r), b, 1e-12, 200)
    assert st == O.OK and rr <= 1e-12
    want = np.linalg.solve(A, b.ravel())
    assert np.linalg.norm(x.ravel() - want) <= 1e-9 * np.linalg.norm(want) * np.linalg.cond(A)
    # plain B through the same loop takes the C oracle's iterations (+-1)
    x2, it2, rr2, st2 = O.pcg_with(bands, lambda r: O.apply(F, r), b, 1e-10, 200)
    x3, it3, rr3, st3, _ = O.pcg(bands, F, b, 1e-10, 200)
    assert st2 == st3 == O.OK and abs(it2 - it3) <= 1


@pytest.mark.parametrize("mode", ["newton", "diag"])
@pytest.mark.parametrize("name,kappa", FIELDS)
def test_c_sym_combo_equals_the_dense_closed_form(name, kappa, mode):
    """The C oracle's symmetric combination (orc_sym_combo_apply) against the
    closed form built from dense B^{-1}, B_ILU^{-1} and A."""
    bc = W.BC_ALL_DIRICHLET
    bands, F, dt, A, Binv, C, _ = dense_ops(kappa, bc, mode)
    I = np.eye(A.shape[0])
    want = C @ (2 * np.linalg.inv(C) - A) @ C + (I - C @ A) @ Binv @ (I - A @ C)
    E = np.eye(A.shape[0])
    got = np.stack([O.sym_combo_apply_c(bands, F, dt, E[j].reshape(kappa.shape)).ravel()
                    for j in range(A.shape[0])], axis=1)
    assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()


def test_c_pcg_with_sym_combo_matches_dense_solve_and_python_loop():
    kappa = FIELDS[1][1]
    bands, F, dt, A, _, _, _ = dense_ops(kappa, W.BC_ALL_DIRICHLET, "newton")
    b = W.rhs_uniform(*kappa.shape[::-1], 6)
    x, it, rr, st, _ = O.pcg(bands, F, b, 1e-12, 200, dt=dt, smoother="ilu0sym")
    assert st == O.OK and rr <= 1e-12
    want = np.linalg.solve(A, b.ravel())
    assert np.linalg.norm(x.ravel() - want) <= 1e-9 * np.linalg.norm(want) * np.linalg.cond(A)
    x2, it2, rr2, st2 = O.pcg_with(bands, lambda r: O.sym_combo_apply(bands, F, dt, r), b, 1e-12, 200)
    assert st2 == O.OK and abs(it - it2) <= 1
