"""Pin of the dense reference of the filter-vector target (tests/target_ref.py,
inverse iteration on B^{-1}A built from the oracle) against scipy's
generalized symmetric eigensolver: after enough steps its iterate is the
eigenvector of the pencil (A, B) of smallest eigenvalue, up to scale, and its
eigenvalue estimate is that eigenvalue."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from tests.target_ref import filter_target


def test_inverse_iteration_reaches_the_smallest_generalised_eigenvector():
    """Newton blocks: B >= A, the spectrum of B^{-1}A lies in (0, 1] and t = 1
    sits at its top (B t = A t); from a start with components along the
    bottom the iteration converges there."""
    kappa = W.kappa_subcubes(6, 5, 7, 7, cubes=2)
    v0 = W.filter_random(6, 5, 7, 8)
    t, lam, A, Binv = filter_target(kappa, W.BC_Z0_DIRICHLET, "newton", 200, -10.0, v0)
    B = np.linalg.inv(Binv)
    w, V = sla.eigh(A, 0.5 * (B + B.T))
    v = V[:, 0] / V[np.argmax(np.abs(V[:, 0])), 0]
    assert w[0] < w[1] * 0.999          # separated, so the iteration converges
    assert abs(lam - w[0]) <= 1e-10 * w[0]
    assert np.abs(t.ravel() - v).max() <= 1e-8


def test_diagonal_blocks_keep_the_filter_vector_at_the_bottom():
    """Diagonal blocks: B <= A, the spectrum lies in [1, inf) and t = 1 is an
    eigenvector of eigenvalue 1 (B t = A t), the smallest; the iteration stays."""
    kappa = W.kappa_subcubes(6, 5, 7, 7, cubes=2)
    t, lam, A, Binv = filter_target(kappa, W.BC_Z0_DIRICHLET, "diag", 20, -10.0)
    assert abs(lam - 1.0) <= 1e-12
    assert np.abs(t - 1.0).max() <= 1e-10


def test_the_rowsum_vector_is_an_eigenvector_of_the_newton_preconditioned_operator():
    """B t = A t makes t = 1 an eigenvector of B^{-1}A (eigenvalue 1), so an
    inverse iteration started exactly at 1 stays there: the start must carry
    other components."""
    kappa = W.kappa_subcubes(6, 5, 7, 7, cubes=2)
    t, lam, A, Binv = filter_target(kappa, W.BC_Z0_DIRICHLET, "newton", 1, -10.0)
    assert abs(lam - 1.0) <= 1e-10 and np.abs(t - 1.0).max() <= 1e-10
