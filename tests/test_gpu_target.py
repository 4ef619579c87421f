"""The filter-vector target of the library (ntd_filter_target: inverse
iteration on B^{-1}A, Sec. 1) and ntd_vec_normalize against dense references
built from the oracle's preconditioner.

Reference: B^{-1} formed densely from the oracle's apply (columns = applies to
unit vectors), A from the oracle's bands, and the iteration written out with
dense solves: v <- y / (entry of y of largest magnitude), y = (B^{-1}A)^{-1} v =
A^{-1} B v.  The GPU's inner solves run to 1e-13, so the two agree to about
1e-9 of the largest entry; the bar is 1e-7.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as O  # noqa: F401  (the dense reference builds on it)
import workloads as W
from tests.target_ref import filter_target as dense_target

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def G(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def C(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


CASES = [("jump", (6, 7, 8), "newton"), ("jump", (6, 7, 8), "diag"),
         ("spheres", (9, 8, 10), "newton"), ("layers", (10, 6, 5), "diag")]


def field(kind, shape):
    nz, ny, nx = shape
    if kind == "jump":
        return W.kappa_subcubes(nx, ny, nz, 7, cubes=2), W.BC_Z0_DIRICHLET.copy()
    if kind == "spheres":
        return (W.kappa_spheres(nx, ny, nz, 3, count=4, r_lo=0.15, r_hi=0.3, inside=1e3),
                W.BC_ALL_DIRICHLET.copy())
    return W.kappa_layers(nx, ny, nz, 5, layers=4, log10_lo=-2, log10_hi=2), W.BC_ALL_DIRICHLET.copy()


@pytest.mark.parametrize("kind,shape,schur", CASES)
def test_filter_target_matches_dense_inverse_iteration(kind, shape, schur):
    import paper_1909_09771_amd as P
    kappa, bc = field(kind, shape)
    v0 = W.filter_random(shape[2], shape[1], shape[0], 11)   # t = 1 itself is an eigenvector
    want, lam_want, A, Binv = dense_target(kappa, bc, schur, 20, 1e-3, v0)
    S = P.Solver(G(kappa), bc, prec="fp64", schur=schur)
    t, inner, lam = S.filter_target(G(v0), outer=20, inner_tol=1e-13, inner_maxit=2000,
                                    floor=1e-3)
    t = C(t)
    err = np.abs(t - want).max()
    ev = np.sort(np.linalg.eigvals(Binv @ A).real)
    print("%s %s %s: max |t - t_dense| %.2e, lambda %.6e (dense %.6e, smallest eigenvalue "
          "%.6e), %d inner steps, %.0f%% of the unclipped target below the floor"
          % (kind, shape, schur, err, lam, lam_want, ev[0], inner, 100 * np.mean(want <= 1e-3)))
    assert err <= 1e-7
    assert abs(lam - lam_want) <= 1e-7 * lam_want
    if schur == "newton":   # close to the bottom of the spectrum after 20 steps
        assert abs(lam - ev[0]) <= 1e-3 * ev[0]
    assert t.min() >= 1e-3 and abs(t.max() - 1.0) <= 1e-12


def test_vec_normalize():
    import paper_1909_09771_amd as P
    rng = np.random.default_rng(3)
    v = rng.standard_normal(100003)
    v[777] = -9.0                      # the entry of largest magnitude is negative
    g = G(v)
    sc = P.vec_normalize(g, floor=1e-3)
    want = np.maximum(v * (1.0 / -9.0), 1e-3)
    assert sc == pytest.approx(-1.0 / 9.0, rel=1e-15)
    assert np.array_equal(C(g), want)
    g2 = G(v)
    P.vec_normalize(g2)                # no clipping
    assert np.array_equal(C(g2), v * (1.0 / -9.0))
    with pytest.raises(P.NTDError):
        P.vec_normalize(G(np.zeros(10)))


@pytest.mark.parametrize("where", [0, 777, 100002])
def test_vec_normalize_rejects_nan_and_zero(where):
    """A NaN entry anywhere (first, inside, last element) wins the largest-
    magnitude reduction, so the scale is not finite and the call fails with
    NTD_EINVAL; so does an all-zero vector."""
    import paper_1909_09771_amd as P
    v = np.random.default_rng(4).standard_normal(100003)
    v[5000] = 50.0                     # a larger finite entry elsewhere
    v[where] = np.nan
    with pytest.raises(P.NTDError) as e:
        P.vec_normalize(G(v), floor=1e-3)
    assert e.value.status == P.EINVAL
    with pytest.raises(P.NTDError) as e:
        P.vec_normalize(G(np.zeros(4097)), floor=1e-3)
    assert e.value.status == P.EINVAL
