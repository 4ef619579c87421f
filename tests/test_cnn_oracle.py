"""Pins of the learned-filter oracle (oracle/cnn.py) against things other than
itself: scipy's n-d correlation, the adjoint and bilinear identities of a
convolution, central finite differences of the loss, torch's bfloat16 cast,
Adam's closed-form first step and a dense symmetric eigensolver."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.linalg
import scipy.ndimage
import torch

import oracle as O
import oracle.cnn as C
import workloads as W


def rand_field(shape, ch, seed):
    return np.random.default_rng(seed).uniform(-1, 1, size=tuple(shape) + (ch,))


def test_param_count():
    assert W.CNN_LAYERS == C.LAYERS and W.cnn_init_params(0).size == C.param_count()
    assert C.param_count() == 16 * 27 + 16 + 2 * (16 * 27 * 16 + 16) + 27 * 16 + 1 == 14737


def test_bf16_matches_torch_cast():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 10, 4000), rng.uniform(-1e-30, 1e-30, 100),
                        [0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 65504.0]])
    want = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(C.bf16(x), want)
    assert C.bf16(1.0 + 2.0 ** -8) == 1.0 and C.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


@pytest.mark.parametrize("ci,co", [(1, 16), (16, 16), (16, 1), (3, 2)])
def test_conv_matches_scipy_correlate(ci, co):
    shape = (5, 6, 7)
    X = rand_field(shape, ci, 11)
    Wt = np.random.default_rng(12).normal(size=(co, 27, ci))
    b = np.random.default_rng(13).normal(size=co)
    Z = C.conv(X, Wt, b)
    for o in range(co):
        want = np.full(shape, b[o])
        for c in range(ci):
            want += scipy.ndimage.correlate(X[..., c], Wt[o, :, c].reshape(3, 3, 3),
                                            mode="constant", cval=0.0)
        np.testing.assert_allclose(Z[..., o], want, rtol=1e-12, atol=1e-12)


def test_conv_adjoint_identity():
    shape = (4, 5, 6)
    X, G = rand_field(shape, 16, 21), rand_field(shape, 3, 22)
    Wt = np.random.default_rng(23).normal(size=(3, 27, 16))
    lhs = np.sum(C.conv(X, Wt) * G)
    rhs = np.sum(X * C.conv_adjoint(G, Wt))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_weight_grad_bilinear_identity():
    """conv is linear in W, so <conv(X, W), G> = <W, dW(X, G)> and sum(G) is db."""
    shape = (3, 4, 5)
    X, G = rand_field(shape, 2, 31), rand_field(shape, 4, 32)
    Wt = np.random.default_rng(33).normal(size=(4, 27, 2))
    dW, db = C.weight_grad(X, G)
    assert abs(np.sum(C.conv(X, Wt) * G) - np.sum(Wt * dW)) <= 1e-11 * np.abs(dW).sum()
    np.testing.assert_allclose(db, G.reshape(-1, 4).sum(0), rtol=1e-13)


def test_feature_ignores_a_rescaling_of_kappa():
    k = W.kappa_subcubes(6, 5, 4, 7, cubes=2)
    np.testing.assert_allclose(C.feature(k, exact=True), C.feature(37.5 * k, exact=True),
                               atol=1e-14)


def test_softplus_and_sigmoid():
    y = np.linspace(-30, 30, 61)
    assert C.softplus(np.array([0.0]))[0] == pytest.approx(np.log(2.0), rel=1e-15)
    h = 1e-6
    np.testing.assert_allclose((C.softplus(y + h) - C.softplus(y - h)) / (2 * h), C.sigmoid(y),
                               rtol=1e-7, atol=1e-12)


def test_constant_kappa_gives_t_one_at_init():
    p = W.cnn_init_params(5)
    for exact in (True, False):
        t = C.forward(p, W.kappa_const(5, 4, 3, 2.0), exact=exact)["t"]
        np.testing.assert_allclose(t, 1.0, rtol=1e-6)


def test_loss_grad_matches_finite_differences():
    kappa = W.kappa_subcubes(5, 4, 3, 41, cubes=2, log10_lo=-2, log10_hi=2)
    target = np.random.default_rng(42).uniform(0.1, 1.0, kappa.shape)
    p = W.cnn_init_params(43).astype(np.float64)
    p += np.random.default_rng(44).normal(0, 0.05, p.size)   # biases off zero
    loss, g = C.loss_grad(p, kappa, target, exact=True)
    rng = np.random.default_rng(45)
    offs = np.cumsum([0] + [co * 27 * ci + co for ci, co in C.LAYERS])
    idx = np.concatenate([rng.choice(np.arange(offs[l], offs[l + 1]), 12, replace=False)
                          for l in range(4)] + [offs[1:] - 1])   # every layer, each last bias
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (C.loss_grad(pp, kappa, target, exact=True)[0]
              - C.loss_grad(pm, kappa, target, exact=True)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * abs(g).max() + 1e-5 * abs(fd), (i, fd, g[i])


def test_adam_first_step_moves_by_lr_times_sign():
    g = np.array([3.0, -0.5, 1e-3, -7.0])
    p, m, v = C.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    np.testing.assert_allclose(p, -0.01 * np.sign(g), rtol=1e-4)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


@pytest.mark.parametrize("bc", [W.BC_ALL_DIRICHLET, W.BC_Z0_DIRICHLET])
def test_eigen_target_is_lowest_eigenvector(bc):
    kappa = W.kappa_subcubes(6, 5, 4, 51, cubes=2, log10_lo=-1, log10_hi=1)
    bands = O.assemble(kappa, bc)
    d, ax, ay, az = bands
    N = d.size
    A = np.diag(d.ravel())
    for band, off in ((ax, 1), (ay, 6), (az, 30)):
        u = band.ravel()[:N - off]
        A += np.diag(u, off) + np.diag(u, -off)
    lam, vec = scipy.linalg.eigh(A)
    v = np.abs(vec[:, 0])
    v /= v.max()
    t = C.eigen_target(bands, iters=200, floor=0.0)
    np.testing.assert_allclose(t.ravel(), v, atol=1e-9)
    rate = lam[0] / lam[1]
    t20 = C.eigen_target(bands, iters=20, floor=1e-3)
    assert np.abs(t20.ravel() - np.maximum(v, 1e-3)).max() <= 10 * rate ** 20 + 1e-12
