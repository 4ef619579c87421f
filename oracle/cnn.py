"""FP64 CPU oracle of the learned filter vector: a small 3D CNN that maps the
coefficient field kappa to a filter vector t > 0, and its training target.

TEST INFRASTRUCTURE ONLY: the test-suite and the smoke check use this module;
the GPU library never imports or runs it, and the two share no code.

Why a filter vector is learned (Sec. 1 of arXiv:1909.09771): B(t) satisfies
B t = A t, and the closer t is to the eigenvectors of A with the smallest
eigenvalues, the better B(t) treats that end of the spectrum; t = 1 is the
classical rowsum choice.  The network reads only kappa (a field that may be
rescaled without changing A's eigenvectors, so the feature is log10 kappa minus
its mean) and predicts a positive t.

Network (one layer = 3x3x3 cross-correlation with zero padding, plus a bias):
    H0 = feature(kappa)                       1 channel
    H_l = relu(conv_l(H_{l-1}))  l = 1, 2, 3  16 channels each
    y = conv_4(H3)                            1 channel
    t = softplus(y) + EPS_T
Loss: mean over the grid of (t - t*)^2 against the target t*.

Parameters are one flat float32 vector: for each layer, W[cout][tap][cin] then
b[cout], where tap = 9 (dz+1) + 3 (dy+1) + (dx+1) indexes the neighbour offset
(dz, dy, dx) in {-1, 0, 1}^3 and the layer reads H[z+dz, y+dy, x+dx].

Precision: the GPU kernels multiply bfloat16 operands and accumulate in
float32.  With exact=False this oracle rounds to bfloat16 (round to nearest
even, through float32) at the same points -- the feature, the weights, each
hidden activation and each back-propagated gradient map -- and accumulates in
float64; with exact=True nothing is rounded (used by the finite-difference and
library pins).

Arrays are numpy float64 of shape (nz, ny, nx) for scalar fields and
(nz, ny, nx, C) for channel fields (channels last).
"""
from __future__ import annotations

import numpy as np

LAYERS = [(1, 16), (16, 16), (16, 16), (16, 1)]       # (cin, cout)
TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
EPS_T = 1.0e-3
FEATURE_SCALE = 3.0


def param_count() -> int:
    return sum(co * 27 * ci + co for ci, co in LAYERS)


def layer_views(params):
    """[(W[cout][27][cin], b[cout])] as float64 copies of the flat vector."""
    p = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for ci, co in LAYERS:
        W = p[o:o + co * 27 * ci].reshape(co, 27, ci)
        o += co * 27 * ci
        b = p[o:o + co]
        o += co
        out.append((W.copy(), b.copy()))
    assert o == p.size
    return out


def flatten(grads) -> np.ndarray:
    return np.concatenate([np.concatenate([dW.ravel(), db.ravel()]) for dW, db in grads])


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) through float32; returns float64."""
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def shifted(X, off):
    """S[z, y, x] = X[z+dz, y+dy, x+dx], zero where the neighbour leaves the grid."""
    dz, dy, dx = off
    nz, ny, nx = X.shape[:3]
    S = np.zeros_like(X)
    zs, zd = slice(max(dz, 0), nz + min(dz, 0)), slice(max(-dz, 0), nz + min(-dz, 0))
    ys, yd = slice(max(dy, 0), ny + min(dy, 0)), slice(max(-dy, 0), ny + min(-dy, 0))
    xs, xd = slice(max(dx, 0), nx + min(dx, 0)), slice(max(-dx, 0), nx + min(-dx, 0))
    S[zd, yd, xd] = X[zs, ys, xs]
    return S


def conv(X, W, b=None):
    """Z[v, co] = b[co] + sum_tap sum_ci W[co, tap, ci] X[v + off(tap), ci]."""
    co = W.shape[0]
    Z = np.zeros(X.shape[:3] + (co,))
    for tap, off in enumerate(TAPS):
        Z += shifted(X, off) @ W[:, tap, :].T
    if b is not None:
        Z += b
    return Z


def conv_adjoint(G, W):
    """The adjoint of conv in its input: X[v, ci] = sum_tap sum_co W[co, tap, ci] G[v - off(tap), co]."""
    ci = W.shape[2]
    X = np.zeros(G.shape[:3] + (ci,))
    for tap, (dz, dy, dx) in enumerate(TAPS):
        X += shifted(G, (-dz, -dy, -dx)) @ W[:, tap, :]
    return X


def weight_grad(H, G):
    """dW[co, tap, ci] = sum_v G[v, co] H[v + off(tap), ci]; db[co] = sum_v G[v, co]."""
    co, ci = G.shape[3], H.shape[3]
    Gm = G.reshape(-1, co)
    dW = np.zeros((co, 27, ci))
    for tap, off in enumerate(TAPS):
        dW[:, tap, :] = Gm.T @ shifted(H, off).reshape(-1, ci)
    return dW, Gm.sum(axis=0)


def feature(kappa, exact=False):
    L = np.log10(np.asarray(kappa, dtype=np.float64))
    x = (L - L.mean()) / FEATURE_SCALE
    return (x if exact else bf16(x))[..., None]


def softplus(y):
    return np.logaddexp(0.0, y)


def sigmoid(y):
    return 0.5 * (1.0 + np.tanh(0.5 * y))


def forward(params, kappa, exact=False) -> dict:
    """Returns dict(H=[H0, H1, H2, H3], y, t) (y and t of shape (nz, ny, nx))."""
    rnd = (lambda a: a) if exact else bf16
    layers = [(rnd(W), b) for W, b in layer_views(params)]
    H = [feature(kappa, exact)]
    for l in range(3):
        W, b = layers[l]
        H.append(rnd(np.maximum(conv(H[-1], W, b), 0.0)))
    W, b = layers[3]
    y = conv(H[3], W, b)[..., 0]
    return dict(H=H, y=y, t=softplus(y) + EPS_T, layers=layers)


def loss_grad(params, kappa, target, exact=False):
    """Loss mean((t - t*)^2) and its gradient in the flat parameter layout."""
    rnd = (lambda a: a) if exact else bf16
    f = forward(params, kappa, exact)
    H, y, t, layers = f["H"], f["y"], f["t"], f["layers"]
    n = t.size
    diff = t - np.asarray(target, dtype=np.float64)
    loss = float(np.sum(diff * diff) / n)
    G = rnd(2.0 * diff * sigmoid(y) / n)[..., None]      # d loss / d y
    grads = [None] * 4
    for l in (3, 2, 1, 0):
        grads[l] = weight_grad(H[l], G)
        if l > 0:
            G = rnd(conv_adjoint(G, layers[l][0]) * (H[l] > 0))
    return loss, flatten(grads)


def adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015) with bias-corrected moments."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def eigen_target(bands, iters: int = 20, floor: float = 1.0e-3):
    """Target filter vector: the eigenvector of A with the smallest eigenvalue,
    by inverse iteration v <- A^{-1} v / max(A^{-1} v) from v = 1 (A is a
    symmetric M-matrix, so A^{-1} > 0 and every iterate stays positive),
    clipped below at `floor`.  bands = (d, ax, ay, az) from the assembly; the
    solve is a sparse direct factorisation (scipy)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    d, ax, ay, az = (np.asarray(a, dtype=np.float64) for a in bands)
    nz, ny, nx = d.shape
    N = d.size
    A = sp.diags([d.ravel()], [0], shape=(N, N), format="csr")
    for band, off in ((ax, 1), (ay, nx), (az, nx * ny)):
        u = band.ravel()[:N - off]
        A = A + sp.diags([u, u], [off, -off], shape=(N, N), format="csr")
    lu = spl.splu(A.tocsc())
    v = np.ones(N)
    for _ in range(iters):
        v = lu.solve(v)
        v /= v.max()
    return np.maximum(v, floor).reshape(nz, ny, nx)
