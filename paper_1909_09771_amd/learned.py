"""The learned filter vector: training targets, training and evaluation.

Sec. 1 of arXiv:1909.09771: the preconditioner B(t) satisfies B t = A t, so a
filter vector t close to A's eigenvectors of smallest eigenvalue should serve
that end of the spectrum better than the rowsum choice t = 1.  Here a small 3D
network (FilterNet, kernels in ntd_cnn.hip) predicts t from kappa.

* Targets, two kinds:
  - binva_targets: the eigenvector of B^{-1}A (B = B(t = 1)) of smallest
    eigenvalue, by inverse iteration in the library (ntd_filter_target), the
    error component the filtered iteration damps slowest (Sec. 1), clipped
    below at 1e-3 (it can change sign);
  - eigen_targets: the lowest eigenvector of A, by inverse iteration
    v <- A^{-1} v / max(A^{-1} v) from v = 1, every solve a batched FP64 PCG of
    the library (B(1), diagonal Schur blocks), clipped below at 1e-3.  A is a
    symmetric M-matrix, so this eigenvector is positive.
* Training: Adam on mean (t - t*)^2, one field per step.
* Evaluation: PCG iterations and time to a tolerance with t = 1 and with the
  predicted t on held-out fields.  If the factorization with the predicted t
  loses a positive pivot, t = 1 is used (and reported).

Every convolution, loss, gradient, optimizer step, factorization, PCG,
inverse iteration and normalisation runs in the library's kernels.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import ENOTSPD, OK, Batch, FilterNet, NTDError, Solver, vec_normalize


def eigen_targets(kappas, bcs, iters: int = 20, tol: float = 1e-6, floor: float = 1e-3,
                  maxit: int = 2000, accept: float = 1e-4):
    """Lowest-eigenvector targets for a list of fields (float64 CUDA tensors).
    Each inner solve runs to a true relative residual <= tol; the iteration
    damps the error of every solve by the eigenvalue ratio, so the target
    carries an error of order tol.  High-contrast fields can have an attainable
    accuracy above tol: an entry that stops without converging (out of
    iterations, or p'Ap lost to rounding) is still used if its true relative
    residual is <= accept."""
    B = Batch(kappas, bcs, nrhs=1, prec="fp64", schur="diag")
    try:
        vs = [torch.ones_like(k) for k in kappas]
        for _ in range(iters):
            xs, its, rrs, sts = B.pcg(vs, tol=tol, maxit=maxit)
            bad = [(e, st, rrs[e], its[e]) for e, st in enumerate(sts)
                   if st != OK and not rrs[e] <= accept]
            if bad:
                raise RuntimeError("inverse iteration: PCG failed (field, status, relres, "
                                   "iterations): %s" % bad)
            for x in xs:
                vec_normalize(x)           # largest entry +1 (the iterates stay positive)
            vs = xs
    finally:
        B.close()
    for v in vs:
        vec_normalize(v, floor)
    return vs


def binva_targets(kappas, bcs, starts, schur: str = "newton", outer: int = 20,
                  inner_tol: float = 1e-10, inner_maxit: int = 20000, floor: float = 1e-3,
                  progress=None):
    """Smallest-eigenvalue eigenvectors of B^{-1}A, B = B(t = 1) with the given
    Schur block, clipped below at floor (ntd_filter_target), from the start
    vectors `starts` (t = 1 itself is an eigenvector of B(1)^{-1}A, since
    B t = A t, so a start must carry other components); returns the targets and
    the eigenvalue estimates.  progress(i, lam, inner_steps, seconds), if
    given, is called after each field."""
    out, lams = [], []
    for i, (k, bc, v0) in enumerate(zip(kappas, bcs, starts)):
        t0 = time.perf_counter()
        S = Solver(k, bc, prec="fp64", schur=schur)
        try:
            t, inner, lam = S.filter_target(v0, outer=outer, inner_tol=inner_tol,
                                            inner_maxit=inner_maxit, floor=floor)
        finally:
            S.close()
        out.append(t)
        lams.append(lam)
        if progress is not None:
            progress(i, lam, inner, time.perf_counter() - t0)
    return out, lams


def train_on_binva_targets(kappas, bcs, starts, params, epochs: int = 20, lr: float = 2e-3,
                           outer: int = 8, inner_tol: float = 1e-6, progress=None):
    """A network trained on the method's own targets: for each field the
    smallest-eigenvalue eigenvector of B(1)^{-1}A with Newton Schur blocks
    (binva_targets from `starts`, `outer` inverse iterations, inner solves to
    inner_tol), then Adam for `epochs` epochs from the initial weights
    `params`.  Returns (net, loss per epoch, seconds spent on the targets,
    eigenvalue estimates)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tgt, lams = binva_targets(kappas, bcs, starts, schur="newton", outer=outer,
                              inner_tol=inner_tol, inner_maxit=200000, progress=progress)
    torch.cuda.synchronize()
    t_targets = time.perf_counter() - t0
    net = FilterNet(params, device=kappas[0].device)
    hist = train(net, kappas, tgt, epochs, lr)
    net.release_workspaces()
    return net, hist, t_targets, lams


def train(net: FilterNet, kappas, targets, epochs: int, lr: float, seed: int = 0):
    """Adam over the fields in a seeded random order each epoch; returns the
    mean loss of every epoch."""
    rng = np.random.default_rng(seed)
    history = []
    for _ in range(epochs):
        tot = 0.0
        for i in rng.permutation(len(kappas)):
            tot += net.train_step(kappas[i], targets[i], lr)
        history.append(tot / len(kappas))
    return history


def solve_with(kappa, bc, b, t, tol, maxit, prec, schur, smoother):
    """Setup + PCG; returns dict(iters, relres, status, seconds, fallback)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fallback = False
    try:
        S = Solver(kappa, bc, t=t, prec=prec, schur=schur, smoother=smoother)
    except NTDError as e:
        if e.status != ENOTSPD or t is None:
            raise
        fallback = True
        S = Solver(kappa, bc, t=None, prec=prec, schur=schur, smoother=smoother)
    x, it, rr, st = S.pcg(b, tol=tol, maxit=maxit)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    S.close()
    return dict(iters=int(it), relres=float(rr), status=int(st), seconds=el, fallback=fallback)


def compare(net: FilterNet, kappa, bc, b, tol=1e-8, maxit=5000, prec="mixed", schur="newton",
            smoother="ilu0"):
    """PCG with t = 1 and with the network's t (its prediction timed with it)."""
    ones = solve_with(kappa, bc, b, None, tol, maxit, prec, schur, smoother)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t = net.predict(kappa)
    torch.cuda.synchronize()
    pred_s = time.perf_counter() - t0
    learned = solve_with(kappa, bc, b, t, tol, maxit, prec, schur, smoother)
    learned["seconds"] += pred_s
    learned["predict_s"] = pred_s
    learned["t_max_over_min"] = float(t.max() / t.min())
    return dict(ones=ones, learned=learned)
