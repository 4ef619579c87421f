"""Parity at the benchmark's full size, in the configuration it times.

Workload jump256: 256^3 grid, kappa on 8^3 subcubes 10^U(-3,3) (seed 601),
Dirichlet at z = 0 and Neumann on the other faces, b ~ U[-1,1] (seed 602),
t = 1, Newton Schur blocks with the ILU(0) combination of eq. com (Sec. 3) and
with the symmetric ILU(0)-B-ILU(0) combination (the benchmark's default).
The FP64 oracle computes the assembly, the SpMV, the three-level setup, the
ILU(0) factorization and one application of each preconditioner at this size
in seconds, so those are compared element by element.  PCG to 1e-8 is checked
through the true residual of the GPU's solution, recomputed by the oracle.
Tolerances are those of the small-size parity tests.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def G(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def C(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def full():
    import paper_1909_09771_amd as P
    w = W.workload("jump256")
    bands = O.assemble(w["kappa"], w["bc"])
    F = O.setup(bands, mode="newton")
    dt, st = O.ilu0(bands, 2)
    assert st == 0
    print("jump256: oracle setup done", flush=True)
    kappa = G(w["kappa"])
    solvers = {prec: P.Solver(kappa, w["bc"], prec=prec, schur="newton", smoother="ilu0")
               for prec in ("mixed", "fp64")}
    for prec in ("mixed", "fp64"):
        solvers[prec + "-sym"] = P.Solver(kappa, w["bc"], prec=prec, schur="newton",
                                          smoother="ilu0sym")
    print("jump256: GPU setups done", flush=True)
    yield dict(w=w, bands=bands, F=F, dt=dt, S=solvers)
    for S in solvers.values():
        S.close()
    torch.cuda.empty_cache()


def test_full_assembly_and_spmv(full):
    S = full["S"]["mixed"]
    for name, want in zip(("d", "ax", "ay", "az"), full["bands"]):
        np.testing.assert_allclose(C(S.export(name)), want, rtol=1e-15, atol=0, err_msg=name)
    b = full["w"]["b"]
    assert relmax(C(S.spmv(G(b))), O.spmv(full["bands"], b)) <= 1e-14


def test_full_ilu0(full):
    r = full["w"]["b"]
    want = O.ilu0_apply(full["bands"], full["dt"], r, 2)
    # FP64 to 1e-12; MIXED reads the sweeps' coefficients in FP32: 1e-5
    for prec, tol in (("fp64", 1e-12), ("mixed", 1e-5)):
        S = full["S"][prec]
        np.testing.assert_allclose(C(S.export("dt")), full["dt"], rtol=1e-13)
        err = relmax(C(S.apply_ilu0(G(r))), want)
        print("jump256 ILU(0) apply %s: %.2e" % (prec, err))
        assert err <= tol


@pytest.mark.parametrize("prec,tol", [("mixed", 1e-5), ("fp64", 1e-9)])
def test_full_apply(full, prec, tol):
    S = full["S"][prec]
    r = np.random.default_rng(811).uniform(-1.0, 1.0, full["w"]["b"].shape)
    want = O.apply(full["F"], r)
    assert relmax(C(S.apply_ntd(G(r))), want) <= tol
    want = O.combo_apply(full["bands"], full["F"], full["dt"], r, 2)
    assert relmax(C(S.apply(G(r))), want) <= tol


def test_full_filter_property_fp64(full):
    """B t = A t (Sec. 1, eq. filter) with t = 1: B^{-1}(A 1) = 1 up to
    rounding amplified by the kappa contrast of 10^6."""
    S = full["S"]["fp64"]
    one = np.ones_like(full["w"]["b"])
    got = C(S.apply_ntd(G(O.spmv(full["bands"], one))))
    assert np.abs(got - 1.0).max() <= 1e-8


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_full_pcg_true_residual(full, prec):
    S = full["S"][prec]
    b = full["w"]["b"]
    x, it, rr, st = S.pcg(G(b), tol=1e-8, maxit=2000)
    print("jump256 PCG %s: %d iterations, relres %.3e" % (prec, it, rr), flush=True)
    assert st == 0 and rr <= 1e-8
    res = b - O.spmv(full["bands"], C(x))
    assert np.linalg.norm(res) <= 1.01e-8 * np.linalg.norm(b)


@pytest.mark.parametrize("prec,tol", [("mixed", 1e-5), ("fp64", 1e-9)])
def test_full_apply_symmetric(full, prec, tol):
    S = full["S"][prec + "-sym"]
    r = np.random.default_rng(812).uniform(-1.0, 1.0, full["w"]["b"].shape)
    want = O.sym_combo_apply(full["bands"], full["F"], full["dt"], r, 2)
    assert relmax(C(S.apply(G(r))), want) <= tol


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_full_pcg_symmetric_true_residual(full, prec):
    S = full["S"][prec + "-sym"]
    b = full["w"]["b"]
    x, it, rr, st = S.pcg(G(b), tol=1e-8, maxit=2000)
    print("jump256 PCG symmetric %s: %d iterations, relres %.3e" % (prec, it, rr), flush=True)
    assert st == 0 and rr <= 1e-8
    res = b - O.spmv(full["bands"], C(x))
    assert np.linalg.norm(res) <= 1.01e-8 * np.linalg.norm(b)
