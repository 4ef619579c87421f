"""GPU-vs-oracle parity on the configurations the other parity files do not
cover, through the C ABI:

  * the plain method (Newton Schur blocks, no smoother) on the 32^3 Poisson
    problem with b ~ U[-1,1] -- PCG iterations against the oracle's;
  * the paper's test matrices (Sec. 3): Type 1 (skyscrapers), Type 2 as
    printed (an empty ring, kappa = 1) and the non-empty 1/(2 sqrt 2) ring, at
    40^3 with b = A x*: the B and eq. com applications element by element and
    eq. com PCG within one iteration of the oracle (FP64);
  * the 128^3 subcube field (Dirichlet at z = 0, Neumann elsewhere): the MIXED
    application element by element against the oracle, and MIXED and FP64
    PCG to 1e-8 side by side, the true residual of each solution recomputed
    by the oracle;
  * breakdown: factors of a negative definite B loaded into the handle make
    r.z < 0, and PCG stops with NTD_EBREAKDOWN before its first step.

Bars as in test_gpu_parity.py: |z - z_o| <= tol * max |z_o| with tol 1e-9
(FP64) and 1e-5 (MIXED); iterations +-1 in FP64.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def P():
    import paper_1909_09771_amd as lib
    return lib


def G(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def C(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_plain_newton_pcg_poisson32(prec):
    """The plain method of the 32^3 configuration: B alone with the Newton
    Schur blocks of Sec. 2.1, t = 1, PCG to 1e-8."""
    w = W.workload("poisson32")
    kappa, bc, b = w["kappa"], w["bc"], w["b"]
    S = P().Solver(G(kappa), bc, prec=prec, schur="newton")
    x, it, rr, st = S.pcg(G(b), tol=1e-8, maxit=500)
    bands = O.assemble(kappa, bc)
    xo, ito, rro, sto, _ = O.pcg(bands, O.setup(bands, mode="newton"), b, 1e-8, 500)
    print("plain Newton PCG poisson32 %s: %d iterations, oracle %d" % (prec, it, ito))
    assert st == P().OK and sto == O.OK and rr <= 1e-8
    assert abs(it - ito) <= (1 if prec == "fp64" else ito // 4 + 3)
    res = b - O.spmv(bands, C(x))
    assert np.linalg.norm(res) <= 1.01e-8 * np.linalg.norm(b)


PAPER_TYPES = ["paper1", "paper2", "paper2ring"]


@pytest.fixture(scope="module", params=PAPER_TYPES)
def paper40(request):
    n = 40
    w = W.scaled_workload(request.param, n)
    bands = O.assemble(w["kappa"], w["bc"])
    F = O.setup(bands, mode="newton")
    dt, st = O.ilu0(bands, 2)
    assert st == O.OK
    return dict(name=request.param, w=w, bands=bands, F=F, dt=dt,
                b=O.spmv(bands, w["xstar"]))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("mixed", 1e-5)])
def test_paper_type_apply_parity(paper40, prec, tol):
    c = paper40
    S = P().Solver(G(c["w"]["kappa"]), c["w"]["bc"], prec=prec, schur="newton", smoother="ilu0")
    r = np.random.default_rng(41).uniform(-1, 1, c["w"]["kappa"].shape)
    e_ntd = relmax(C(S.apply_ntd(G(r))), O.apply(c["F"], r))
    e_com = relmax(C(S.apply(G(r))), O.combo_apply(c["bands"], c["F"], c["dt"], r, 2))
    print("%s %s: B apply %.2e, eq. com apply %.2e" % (c["name"], prec, e_ntd, e_com))
    assert e_ntd <= tol and e_com <= tol


@pytest.mark.parametrize("tol", [1e-7, 1e-10])
def test_paper_type_pcg_parity(paper40, tol):
    c = paper40
    S = P().Solver(G(c["w"]["kappa"]), c["w"]["bc"], prec="fp64", schur="newton", smoother="ilu0")
    x, it, rr, st = S.pcg(G(c["b"]), tol=tol, maxit=500)
    xo, ito, rro, sto, _ = O.pcg(c["bands"], c["F"], c["b"], tol, 500, dt=c["dt"])
    print("%s tol %g: GPU %d iterations, oracle %d" % (c["name"], tol, it, ito))
    assert st == P().OK and sto == O.OK and rr <= tol
    assert abs(it - ito) <= 1
    res = c["b"] - O.spmv(c["bands"], C(x))
    assert np.linalg.norm(res) <= 1.01 * tol * np.linalg.norm(c["b"])


@pytest.fixture(scope="module")
def jump128():
    w = W.workload("jump128")
    bands = O.assemble(w["kappa"], w["bc"])
    F = O.setup(bands, mode="newton")
    dt, st = O.ilu0(bands, 2)
    assert st == O.OK
    print("jump128: oracle setup done", flush=True)
    return dict(w=w, bands=bands, F=F, dt=dt)


def test_jump128_mixed_apply_parity(jump128):
    c = jump128
    S = P().Solver(G(c["w"]["kappa"]), c["w"]["bc"], prec="mixed", schur="newton",
                   smoother="ilu0sym")
    r = np.random.default_rng(43).uniform(-1, 1, c["w"]["kappa"].shape)
    want = O.sym_combo_apply(c["bands"], c["F"], c["dt"], r)
    e_sym = relmax(C(S.apply(G(r))), want)
    e_ntd = relmax(C(S.apply_ntd(G(r))), O.apply(c["F"], r))
    print("jump128 MIXED: B apply %.2e, symmetric combination %.2e" % (e_ntd, e_sym))
    assert e_ntd <= 1e-5 and e_sym <= 1e-5


def test_jump128_mixed_vs_fp64_pcg(jump128):
    """The 128^3 configuration: float factors and sweeps with FP64 CG, next to
    all-FP64, both to 1e-8 with the benchmark's preconditioner."""
    c = jump128
    b = c["w"]["b"]
    out = {}
    for prec in ("mixed", "fp64"):
        S = P().Solver(G(c["w"]["kappa"]), c["w"]["bc"], prec=prec, schur="newton",
                       smoother="ilu0sym")
        x, it, rr, st = S.pcg(G(b), tol=1e-8, maxit=2000)
        assert st == P().OK and rr <= 1e-8, (prec, st, rr)
        xs = C(x)
        tr = np.linalg.norm(b - O.spmv(c["bands"], xs)) / np.linalg.norm(b)
        print("jump128 %s: %d iterations, relres %.3e, oracle-recomputed %.3e" % (prec, it, rr, tr))
        assert tr <= 1.01e-8 and abs(tr - rr) <= 1e-3 * rr
        out[prec] = (xs, it)
    assert abs(out["mixed"][1] - out["fp64"][1]) <= out["fp64"][1] // 10 + 2
    d = O.spmv(c["bands"], out["mixed"][0] - out["fp64"][0])
    assert np.linalg.norm(d) <= 2.02e-8 * np.linalg.norm(b)


def test_pcg_breaks_down_on_negative_definite_factors():
    """Pivots -1 and no couplings on one plane make B = -I: r.z = -|r|^2, and
    PCG stops with NTD_EBREAKDOWN before any product with A (x = 0), as the
    oracle does with the same factors."""
    shape = (1, 5, 70)
    kappa = W.kappa_subcubes(70, 5, 1, 3, cubes=2)
    bc = W.BC_ALL_DIRICHLET
    zero, neg = np.zeros(shape), -np.ones(shape)
    b = W.rhs_uniform(70, 5, 1, 44)
    for prec in ("fp64", "mixed"):
        S = P().Solver(G(kappa), bc, prec=prec, schur="newton")
        S.load_factors(G(zero), G(neg), G(zero))
        r = G(b)
        assert relmax(C(S.apply(r)), -b) <= 1e-7
        x, it, rr, st = S.pcg(r, tol=1e-8, maxit=50)
        assert st == P().EBREAKDOWN and it == 0 and float(x.abs().max()) == 0.0
    bands = O.assemble(kappa, bc)
    F = {"e1": zero, "M": neg, "f2": zero, "g3": np.zeros(shape)}
    assert O.pcg(bands, F, b, 1e-8, 50)[3] == O.EBREAKDOWN


def test_spheres96_converges_to_its_attainable_tolerance():
    """The high-contrast inclusion field (200 spheres, kappa = 1e6 inside, b = 1)
    at 96^3: a MIXED solve with the diagonal Schur blocks and the symmetric
    ILU(0) combination reaches 1e-6 (near the attainable accuracy of this
    field in FP64), and the oracle's own SpMV confirms the true residual."""
    n = 96
    w = W.scaled_workload("spheres", n)
    S = P().Solver(G(w["kappa"]), w["bc"], prec="mixed", schur="diag", smoother="ilu0sym")
    x, it, rr, st, hist = S.pcg_history(G(w["b"]), tol=1e-6, maxit=3000)
    bands = O.assemble(w["kappa"], w["bc"])
    tr = np.linalg.norm(w["b"] - O.spmv(bands, C(x))) / np.linalg.norm(w["b"])
    print("spheres96: %d iterations, relres %.3e, oracle-recomputed %.3e" % (it, rr, tr))
    assert st == P().OK and rr <= 1e-6 and len(hist) == it
    assert tr <= 1.01e-6 and abs(tr - rr) <= 1e-3 * rr


def test_pcg_progress_callback_leaves_the_solve_unchanged():
    """ntd_pcg_solve_progress: the callback sees every 7th iteration with the
    recursive residual that the history records, and the solution, the
    iteration count and the residual are bitwise those of ntd_pcg_solve."""
    w = W.workload("poisson32")
    S = P().Solver(G(w["kappa"]), w["bc"], prec="mixed", schur="newton", smoother="ilu0sym")
    b = G(w["b"])
    x0, it0, rr0, st0 = S.pcg(b, tol=1e-10, maxit=500)
    seen = []
    x1, it1, rr1, st1, hist = S.pcg_history(b, tol=1e-10, maxit=500, every=7,
                                            progress=lambda i, r: seen.append((i, r)))
    assert st0 == st1 == P().OK and it0 == it1 and rr0 == rr1
    assert torch.equal(x0, x1)
    assert [i for i, _ in seen] == list(range(7, it1 + 1, 7))
    assert all(r == hist[i - 1] for i, r in seen)
    seen2 = []
    x2, it2, rr2, st2 = S.pcg(b, tol=1e-10, maxit=500, every=5,
                              progress=lambda i, r: seen2.append(i))
    assert torch.equal(x0, x2) and it2 == it0 and seen2 == list(range(5, it0 + 1, 5))
