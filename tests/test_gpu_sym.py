"""Parity of the symmetric combination (NTD_SMOOTHER_ILU0_SYM: z1 = B_ILU^{-1} r,
z2 = z1 + B^{-1}(r - A z1), z = z2 + B_ILU^{-1}(r - A z2)) with the oracle, through
the C ABI.  Bars as for the combination of eq. com: apply 1e-9 (FP64) and 1e-5
(MIXED) element by element relative to the largest entry of the oracle's
result; PCG iterations within +-1 of the oracle in FP64."""
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


def relelem(a, b):
    """Largest element-wise error relative to the largest entry of b."""
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


FIELDS = {
    "spheres": lambda: W.kappa_spheres(21, 7, 9, 301, count=12, r_lo=0.1, r_hi=0.25),
    "subcubes": lambda: W.kappa_subcubes(33, 10, 12, 78, cubes=3),
}


@pytest.fixture(scope="module", params=sorted(FIELDS))
def field(request):
    kappa = FIELDS[request.param]()
    bc = W.BC_ALL_DIRICHLET.copy()
    bands = O.assemble(kappa, bc)
    dt, st = O.ilu0(bands)
    assert st == 0
    return dict(name=request.param, kappa=kappa, bc=bc, bands=bands, dt=dt)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("mixed", 1e-5)])
@pytest.mark.parametrize("schur", ["newton", "diag"])
def test_sym_apply_parity(field, prec, tol, schur):
    import paper_1909_09771_amd as P
    F = O.setup(field["bands"], mode=schur)
    r = np.random.default_rng(5).uniform(-1, 1, field["kappa"].shape)
    S = P.Solver(G(field["kappa"]), field["bc"], prec=prec, schur=schur, smoother="ilu0sym")
    z = C(S.apply(G(r)))
    want = O.sym_combo_apply(field["bands"], F, field["dt"], r)
    err = relelem(z, want)
    print("%s %s %s: rel err %.2e" % (field["name"], prec, schur, err))
    assert err <= tol
    # the timed application is the same launches
    z2 = torch.empty_like(G(r))
    ms = S.apply_profile(G(r), z2)
    assert np.array_equal(C(z2), z) and min(ms) >= 0.0
    S.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_sym_pcg_parity(field, prec):
    import paper_1909_09771_amd as P
    F = O.setup(field["bands"], mode="diag")
    b = np.random.default_rng(6).uniform(-1, 1, field["kappa"].shape)
    xo, ito, rro, sto = O.pcg_with(field["bands"],
                                   lambda r: O.sym_combo_apply(field["bands"], F, field["dt"], r),
                                   b, 1e-8, 1000)
    S = P.Solver(G(field["kappa"]), field["bc"], prec=prec, schur="diag", smoother="ilu0sym")
    x, it, rr, st = S.pcg(G(b), tol=1e-8, maxit=1000)
    print("%s %s: %d iterations, oracle %d" % (field["name"], prec, it, ito))
    assert st == P.OK and sto == O.OK and rr <= 1e-8
    assert abs(it - ito) <= (1 if prec == "fp64" else ito // 4 + 3)
    res = b - O.spmv(field["bands"], C(x))
    assert np.linalg.norm(res) <= 1.01e-8 * np.linalg.norm(b)
    S.close()


def test_apply_ilu0_needs_a_smoother_and_accepts_the_symmetric_one(field):
    import paper_1909_09771_amd as P
    r = G(np.random.default_rng(7).uniform(-1, 1, field["kappa"].shape))
    S = P.Solver(G(field["kappa"]), field["bc"], prec="fp64", schur="diag", smoother="ilu0sym")
    want = O.ilu0_apply(field["bands"], field["dt"], C(r))
    assert relelem(C(S.apply_ilu0(r)), want) <= 1e-12
    S.close()
