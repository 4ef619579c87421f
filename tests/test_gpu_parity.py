"""GPU-vs-oracle parity of every step of the hot path, through the C ABI.

Inputs are seeded and synthetic (workloads.py); expected values come from the
FP64 CPU oracle (oracle/) on the same inputs.  Tolerances:
  * assembly: identical operations in the same order -> 1e-15 relative;
  * SpMV: 1e-14 relative to the row magnitude (fused multiply-add on the GPU);
  * dot: |error| <= 1e-14 * sum |x_i y_i|;
  * setup factors (FP64): 1e-9 relative (recurrences amplify FMA differences);
  * apply, element by element against the largest entry of the oracle's
    result (|z - z_o| <= tol * max |z_o|): FP64 with the oracle's factors
    1e-12, with the GPU's own factors 1e-9; MIXED 1e-5;
  * PCG: the same iteration count within +-1, true relative residual <= tol,
    solution difference <= 10 * cond-free bound of the two residuals.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def ntd():
    import paper_1909_09771_amd as P
    return P


def G(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def C(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def case(shape, kind, seed=7):
    nz, ny, nx = shape
    if kind == "poisson":
        return W.kappa_const(nx, ny, nz), W.BC_ALL_DIRICHLET.copy()
    if kind == "jump":
        return W.kappa_subcubes(nx, ny, nz, seed, cubes=4), W.BC_Z0_DIRICHLET.copy()
    if kind == "rand":
        rng = np.random.default_rng(seed)
        bc = np.array([0, 1, 1, 0, 1, 1], dtype=np.int32)
        return 10.0 ** rng.uniform(-2, 2, size=shape), bc
    raise KeyError(kind)


SHAPES = [(32, 32, 32), (7, 11, 37), (5, 1, 64), (1, 9, 65), (3, 4, 1), (1, 1, 1), (2, 1, 1),
          (1, 2, 1), (1, 1, 2), (4, 6, 200), (2, 3, 350)]


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("shape", SHAPES)
def test_assemble_parity(shape):
    kappa, bc = case(shape, "rand")
    S = ntd().Solver(G(kappa), bc, prec="fp64", schur="diag")
    ref = O.assemble(kappa, bc)
    for name, want in zip(("d", "ax", "ay", "az"), ref):
        got = C(S.export(name))
        np.testing.assert_allclose(got, want, rtol=1e-15, atol=0, err_msg=name)


@pytest.mark.parametrize("shape", [(32, 32, 32), (7, 11, 37), (1, 1, 5), (3, 1, 350),
                                   (5, 6, 2), (1, 1, 2), (4, 3, 64)])
def test_spmv_and_dot_parity(shape):
    kappa, bc = case(shape, "rand", seed=3)
    S = ntd().Solver(G(kappa), bc, prec="fp64", schur="diag")
    bands = O.assemble(kappa, bc)
    x = np.random.default_rng(1).standard_normal(shape)
    y = C(S.spmv(G(x)))
    want = O.spmv(bands, x)
    scale = np.abs(bands[0]).max() * np.abs(x).max()
    assert np.abs(y - want).max() <= 1e-14 * scale
    v = np.random.default_rng(2).standard_normal(shape)
    got = S.dot(G(x), G(v))
    assert abs(got - O.dot(x, v)) <= 1e-14 * np.sum(np.abs(x * v))


@pytest.mark.parametrize("shape", [(32, 32, 32), (3, 1, 350), (5, 6, 2), (1, 1, 2), (7, 11, 37)])
def test_spmv_pair_kernel_matches_single_point_kernel_bitwise(shape):
    """Lines of even length with 16-byte aligned vectors take the SpMV over pairs
    of points; an x and y 8 bytes off that alignment take the one-point kernel.
    Both form every point's sum in the same order: y must agree bit for bit (odd
    lines take the one-point kernel both ways)."""
    kappa, bc = case(shape, "rand", seed=5)
    S = ntd().Solver(G(kappa), bc, prec="fp64", schur="diag")
    x = np.random.default_rng(7).standard_normal(shape)
    n = x.size
    y_pair = C(S.spmv(G(x)))
    xb = torch.zeros(n + 1, dtype=torch.float64, device=DEV)
    yb = torch.zeros(n + 1, dtype=torch.float64, device=DEV)
    xb[1:] = G(x).reshape(-1)
    S.spmv(xb[1:].view(shape), out=yb[1:].view(shape))
    assert xb[1:].data_ptr() % 16 == 8
    assert np.array_equal(y_pair, C(yb[1:]).reshape(shape))
    S.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("smoother", ["none", "ilu0", "ilu0sym"])
@pytest.mark.parametrize("shape", [(16, 16, 16), (5, 7, 350), (3, 4, 37)])
def test_pack_pair_kernel_matches_single_point_kernel_bitwise(shape, smoother, prec):
    """The packing of the right-hand side (r, or r - A zi with the smoother)
    takes pairs of points for lines of even length and a 16-byte aligned r, one
    point per thread for an r 8 bytes off that alignment.  The preconditioner's
    output must agree bit for bit (nx = 350 puts the chain split inside a pair;
    nx = 37 takes the one-point kernel both ways)."""
    kappa, bc = case(shape, "rand", seed=9)
    S = ntd().Solver(G(kappa), bc, prec=prec, schur="newton", smoother=smoother)
    r = np.random.default_rng(11).uniform(-1.0, 1.0, shape)
    z_pair = C(S.apply(G(r)))
    n = r.size
    rb = torch.zeros(n + 1, dtype=torch.float64, device=DEV)
    zb = torch.zeros(n + 1, dtype=torch.float64, device=DEV)
    rb[1:] = G(r).reshape(-1)
    assert rb[1:].data_ptr() % 16 == 8
    S.apply(rb[1:].view(shape), out=zb[1:].view(shape))
    assert np.array_equal(z_pair, C(zb[1:]).reshape(shape))
    S.close()


@pytest.mark.parametrize("schur", ["newton", "diag"])
@pytest.mark.parametrize("shape,kind", [((16, 16, 16), "jump"), ((7, 11, 37), "rand"),
                                        ((9, 8, 3), "poisson"), ((1, 9, 65), "rand"),
                                        ((6, 1, 33), "jump")])
def test_setup_parity(shape, kind, schur):
    kappa, bc = case(shape, kind)
    # the diagonal block with a rough random t is not SPD on these problems (the
    # oracle refuses it too, see test_setup_not_spd_status_matches_oracle): use t = 1
    t = W.filter_random(shape[2], shape[1], shape[0], 5) if schur == "newton" else np.ones(shape)
    S = ntd().Solver(G(kappa), bc, t=G(t), prec="fp64", schur=schur)
    F = O.setup(O.assemble(kappa, bc), t, mode=schur)
    for name, want in (("e1", F["e1"]), ("minv", 1.0 / F["M"]), ("f2", F["f2"]), ("dT", F["dT"]),
                       ("dP", F["dP"]), ("xP", F["xP"])):
        got = C(S.export(name))
        err = np.abs(got - want).max()
        assert err <= 1e-9 * max(np.abs(want).max(), 1e-300), (name, err)


@pytest.mark.parametrize("shape,kind", [((32, 32, 32), "poisson"), ((24, 20, 36), "jump"),
                                        ((7, 11, 37), "rand"), ((5, 1, 64), "rand"),
                                        ((1, 9, 65), "jump"), ((1, 1, 1), "poisson"),
                                        ((2, 1, 1), "rand"), ((1, 2, 1), "rand"),
                                        ((4, 6, 200), "jump"), ((2, 3, 350), "rand"),
                                        ((2, 2, 1024), "rand")])
def test_apply_fp64_parity_with_oracle_factors(shape, kind):
    kappa, bc = case(shape, kind)
    F = O.setup(O.assemble(kappa, bc), mode="newton")
    S = ntd().Solver(G(kappa), bc, prec="fp64", schur="newton")
    S.load_factors(G(F["e1"]), G(F["M"]), G(F["f2"]))
    r = np.random.default_rng(11).uniform(-1, 1, shape)
    z = C(S.apply(G(r)))
    assert relmax(z, O.apply(F, r)) <= 1e-12


@pytest.mark.parametrize("schur", ["newton", "diag"])
@pytest.mark.parametrize("shape,kind", [((32, 32, 32), "poisson"), ((24, 20, 36), "jump"),
                                        ((7, 11, 37), "rand")])
def test_apply_fp64_parity_end_to_end(shape, kind, schur):
    kappa, bc = case(shape, kind)
    S = ntd().Solver(G(kappa), bc, prec="fp64", schur=schur)
    F = O.setup(O.assemble(kappa, bc), mode=schur)
    r = np.random.default_rng(12).uniform(-1, 1, shape)
    assert relmax(C(S.apply(G(r))), O.apply(F, r)) <= 1e-9


@pytest.mark.parametrize("schur", ["newton", "diag"])
@pytest.mark.parametrize("shape,kind", [((32, 32, 32), "poisson"), ((24, 20, 36), "jump"),
                                        ((7, 11, 37), "rand"), ((2, 3, 350), "rand")])
def test_apply_mixed_within_1e5(shape, kind, schur):
    kappa, bc = case(shape, kind)
    S = ntd().Solver(G(kappa), bc, prec="mixed", schur=schur)
    F = O.setup(O.assemble(kappa, bc), mode=schur)
    r = np.random.default_rng(13).uniform(-1, 1, shape)
    z = C(S.apply(G(r)))
    want = O.apply(F, r)
    assert relmax(z, want) <= 1e-5


# one shape per supported elements-per-lane count (line length nx -> EPL):
# 32 -> 1, 65 -> 2, 150 -> 3, 256 -> 4, 300 -> 5, 350 -> 6, 420 -> 7, 512 -> 8,
# 600 -> 10, 700 -> 12, 900 -> 14, 1024 -> 16
EPL_SHAPES = [(3, 5, 32), (3, 4, 65), (2, 5, 150), (3, 4, 256), (2, 3, 300), (2, 3, 350),
              (2, 3, 420), (2, 2, 512), (2, 2, 600), (2, 2, 700), (2, 2, 900), (2, 2, 1024)]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
@pytest.mark.parametrize("shape", EPL_SHAPES)
def test_apply_every_lane_width(shape, prec, tol):
    kappa, bc = case(shape, "rand", seed=17)
    F = O.setup(O.assemble(kappa, bc), mode="diag")
    S = ntd().Solver(G(kappa), bc, prec=prec, schur="diag")
    S.load_factors(G(F["e1"]), G(F["M"]), G(F["f2"]))
    r = np.random.default_rng(19).uniform(-1, 1, shape)
    z = C(S.apply(G(r)))
    want = O.apply(F, r)
    assert relmax(z, want) <= tol


@pytest.mark.parametrize("schur", ["newton", "diag"])
def test_filter_property_on_gpu(schur):
    shape = (40, 36, 48)
    kappa, bc = case(shape, "jump")
    t = W.filter_random(shape[2], shape[1], shape[0], 6) if schur == "newton" else np.ones(shape)
    S = ntd().Solver(G(kappa), bc, t=G(t), prec="fp64", schur=schur)
    tg = G(t)
    z = C(S.apply(S.spmv(tg)))
    assert relmax(z, t) <= 1e-10


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_pcg_parity_poisson32(prec):
    w = W.workload("poisson32")
    kappa, bc, b = w["kappa"], w["bc"], w["b"]
    S = ntd().Solver(G(kappa), bc, prec=prec, schur="diag")
    x, it, rr, st = S.pcg(G(b), tol=1e-8, maxit=200)
    bands = O.assemble(kappa, bc)
    xo, ito, rro, sto = O.pcg(bands, O.setup(bands, mode="diag"), b, 1e-8, 200)[:4]
    assert st == 0 and sto == 0
    assert rr <= 1e-8
    assert abs(it - ito) <= (1 if prec == "fp64" else 3)
    xg = C(x)
    # both solutions have true residual <= 1e-8; compare through A: ||A(xg - xo)|| <= 2e-8 ||b||
    d = O.spmv(bands, xg - xo)
    assert np.linalg.norm(d) <= 2.01e-8 * np.linalg.norm(b)


def test_pcg_jump_mixed_vs_fp64_oracle():
    shape = (24, 20, 36)
    kappa, bc = case(shape, "jump")
    b = W.rhs_uniform(shape[2], shape[1], shape[0], 9)
    S = ntd().Solver(G(kappa), bc, prec="mixed", schur="diag")
    x, it, rr, st = S.pcg(G(b), tol=1e-8, maxit=500)
    bands = O.assemble(kappa, bc)
    xo, ito, rro, sto = O.pcg(bands, O.setup(bands, mode="diag"), b, 1e-8, 500)[:4]
    assert st == 0 and rr <= 1e-8 and sto == 0
    # float factors cost some iterations on jump problems; the accuracy is unchanged
    print("mixed iterations %d, FP64 oracle iterations %d" % (it, ito))
    assert it <= ito + ito // 2 + 3


def test_pcg_filter_rhs_one_iteration():
    shape = (16, 12, 20)
    kappa, bc = case(shape, "jump")
    t = np.ones(shape)
    S = ntd().Solver(G(kappa), bc, prec="fp64", schur="newton")
    b = S.spmv(G(t))
    x, it, rr, st = S.pcg(b, tol=1e-10, maxit=20)
    assert st == 0 and it == 1
    assert relmax(C(x), t) <= 1e-10


def test_pcg_status_codes():
    shape = (8, 8, 8)
    kappa, bc = case(shape, "jump")
    S = ntd().Solver(G(kappa), bc, prec="fp64", schur="diag")
    b = G(W.rhs_uniform(8, 8, 8, 4))
    x, it, rr, st = S.pcg(b, tol=1e-14, maxit=1)
    assert st == ntd().ENOCONV and it == 1
    x, it, rr, st = S.pcg(torch.zeros_like(b), tol=1e-8, maxit=5)
    assert st == 0 and it == 0 and float(x.abs().max()) == 0.0


def test_setup_not_spd_status_matches_oracle():
    """A rough random filter with the diagonal Schur block makes a pivot
    non-positive; the GPU setup must report it exactly when the oracle does."""
    P = ntd()
    for shape, seed in (((16, 16, 16), 5), ((7, 11, 37), 5), ((6, 6, 6), 1)):
        kappa, bc = case(shape, "jump")
        t = W.filter_random(shape[2], shape[1], shape[0], seed)
        st_o = O.setup(O.assemble(kappa, bc), t, mode="diag", raise_on_error=False)["status"]
        try:
            P.Solver(G(kappa), bc, t=G(t), prec="fp64", schur="diag")
            st_g = P.OK
        except P.NTDError as e:
            st_g = e.status
        assert st_g == st_o, (shape, st_g, st_o)


def test_setup_rejects_bad_kappa_and_t():
    P = ntd()
    kappa, bc = case((4, 4, 4), "poisson")
    bad = kappa.copy()
    bad[1, 2, 3] = 0.0
    with pytest.raises(P.NTDError) as ei:
        P.Solver(G(bad), bc, prec="fp64")
    assert ei.value.status == P.EINVAL
    t = np.ones((4, 4, 4))
    t[0, 0, 0] = np.nan
    with pytest.raises(P.NTDError):
        P.Solver(G(kappa), bc, t=G(t), prec="fp64")


def test_deterministic_repeat():
    shape = (24, 20, 36)
    kappa, bc = case(shape, "jump")
    for prec in ("fp64", "mixed"):
        S = ntd().Solver(G(kappa), bc, prec=prec, schur="diag")
        r = G(np.random.default_rng(3).uniform(-1, 1, shape))
        a, b = C(S.apply(r)), C(S.apply(r))
        assert np.array_equal(a, b)
        d1 = S.dot(r, S.spmv(r))
        d2 = S.dot(r, S.spmv(r))
        assert d1 == d2


# ---------------------------------------------------------------------------
# ILU(0) smoother and the combination preconditioner (Sec. 3, eq. com)
# ---------------------------------------------------------------------------

ILU_SHAPES = [((16, 12, 20), "jump"), ((7, 11, 37), "rand"), ((5, 4, 3), "rand"), ((1, 6, 9), "jump"),
              ((9, 1, 1), "rand"), ((2, 2, 2), "poisson"), ((41, 35, 24), "jump")]
# lines longer than 256: 6 values per lane with whole-chunk loads (nx = 300) and
# element loads (350), 8 per lane (500: the block split falls inside a line;
# 512: whole chunks) and 16 per lane (600)
ILU_WIDE_SHAPES = [((3, 4, 300), "rand"), ((2, 5, 350), "jump"), ((3, 3, 500), "rand"),
                   ((2, 3, 512), "jump"), ((2, 2, 600), "rand")]
# the same line lengths with ny, nz above the 8 x 8 line tile, so that every
# values-per-lane variant hands neighbour lines across tiles in both sweeps and
# meets the block split between tiles
ILU_TILED_WIDE_SHAPES = [((19, 17, 350), "rand"), ((18, 11, 500), "jump"), ((17, 9, 512), "rand"),
                         ((12, 10, 600), "jump"), ((10, 9, 300), "rand")]


@pytest.mark.parametrize("shape,kind", ILU_SHAPES + ILU_WIDE_SHAPES + ILU_TILED_WIDE_SHAPES)
def test_ilu0_factor_and_apply_parity(shape, kind):
    kappa, bc = case(shape, kind)
    S = ntd().Solver(G(kappa), bc, prec="fp64", schur="newton", smoother="ilu0")
    bands = O.assemble(kappa, bc)
    dt, st = O.ilu0(bands, 2)
    assert st == 0
    np.testing.assert_allclose(C(S.export("dt")), dt, rtol=1e-13)
    r = np.random.default_rng(23).uniform(-1, 1, shape)
    z = C(S.apply_ilu0(G(r)))
    assert relmax(z, O.ilu0_apply(bands, dt, r, 2)) <= 1e-12


@pytest.mark.parametrize("shape,kind", ILU_SHAPES + ILU_WIDE_SHAPES + ILU_TILED_WIDE_SHAPES)
def test_ilu0_apply_parity_mixed(shape, kind):
    """MIXED reads the ILU(0) sweeps' coefficients (the couplings and 1/dt) in
    FP32, with FP64 arithmetic: every values-per-lane variant, with and without
    vector loads, within 1e-5 of the oracle element by element."""
    kappa, bc = case(shape, kind)
    S = ntd().Solver(G(kappa), bc, prec="mixed", schur="newton", smoother="ilu0")
    bands = O.assemble(kappa, bc)
    dt, st = O.ilu0(bands, 2)
    assert st == 0
    np.testing.assert_allclose(C(S.export("dt")), dt, rtol=1e-13)
    r = np.random.default_rng(24).uniform(-1, 1, shape)
    assert relmax(C(S.apply_ilu0(G(r))), O.ilu0_apply(bands, dt, r, 2)) <= 1e-5


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("mixed", 1e-5)])
@pytest.mark.parametrize("shape,kind", ILU_SHAPES[:4])
def test_combination_apply_parity(shape, kind, prec, tol):
    kappa, bc = case(shape, kind)
    S = ntd().Solver(G(kappa), bc, prec=prec, schur="newton", smoother="ilu0")
    bands = O.assemble(kappa, bc)
    F = O.setup(bands, mode="newton")
    dt, _ = O.ilu0(bands, 2)
    r = np.random.default_rng(29).uniform(-1, 1, shape)
    want = O.combo_apply(bands, F, dt, r, 2)
    z = C(S.apply(G(r)))
    assert relmax(z, want) <= tol
    zn = C(S.apply_ntd(G(r)))
    assert relmax(zn, O.apply(F, r)) <= tol


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_pcg_combination_parity(prec):
    shape = (24, 20, 36)
    kappa, bc = case(shape, "jump")
    b = W.rhs_uniform(shape[2], shape[1], shape[0], 31)
    S = ntd().Solver(G(kappa), bc, prec=prec, schur="newton", smoother="ilu0")
    x, it, rr, st = S.pcg(G(b), tol=1e-8, maxit=500)
    bands = O.assemble(kappa, bc)
    dt, _ = O.ilu0(bands, 2)
    xo, ito, rro, sto = O.pcg(bands, O.setup(bands, mode="newton"), b, 1e-8, 500, dt=dt)[:4]
    print("combination PCG: %s iterations %d, FP64 oracle %d" % (prec, it, ito))
    assert st == 0 and sto == 0 and rr <= 1e-8
    assert abs(it - ito) <= (1 if prec == "fp64" else ito // 4 + 3)
    d = O.spmv(bands, C(x) - xo)
    assert np.linalg.norm(d) <= 2.01e-8 * np.linalg.norm(b)


@pytest.mark.parametrize("smoother", ["none", "ilu0"])
def test_apply_profile_matches_apply(smoother):
    """The timed preconditioner (as PCG launches it) gives the same output as
    the plain entry point and reports non-negative launch durations."""
    shape = (12, 10, 40)
    kappa, bc = case(shape, "jump")
    S = ntd().Solver(G(kappa), bc, prec="mixed", schur="newton", smoother=smoother)
    r = G(np.random.default_rng(37).uniform(-1, 1, shape))
    z = torch.empty_like(r)
    ms = S.apply_profile(r, z)
    assert len(ms) == 4 and min(ms) >= 0.0
    if smoother == "ilu0":
        assert ms[3] > 0.0
    np.testing.assert_array_equal(C(z), C(S.apply(r)))
