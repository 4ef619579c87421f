"""Parity of the batched solve (many systems, several right-hand sides each)
with the FP64 oracle, entry by entry, through the C ABI.

The batch packs every system with the elements per lane of its longest line,
so the shorter systems below run with pass-through slots; their results are
held to the same bars as the single-system path: apply 1e-9 (FP64, the GPU's
own factors) and 1e-5 (MIXED) element by element relative to the largest
entry of the oracle's result; PCG iterations within +-1 of the oracle
in FP64, true relative residual <= tol.  Graph replay and eager launches must
give bitwise identical results.
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


def relelem(a, b):
    """Largest element-wise error relative to the largest entry of b."""
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# (nz, ny, nx), kind; nx 33 needs 1 element per lane, 70 needs 2: the first
# and third systems run padded to 2
SYSTEMS = [((12, 10, 33), "layers", 1), ((9, 7, 70), "rand", 2), ((5, 16, 20), "layers", 3)]


def build(kind, shape, seed):
    nz, ny, nx = shape
    if kind == "layers":
        return W.kappa_layers(nx, ny, nz, 4100 + seed), W.BC_ALL_DIRICHLET.copy()
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(-2, 2, size=shape), np.array([0, 1, 1, 0, 1, 1], dtype=np.int32)


@pytest.fixture(scope="module")
def systems():
    out = []
    for shape, kind, seed in SYSTEMS:
        kappa, bc = build(kind, shape, seed)
        out.append(dict(shape=shape, kappa=kappa, bc=bc, bands=O.assemble(kappa, bc)))
    return out


def make_batch(systems, nrhs, prec, schur):
    import paper_1909_09771_amd as P
    return P.Batch([G(s["kappa"]) for s in systems], [s["bc"] for s in systems], nrhs=nrhs,
                   prec=prec, schur=schur)


def rhs_list(systems, nrhs, seed):
    rng = np.random.default_rng(seed)
    return [rng.uniform(-1.0, 1.0, s["shape"]) for s in systems for _ in range(nrhs)]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("mixed", 1e-5)])
@pytest.mark.parametrize("schur", ["diag", "newton"])
def test_batch_apply_parity(systems, prec, tol, schur):
    nrhs = 3
    B = make_batch(systems, nrhs, prec, schur)
    rs = rhs_list(systems, nrhs, 41)
    zs = [C(z) for z in B.apply([G(r) for r in rs])]
    for e, (r, z) in enumerate(zip(rs, zs)):
        s = systems[e // nrhs]
        want = O.apply(O.setup(s["bands"], mode=schur), r)
        assert relelem(z, want) <= tol, "entry %d" % e
    B.close()


def test_batch_apply_matches_single_system_bitwise(systems):
    """The unpadded system (its own elements per lane equal the batch's) gives
    the single-system apply's output bit for bit."""
    import paper_1909_09771_amd as P
    nrhs = 2
    B = make_batch(systems, nrhs, "mixed", "diag")
    rs = rhs_list(systems, nrhs, 43)
    zs = B.apply([G(r) for r in rs])
    s = systems[1]
    S = P.Solver(G(s["kappa"]), s["bc"], prec="mixed", schur="diag")
    for q in range(nrhs):
        e = 1 * nrhs + q
        assert np.array_equal(C(zs[e]), C(S.apply(G(rs[e]))))
    B.close()
    S.close()


def test_batch_apply_profile_matches_apply(systems):
    B = make_batch(systems, 2, "mixed", "diag")
    rs = [G(r) for r in rhs_list(systems, 2, 47)]
    z1 = [C(z) for z in B.apply(rs)]
    zs = B.empty_like_entries()
    ms = B.apply_profile(rs, zs)
    assert len(ms) == 4 and min(ms) >= 0.0 and ms[0] > 0.0
    for a, b in zip(z1, zs):
        assert np.array_equal(a, C(b))
    B.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_pcg_parity(systems, prec):
    nrhs = 2
    tol = 1e-8
    B = make_batch(systems, nrhs, prec, "diag")
    bs = rhs_list(systems, nrhs, 53)
    xs, its, rrs, sts = B.pcg([G(b) for b in bs], tol=tol, maxit=500)
    for e, b in enumerate(bs):
        s = systems[e // nrhs]
        xo, ito, rro, sto = O.pcg(s["bands"], O.setup(s["bands"], mode="diag"), b, tol, 500)[:4]
        print("batch PCG %s entry %d: %d iterations, oracle %d" % (prec, e, its[e], ito))
        assert sts[e] == 0 and sto == 0 and rrs[e] <= tol
        assert abs(its[e] - ito) <= (1 if prec == "fp64" else ito // 4 + 3)
        res = b - O.spmv(s["bands"], C(xs[e]))
        assert np.linalg.norm(res) <= 1.01 * tol * np.linalg.norm(b)
    B.close()


def test_batch_pcg_graph_equals_eager(systems):
    """Replays of the captured chunk of iterations (with host checks and eager
    true-residual launches between them) reproduce the eager launches bit for
    bit, on a first and a repeated call."""
    nrhs = 2
    B = make_batch(systems, nrhs, "mixed", "newton")
    bs = [G(b) for b in rhs_list(systems, nrhs, 59)]
    xe, ie, re, se = B.pcg(bs, tol=1e-9, maxit=400, graph=False)
    xe = [C(x) for x in xe]
    for _ in range(2):
        xg, ig, rg, sg = B.pcg(bs, tol=1e-9, maxit=400, graph=True)
        assert ig == ie and se == sg and rg == re
        for a, b in zip(xe, xg):
            assert np.array_equal(a, C(b))
    B.close()


def test_batch_pcg_edge_cases(systems):
    """A zero right-hand side stops at once with x = 0; an entry out of
    iterations reports NTD_ENOCONV with iters = maxit, without holding back
    the others."""
    nrhs = 2
    B = make_batch(systems, nrhs, "fp64", "diag")
    bs = rhs_list(systems, nrhs, 61)
    bs[0] = np.zeros_like(bs[0])
    xs, its, rrs, sts = B.pcg([G(b) for b in bs], tol=1e-8, maxit=500)
    assert its[0] == 0 and sts[0] == 0 and rrs[0] == 0.0
    assert not np.any(C(xs[0]))
    assert all(st == 0 for st in sts)
    xs2, its2, rrs2, sts2 = B.pcg([G(b) for b in bs], tol=1e-14, maxit=3)
    for e in range(1, len(bs)):
        assert sts2[e] == 5 and its2[e] == 3  # NTD_ENOCONV
    B.close()


def test_batch_rejects_bad_kappa(systems):
    """One system with a non-positive kappa fails the whole batch setup with
    NTD_EINVAL (the input check runs over every system before any factorization)."""
    import paper_1909_09771_amd as P
    kappas = [G(s["kappa"]) for s in systems]
    bad = systems[1]["kappa"].copy()
    bad[0, 0, 0] = -1.0
    kappas[1] = G(bad)
    with pytest.raises(P.NTDError) as ei:
        P.Batch(kappas, [s["bc"] for s in systems], nrhs=2, prec="mixed", schur="diag")
    assert ei.value.status == P.EINVAL


@pytest.mark.parametrize("tol", [1e-12, 1e-13, 1e-14])
def test_batch_pcg_follows_the_single_solve_near_the_rounding_floor(systems, tol):
    """Near the attainable accuracy the recursive residual can pass the
    tolerance while the true one does not; the entry then continues its CG
    iteration exactly as the single-system solve does (same iterations, same
    status), instead of repeating its last step."""
    import paper_1909_09771_amd as P
    nrhs = 1
    B = make_batch(systems, nrhs, "fp64", "diag")
    bs = rhs_list(systems, nrhs, 67)
    xs, its, rrs, sts = B.pcg([G(b) for b in bs], tol=tol, maxit=300)
    for e, b in enumerate(bs):
        s = systems[e]
        S = P.Solver(G(s["kappa"]), s["bc"], prec="fp64", schur="diag")
        x1, it1, rr1, st1 = S.pcg(G(b), tol=tol, maxit=300)
        print("tol %.0e entry %d: batch %d its (status %d, relres %.2e), single %d (status %d, "
              "relres %.2e)" % (tol, e, its[e], sts[e], rrs[e], it1, st1, rr1))
        assert sts[e] == st1 and abs(its[e] - it1) <= 1
        S.close()
    B.close()


def test_batch_tune_keeps_parity(systems):
    """The autotuned launch shape is one of the candidates (the sized maximum
    and its halvings), and the batch still solves to the oracle's bar, with
    graph replay equal to eager launches."""
    nrhs = 2
    B = make_batch(systems, nrhs, "mixed", "diag")
    bs = rhs_list(systems, nrhs, 71)
    B.pcg([G(b) for b in bs], tol=1e-8, maxit=500)     # captures a graph first
    gmax = max((s["shape"][0] * s["shape"][1] * s["shape"][2] + 1023) // 1024 for s in systems)
    g = B.tune()
    assert g in {(gmax + (1 << k) - 1) >> k for k in range(4)}
    assert B.tune() in {(gmax + (1 << k) - 1) >> k for k in range(4)}
    xg, ig, rg, sg = B.pcg([G(b) for b in bs], tol=1e-8, maxit=500, graph=True)
    xe, ie, re, se = B.pcg([G(b) for b in bs], tol=1e-8, maxit=500, graph=False)
    assert ig == ie and sg == se
    for a, b in zip(xg, xe):
        assert np.array_equal(C(a), C(b))
    for e, b in enumerate(bs):
        s = systems[e // nrhs]
        ito = O.pcg(s["bands"], O.setup(s["bands"], mode="diag"), b, 1e-8, 500)[1]
        assert sg[e] == 0 and rg[e] <= 1e-8 and abs(ig[e] - ito) <= ito // 4 + 3
    B.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("nr", [2, 4])
def test_batch_sweeps_with_several_rhs_per_wavefront(systems, prec, nr):
    """Sweeping nr right-hand sides of a system per wavefront pair (one record
    load for all of them) gives the one-per-pair results bitwise, and the
    oracle's to the apply bars; PCG through the graph takes the same
    iterations and gives the same solutions."""
    import paper_1909_09771_amd as P
    nrhs = 4
    B = make_batch(systems, nrhs, prec, "newton")
    rs = rhs_list(systems, nrhs, 43)
    base = [C(z) for z in B.apply([G(r) for r in rs])]
    try:
        B.set_sweep_group(nr)
    except P.NTDError as e:   # FP64 lines of 70 points take 2 values per lane: nr 4 is not built
        assert prec == "fp64" and nr == 4 and e.status == P.EINVAL
        B.close()
        return
    multi = [C(z) for z in B.apply([G(r) for r in rs])]
    tol = 1e-9 if prec == "fp64" else 1e-5
    for e, (r, z0, z1) in enumerate(zip(rs, base, multi)):
        assert np.array_equal(z0, z1), "entry %d" % e
        s = systems[e // nrhs]
        want = O.apply(O.setup(s["bands"], mode="newton"), r)
        assert relelem(z1, want) <= tol, "entry %d" % e
    bs = rhs_list(systems, nrhs, 44)
    B.set_sweep_group(1)
    x1, i1, r1, s1 = B.pcg([G(b) for b in bs], tol=1e-8, maxit=500)
    B.set_sweep_group(nr)
    x2, i2, r2, s2 = B.pcg([G(b) for b in bs], tol=1e-8, maxit=500)
    assert i1 == i2 and s1 == s2
    for a, b in zip(x1, x2):
        assert np.array_equal(C(a), C(b))
    B.close()


def test_batch_tune_sweeps_picks_a_supported_group(systems):
    import paper_1909_09771_amd as P
    nrhs = 4
    B = make_batch(systems, nrhs, "mixed", "diag")
    nr = B.tune_sweeps()
    assert nr in (1, 2, 4)
    bs = rhs_list(systems, nrhs, 45)
    xs, its, rrs, sts = B.pcg([G(b) for b in bs], tol=1e-8, maxit=500)
    for e, b in enumerate(bs):
        assert sts[e] == P.OK and rrs[e] <= 1e-8
    B.close()
    with pytest.raises(P.NTDError):
        B2 = make_batch(systems, 3, "mixed", "diag")
        try:
            B2.set_sweep_group(2)      # 2 does not divide 3 right-hand sides
        finally:
            B2.close()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_batch_plane_lds_matches_memory_bitwise(systems, prec):
    """The line sweeps keeping each plane in LDS (the default where every
    workgroup fits at once, as these small systems do) give the results of the
    sweeps through memory bit for bit: apply, and PCG through the graph; also
    with 2 and 4 right-hand sides per wavefront pair."""
    nrhs = 4
    B = make_batch(systems, nrhs, prec, "newton")
    assert B.set_plane_lds(True)
    rs = [G(r) for r in rhs_list(systems, nrhs, 51)]
    z_lds = [C(z) for z in B.apply(rs)]
    assert not B.set_plane_lds(False)
    z_mem = [C(z) for z in B.apply(rs)]
    for e, (a, b) in enumerate(zip(z_lds, z_mem)):
        assert np.array_equal(a, b), "entry %d" % e
    bs = [G(b) for b in rhs_list(systems, nrhs, 52)]
    x0, i0, r0, s0 = B.pcg(bs, tol=1e-8, maxit=500, graph=True)
    assert B.set_plane_lds(True)
    x1, i1, r1, s1 = B.pcg(bs, tol=1e-8, maxit=500, graph=True)
    assert i0 == i1 and s0 == s1
    for e, (a, b) in enumerate(zip(x0, x1)):
        assert np.array_equal(C(a), C(b)), "entry %d" % e
    # several right-hand sides per wavefront pair: one plane buffer each
    import paper_1909_09771_amd as P
    for nr in (2, 4):
        if nr > nrhs:
            continue
        try:
            B.set_sweep_group(nr)
        except P.NTDError as e:   # not built for this precision and line length
            assert e.status == P.EINVAL
            continue
        assert B.set_plane_lds(True)
        z_lds = [C(z) for z in B.apply(rs)]
        B.set_plane_lds(False)
        z_mem2 = [C(z) for z in B.apply(rs)]
        for e, (a, b, c) in enumerate(zip(z_lds, z_mem2, z_mem)):
            assert np.array_equal(a, b) and np.array_equal(a, c), "nr %d entry %d" % (nr, e)
    B.close()


# degenerate level-3 and level-2 chains: one plane, two planes (no interior
# plane on either side of the twist), one line per plane, and four planes
EDGE_SYSTEMS = [((1, 6, 9), "rand", 11), ((2, 5, 17), "rand", 12), ((6, 1, 30), "layers", 13),
                ((4, 3, 64), "rand", 14)]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("mixed", 1e-5)])
def test_batch_plane_lds_edge_shapes(prec, tol):
    """Degenerate shapes through the LDS-plane sweeps: oracle parity element by
    element, and bitwise the sweeps through memory."""
    syst = []
    for shape, kind, seed in EDGE_SYSTEMS:
        kappa, bc = build(kind, shape, seed)
        syst.append(dict(shape=shape, kappa=kappa, bc=bc, bands=O.assemble(kappa, bc)))
    nrhs = 2
    B = make_batch(syst, nrhs, prec, "newton")
    assert B.set_plane_lds(True)
    rs = rhs_list(syst, nrhs, 53)
    z_lds = [C(z) for z in B.apply([G(r) for r in rs])]
    B.set_plane_lds(False)
    z_mem = [C(z) for z in B.apply([G(r) for r in rs])]
    for e, (r, a, b) in enumerate(zip(rs, z_lds, z_mem)):
        s = syst[e // nrhs]
        assert np.array_equal(a, b), "entry %d" % e
        want = O.apply(O.setup(s["bands"], mode="newton"), r)
        assert relelem(a, want) <= tol, "entry %d" % e
    B.close()


def test_batch_plane_lds_at_the_benchmark_plane_size():
    """The LDS-plane sweeps at the batch benchmark's plane size (128^2 lines,
    two values per lane, 65 KB of LDS per workgroup, two workgroups per CU):
    eight 128^3 systems of the batch workload with two right-hand sides each,
    bitwise equal to the sweeps through memory, and two entries against the
    oracle element by element (MIXED bar)."""
    syst = W.batch_systems(count=8, nrhs=2, n_fixed=128)
    nrhs = 2
    import paper_1909_09771_amd as P
    B = P.Batch([G(s["kappa"]) for s in syst], [s["bc"] for s in syst], nrhs=nrhs,
                prec="mixed", schur="diag")
    assert B.set_plane_lds(True)
    rs = [G(b) for s in syst for b in s["bs"]]
    z_lds = [C(z) for z in B.apply(rs)]
    assert not B.set_plane_lds(False)
    z_mem = [C(z) for z in B.apply(rs)]
    for e, (a, b) in enumerate(zip(z_lds, z_mem)):
        assert np.array_equal(a, b), "entry %d" % e
    B.close()
    for e in (0, 13):
        s = syst[e // nrhs]
        want = O.apply(O.setup(O.assemble(s["kappa"], s["bc"]), mode="diag"), s["bs"][e % nrhs])
        assert relelem(z_lds[e], want) <= 1e-5, "entry %d" % e


def test_batch_plane_lds_survives_a_later_smaller_batch():
    """The dynamic-LDS limit of the LDS-plane kernels is shared by every batch:
    a batch with small planes set up after one with 128-line planes must not
    lower it below what the first one launches with."""
    import paper_1909_09771_amd as P
    big = [((8, 128, 128), "layers", 21), ((6, 128, 128), "rand", 22)]
    small = [((5, 10, 33), "layers", 23)]
    def mk(spec):
        out = []
        for shape, kind, seed in spec:
            kappa, bc = build(kind, shape, seed)
            out.append(dict(shape=shape, kappa=kappa, bc=bc))
        return out
    sb, ss = mk(big), mk(small)
    A = P.Batch([G(s["kappa"]) for s in sb], [s["bc"] for s in sb], nrhs=1, prec="mixed",
                schur="diag")
    assert A.set_plane_lds(True)
    rs = [G(r) for r in rhs_list(sb, 1, 71)]
    z1 = [C(z) for z in A.apply(rs)]
    Bs = P.Batch([G(s["kappa"]) for s in ss], [s["bc"] for s in ss], nrhs=1, prec="mixed",
                 schur="diag")
    assert Bs.set_plane_lds(True)
    Bs.apply([G(r) for r in rhs_list(ss, 1, 72)])
    z2 = [C(z) for z in A.apply(rs)]
    for e, (a, b) in enumerate(zip(z1, z2)):
        assert np.array_equal(a, b), "entry %d" % e
    Bs.close()
    A.close()
