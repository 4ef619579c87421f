"""Seeded synthetic inputs for the diffusion problem -div(kappa grad u) = f.

This module only *draws inputs*: coefficient fields kappa, boundary-type sets,
right-hand sides and filter vectors.  It holds none of the preconditioner's
arithmetic, so both the FP64 CPU oracle (test side) and the GPU library's
callers (tests, smoke check, benchmark) can use it without sharing method code.

Conventions (Sec. 2 of arXiv:1909.09771): nx points per line (x, fastest),
ny lines per plane, nz planes; arrays are C-contiguous numpy arrays of shape
(nz, ny, nx), so unknown p = i + nx*(j + ny*k).  Node (i, j, k) sits at
((i+1)/(nx+1), (j+1)/(ny+1), (k+1)/(nz+1)) in the unit cube (vertex-centred
interior grid; boundary points carry no unknown).

Boundary types: a length-6 int array for the faces x-, x+, y-, y+, z-, z+;
0 = Dirichlet (u = 0), 1 = homogeneous Neumann (Sec. 1, eq. diffeqn).
"""
from __future__ import annotations

import numpy as np

DIRICHLET = 0
NEUMANN = 1

BC_ALL_DIRICHLET = np.zeros(6, dtype=np.int32)
# Dirichlet on the z = 0 face only, Neumann on the other five faces.
BC_Z0_DIRICHLET = np.array([NEUMANN, NEUMANN, NEUMANN, NEUMANN, DIRICHLET, NEUMANN],
                           dtype=np.int32)


def node_coords(nx: int, ny: int, nz: int):
    """Broadcastable node coordinates (x, y, z) of the interior grid."""
    x = (np.arange(nx, dtype=np.float64) + 1.0) / (nx + 1)
    y = (np.arange(ny, dtype=np.float64) + 1.0) / (ny + 1)
    z = (np.arange(nz, dtype=np.float64) + 1.0) / (nz + 1)
    return x[None, None, :], y[None, :, None], z[:, None, None]


def kappa_const(nx: int, ny: int, nz: int, value: float = 1.0) -> np.ndarray:
    return np.full((nz, ny, nx), float(value), dtype=np.float64)


def kappa_subcubes(nx: int, ny: int, nz: int, seed: int, cubes: int = 8,
                   log10_lo: float = -3.0, log10_hi: float = 3.0) -> np.ndarray:
    """Piecewise-constant kappa on cubes^3 equal subcubes, kappa = 10**U(lo, hi).

    Node (i, j, k) belongs to subcube (floor(cubes*i/nx), floor(cubes*j/ny),
    floor(cubes*k/nz)).  The subcube values are drawn as one (cubes, cubes,
    cubes) array indexed [cz, cy, cx] from numpy's PCG64 generator.
    """
    rng = np.random.default_rng(seed)
    logk = rng.uniform(log10_lo, log10_hi, size=(cubes, cubes, cubes))
    ci = (cubes * np.arange(nx)) // nx
    cj = (cubes * np.arange(ny)) // ny
    ck = (cubes * np.arange(nz)) // nz
    vals = 10.0 ** logk
    return np.ascontiguousarray(vals[ck[:, None, None], cj[None, :, None], ci[None, None, :]])


def kappa_layers(nx: int, ny: int, nz: int, seed: int, layers: int = 8,
                 log10_lo: float = -4.0, log10_hi: float = 4.0) -> np.ndarray:
    """kappa constant on `layers` equal z-slabs (slab floor(layers*k/nz)), 10**U(lo, hi)."""
    rng = np.random.default_rng(seed)
    logk = rng.uniform(log10_lo, log10_hi, size=layers)
    ck = (layers * np.arange(nz)) // nz
    out = np.empty((nz, ny, nx), dtype=np.float64)
    out[:] = (10.0 ** logk[ck])[:, None, None]
    return out


def kappa_spheres(nx: int, ny: int, nz: int, seed: int, count: int = 200,
                  r_lo: float = 0.02, r_hi: float = 0.08,
                  inside: float = 1.0e6, outside: float = 1.0) -> np.ndarray:
    """High-contrast inclusions: `count` spheres, centres U[0,1]^3, radii U(r_lo, r_hi).

    Membership is tested at node coordinates; spheres may overlap and be clipped
    by the domain.  Draw order: all centres (count x 3, columns x, y, z), then radii.
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(count, 3))
    radii = rng.uniform(r_lo, r_hi, size=count)
    x, y, z = node_coords(nx, ny, nz)
    xs, ys, zs = x[0, 0, :], y[0, :, 0], z[:, 0, 0]
    out = np.full((nz, ny, nx), float(outside), dtype=np.float64)
    for (cx, cy, cz), r in zip(centres, radii):
        # Bounding box of the sphere in index space, then an exact test inside it.
        def rng_idx(coords, c):
            lo = np.searchsorted(coords, c - r, side="left")
            hi = np.searchsorted(coords, c + r, side="right")
            return lo, hi
        i0, i1 = rng_idx(xs, cx)
        j0, j1 = rng_idx(ys, cy)
        k0, k1 = rng_idx(zs, cz)
        if i0 >= i1 or j0 >= j1 or k0 >= k1:
            continue
        dx = (xs[i0:i1] - cx)[None, None, :]
        dy = (ys[j0:j1] - cy)[None, :, None]
        dz = (zs[k0:k1] - cz)[:, None, None]
        inside_mask = dx * dx + dy * dy + dz * dz <= r * r
        blk = out[k0:k1, j0:j1, i0:i1]
        blk[inside_mask] = float(inside)
    return out


def kappa_paper_type1(n: int) -> np.ndarray:
    """Type 1 'skyscraper' field (Sec. 3, test matrices): at node x,
    kappa = 1e3*(floor(10*x_2) + 1) when floor(10*x_i) is even for i = 1, 2, 3,
    else 1.  x_2 is the y coordinate; [.] is read as the integer part."""
    x, y, z = node_coords(n, n, n)
    fx, fy, fz = np.floor(10 * x), np.floor(10 * y), np.floor(10 * z)
    even = ((fx % 2) == 0) & ((fy % 2) == 0) & ((fz % 2) == 0)
    val = 1.0e3 * (fy + 1.0)
    out = np.where(even, np.broadcast_to(val, even.shape), 1.0)
    return np.ascontiguousarray(out, dtype=np.float64)


def kappa_paper_type2(n: int, inner: float | None = None) -> np.ndarray:
    """Type 2 ring field (Sec. 3): kappa = 1e3 where inner <= |x - c| <= 1/2,
    c = (1/2, 1/2, 1/2), else 1.

    The inner radius is printed as "1/2 sqrt 2".  Taken as printed, (1/2)*sqrt(2)
    = 0.707 exceeds the outer radius 1/2, so the ring is empty and kappa = 1
    everywhere (the default, inner=None).  The paper's Type 2 rows of Table 1
    equal its Type 3 (kappa = 1) rows in every iteration count, which is what
    an empty ring gives.  inner = 1/(2 sqrt 2) = 0.354 gives the non-empty
    ring (kappa_paper_type2_ring)."""
    if inner is None:
        inner = 0.5 * np.sqrt(2.0)
    x, y, z = node_coords(n, n, n)
    r = np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2)
    out = np.where((r >= inner) & (r <= 0.5), 1.0e3, 1.0)
    return np.ascontiguousarray(out, dtype=np.float64)


def kappa_paper_type2_ring(n: int) -> np.ndarray:
    """The Type 2 ring with inner radius 1/(2 sqrt 2): a shell of kappa = 1e3
    between radii 0.354 and 0.5 around the cube's centre (touching the faces at
    their centres), kappa = 1 elsewhere."""
    return kappa_paper_type2(n, inner=1.0 / (2.0 * np.sqrt(2.0)))


def rhs_uniform(nx: int, ny: int, nz: int, seed: int) -> np.ndarray:
    """b ~ U[-1, 1] from PCG64(seed), drawn in (nz, ny, nx) order."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(nz, ny, nx))


def filter_ones(nx: int, ny: int, nz: int) -> np.ndarray:
    """The rowsum filter vector t = 1 (Sec. 1, eq. rowsum)."""
    return np.ones((nz, ny, nx), dtype=np.float64)


def filter_random(nx: int, ny: int, nz: int, seed: int, lo: float = 0.5,
                  hi: float = 2.0) -> np.ndarray:
    """A positive filter vector t ~ U[lo, hi], for tests of a general t."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(nz, ny, nx))


# ---------------------------------------------------------------------------
# Named workloads.  Each returns dict(kappa, bc, b, t, n=(nx, ny, nz)).
# ---------------------------------------------------------------------------

def workload(name: str) -> dict:
    name = name.lower()
    if name == "poisson32":          # 32^3, kappa = 1, Dirichlet everywhere
        n = 32
        return dict(n=(n, n, n), kappa=kappa_const(n, n, n), bc=BC_ALL_DIRICHLET.copy(),
                    b=rhs_uniform(n, n, n, 101), t=None)
    if name in ("jump128", "jump256"):  # subcube jumps, Dirichlet at z = 0 only
        n = 128 if name == "jump128" else 256
        sk, sb = (201, 202) if n == 128 else (601, 602)
        return dict(n=(n, n, n), kappa=kappa_subcubes(n, n, n, sk), bc=BC_Z0_DIRICHLET.copy(),
                    b=rhs_uniform(n, n, n, sb), t=None)
    if name == "spheres350":         # 200 high-contrast spheres, b = 1
        n = 350
        return dict(n=(n, n, n), kappa=kappa_spheres(n, n, n, 301), bc=BC_ALL_DIRICHLET.copy(),
                    b=np.ones((n, n, n)), t=None)
    raise KeyError(name)


def batch_systems(count: int = 64, nrhs: int = 4, n_lo: int = 32, n_hi: int = 96,
                  seed: int = 401, n_fixed: int | None = None) -> list:
    """A batch of independent cubic systems: side n_s ~ U{n_lo..n_hi} from
    PCG64(seed) (or n_fixed for every system), kappa constant on 8 z-slabs,
    10**U(-4, 4) from PCG64(4100 + s), Dirichlet on every face, and nrhs
    right-hand sides b ~ U[-1, 1] from PCG64(4200 + 4 s + r).  Returns one
    dict(n, kappa, bc, bs) per system."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(n_lo, n_hi + 1, size=count)
    out = []
    for s in range(count):
        n = int(n_fixed) if n_fixed is not None else int(sides[s])
        out.append(dict(n=(n, n, n), kappa=kappa_layers(n, n, n, 4100 + s),
                        bc=BC_ALL_DIRICHLET.copy(),
                        bs=[rhs_uniform(n, n, n, 4200 + 4 * s + r) for r in range(nrhs)]))
    return out


def scaled_workload(name: str, n: int) -> dict:
    """The generator of a named workload at another cubic size n (same seeds)."""
    name = name.lower()
    if name == "poisson":
        return dict(n=(n, n, n), kappa=kappa_const(n, n, n), bc=BC_ALL_DIRICHLET.copy(),
                    b=rhs_uniform(n, n, n, 101), t=None)
    if name == "jump":
        return dict(n=(n, n, n), kappa=kappa_subcubes(n, n, n, 201), bc=BC_Z0_DIRICHLET.copy(),
                    b=rhs_uniform(n, n, n, 202), t=None)
    if name == "spheres":
        return dict(n=(n, n, n), kappa=kappa_spheres(n, n, n, 301), bc=BC_ALL_DIRICHLET.copy(),
                    b=np.ones((n, n, n)), t=None)
    if name in ("paper1", "paper2", "paper3", "paper2ring"):
        # Sec. 3 test matrices, Dirichlet everywhere.  The paper does not state
        # its right-hand side; b = A x* with a manufactured solution
        # x* ~ U[-1,1] (seed 701) reproduces Table 1's iteration counts.  Each
        # side forms b with its own SpMV from "xstar".
        kappa = {"paper1": kappa_paper_type1, "paper2": kappa_paper_type2,
                 "paper2ring": kappa_paper_type2_ring,
                 "paper3": lambda m: kappa_const(m, m, m)}[name](n)
        return dict(n=(n, n, n), kappa=kappa, bc=BC_ALL_DIRICHLET.copy(),
                    xstar=rhs_uniform(n, n, n, 701), b=None, t=None)
    raise KeyError(name)


def kappa_mixture(n: int, seed: int) -> np.ndarray:
    """A field of the learned-filter sets: from PCG64(seed) draw the kind
    (subcubes / z-layers / spheres, equally likely), the contrast exponent
    c ~ U(2, 6) and a sub-seed; subcubes (4 or 8 per side) and layers (8) take
    kappa = 10**U(0, c), spheres (20..100, radii U(0.02, 0.08)) kappa = 10**c
    inside and 1 outside."""
    rng = np.random.default_rng(seed)
    kind = int(rng.integers(3))
    c = float(rng.uniform(2.0, 6.0))
    sub = int(rng.integers(1 << 30))
    if kind == 0:
        return kappa_subcubes(n, n, n, sub, cubes=int(rng.choice([4, 8])), log10_lo=0.0,
                              log10_hi=c)
    if kind == 1:
        return kappa_layers(n, n, n, sub, layers=8, log10_lo=0.0, log10_hi=c)
    return kappa_spheres(n, n, n, sub, count=int(rng.integers(20, 101)), inside=10.0 ** c,
                         outside=1.0)


CNN_LAYERS = [(1, 16), (16, 16), (16, 16), (16, 1)]   # (cin, cout) of the filter network


def cnn_init_params(seed: int) -> np.ndarray:
    """Initial parameters of the filter network (float32, per layer W[cout][27][cin]
    then b[cout]): He-normal weights (std sqrt(2 / (27 cin))) from PCG64(seed),
    zero biases except the last, log(e^(1 - 1e-3) - 1), which makes the output
    softplus(b) + 1e-3 equal 1 where the features vanish."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in CNN_LAYERS:
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (27 * ci)), size=co * 27 * ci))
        parts.append(np.zeros(co))
    p = np.concatenate(parts)
    p[-1] = np.log(np.expm1(1.0 - 1.0e-3))
    return p.astype(np.float32)
