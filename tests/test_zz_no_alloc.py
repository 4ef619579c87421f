"""ntd_dot_noalloc (the allocation-free dot product for callers that cannot
allocate) against ntd_dot, through the C ABI: the same kernels in the same
order, so the results must agree bitwise, and both within 1e-14 * sum |x y|
of the oracle's compensated sum.  Two calls in a row share the static scratch
array; the second has a smaller input, so stale partial sums of the first call
would show up in it."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)


def test_dot_noalloc_matches_ntd_dot_on_two_calls():
    import paper_1909_09771_amd as P
    L = P.lib()
    res = torch.full((1,), np.nan, dtype=torch.float64, device=DEV)
    for shape, seed in (((37, 41, 129), 1), ((3, 5, 67), 2)):
        n = int(np.prod(shape))
        rng = np.random.default_rng(seed)
        x, y = rng.uniform(-1, 1, shape), rng.uniform(-1, 1, shape)
        xg = torch.from_numpy(x).to(DEV)
        yg = torch.from_numpy(y).to(DEV)
        st = L.ntd_dot_noalloc(_ptr(xg), _ptr(yg), n, _ptr(res), _stream())
        assert st == P.OK
        torch.cuda.synchronize()
        got = float(res.cpu()[0])
        S = P.Solver(torch.ones(shape, dtype=torch.float64, device=DEV), [0] * 6, prec="fp64",
                     schur="diag")
        want = S.dot(xg, yg)
        print("n = %d: noalloc %.17g, ntd_dot %.17g" % (n, got, want))
        assert got == want
        assert abs(got - O.dot(x, y)) <= 1e-14 * np.abs(x * y).sum()


def test_dot_noalloc_edge_cases():
    import paper_1909_09771_amd as P
    L = P.lib()
    x = torch.ones(5, dtype=torch.float64, device=DEV)
    res = torch.full((1,), np.nan, dtype=torch.float64, device=DEV)
    assert L.ntd_dot_noalloc(_ptr(x), _ptr(x), 0, _ptr(res), _stream()) == P.OK
    torch.cuda.synchronize()
    assert float(res.cpu()[0]) == 0.0
    assert L.ntd_dot_noalloc(_ptr(x), _ptr(x), 5, _ptr(res), _stream()) == P.OK
    torch.cuda.synchronize()
    assert float(res.cpu()[0]) == 5.0
    assert L.ntd_dot_noalloc(_ptr(x), _ptr(x), -1, _ptr(res), _stream()) == P.EINVAL
    assert L.ntd_dot_noalloc(_ptr(x), _ptr(x), (1 << 50) + 1, _ptr(res), _stream()) == P.EINVAL
    assert L.ntd_dot_noalloc(None, _ptr(x), 5, _ptr(res), _stream()) == P.EINVAL
