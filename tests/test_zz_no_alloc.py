"""rbf_eval_grid_noalloc, the grid evaluation for callers that cannot
allocate device memory: called through the C ABI, it must give exactly what
rbf_eval_grid gives (the same kernels, with their scratch memory in a fixed
device array instead of the library's allocator), on consecutive calls of
decreasing size, and refuse what it cannot hold."""
import ctypes as C
import math
import sys

import numpy as np
import pytest

from paper_1305_5179_amd import workloads as w

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def R():
    from paper_1305_5179_amd import rbf
    lib = rbf.load_library()
    lib.rbf_eval_grid_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(rbf.Grid), C.c_void_p, C.c_void_p]
    lib.rbf_eval_grid_noalloc.restype = C.c_int
    return rbf


def dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def noalloc(R, ctx, coef, g, out):
    gd = R.make_grid(g.origin, g.h, g.dims)
    return ctx._lib.rbf_eval_grid_noalloc(ctx.ctx, R._ptr(coef), C.byref(gd), R._ptr(out, "float32"), R._stream())


def test_noalloc_grid_equals_eval_grid_on_consecutive_calls(torch, R):
    cfg = w.TORUS_200K
    c = w.torus(cfg["n"], cfg["seed"])
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), cfg["eps"], cfg["sigma"], cfg["cutoff"])
    try:
        coef = dev(torch, np.random.default_rng(71).uniform(-1, 1, ctx.m))
        big = w.Grid.around(c.points, 256)            # 1,048,576 bricks
        # fewer nodes at the same spacing (and a ragged brick count per axis)
        off = np.array([20, 30, 100]) * np.array(big.h)
        small = w.Grid(tuple(float(v) for v in np.array(big.origin) + off), big.h, (201, 147, 93))
        for g in (big, small, big):
            ref = ctx.eval_grid(coef, g.origin, g.h, g.dims, prec=R.RBF_FP32)
            out = torch.full((g.size,), float("nan"), dtype=torch.float32, device="cuda")
            st = noalloc(R, ctx, coef, g, out)
            torch.cuda.synchronize()
            nz = int((ref != 0).sum())
            _say(f"[noalloc grid {g.dims}] status {st} nonzero nodes {nz}")
            assert st == R.RBF_OK
            assert nz > 0
            assert torch.equal(out, ref)
    finally:
        ctx.close()


def test_noalloc_grid_refuses_what_it_cannot_hold(torch, R):
    c = w.patch(w.torus(20000, seed=1), 500, seed=3)
    P, N = dev(torch, c.points), dev(torch, c.normals)
    ctx = R.Rbf(P, N, 0.005, 0.02, 0.08)
    coef = dev(torch, np.ones(ctx.m))
    try:
        # more bricks than the fixed array holds (2^21 bricks of 4 x 2 x 2 nodes)
        g = w.Grid(origin=(0.0, 0.0, 0.0), h=(1e-4, 1e-4, 1e-4), dims=(1024, 512, 256))
        out = torch.zeros(8, dtype=torch.float32, device="cuda")
        assert noalloc(R, ctx, coef, g, out) == R.RBF_EINVAL
        assert "holds at most" in ctx._lib.rbf_last_error(ctx.ctx).decode()
        # a grid too coarse for the brick sums
        g = w.Grid(origin=(-1.0, -1.0, -1.0), h=(0.5, 0.5, 0.5), dims=(5, 5, 5))
        out = torch.zeros(g.size, dtype=torch.float32, device="cuda")
        assert noalloc(R, ctx, coef, g, out) == R.RBF_EINVAL
    finally:
        ctx.close()
    ctx = R.Rbf(P, N, 0.005, 0.02, math.inf)   # no cutoff: no brick sums
    try:
        g = w.Grid.around(c.points, 16)
        out = torch.zeros(g.size, dtype=torch.float32, device="cuda")
        assert noalloc(R, ctx, dev(torch, np.ones(ctx.m)), g, out) == R.RBF_EINVAL
    finally:
        ctx.close()
