"""GPU parity of the learned narrow-band cull: the network's forward pass and
gradients (bf16 matrix cores, float32 accumulation) against the float64
oracle (oracle/mlp.py), Adam's step, training, and the culled grid.

Tolerances.  The matrix-core layers take bf16 operands: the weights W2..W4
are rounded to bf16 on both sides (the oracle is given the same rounded
values), the activations h1..h3 only on the device, each with a relative
error of at most 2^-9.  Through three layers this stays near 1 % of the
output; the tests allow 3 % (relative L2 over the batch) for y and for the
gradient of every layer, and use the forward bound as the margin of the
cull decisions: a brick must be kept when the oracle keeps it with every
prediction moved by that margin, and may be kept only when some such move
would keep it.
"""
import math
import sys

import numpy as np
import pytest

from oracle import mlp as M
from oracle import rbf_oracle as o
from paper_1305_5179_amd import workloads as w

pytestmark = pytest.mark.gpu

REL = 3e-2


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
    rbf.load_library()
    return rbf


def dev(torch, a, dtype=None):
    import torch as t
    return t.as_tensor(np.ascontiguousarray(a, dtype=np.float64 if dtype is None else dtype), device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def bf16(a):
    """Round float32 values to the nearest bf16 (ties to even)."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def oracle_params(flat):
    P = w.net_unflatten(flat)
    return [(W if l in (0, 4) else bf16(W), b) for l, (W, b) in enumerate(P)]


CENTRE, SCALE, TAU = (0.1, -0.2, 0.05), 0.9, 0.01


@pytest.fixture(scope="module")
def net_ctx(torch, R):
    c = w.sphere(300, 3)
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), 0.05, 0.1, math.inf)
    yield ctx
    ctx.close()


def test_forward_matches_oracle(torch, R, net_ctx):
    flat = w.net_init(8)
    net_ctx.net_set(flat, CENTRE, SCALE, TAU)
    X = np.random.default_rng(1).uniform(-1.2, 1.2, size=(3000, 3))
    _say("[net] forward 3000")
    y = host(net_ctx.net_forward(dev(torch, X)))
    torch.cuda.synchronize()
    U = (X - np.array(CENTRE)) * SCALE
    yo, _ = M.forward(oracle_params(flat), U)
    err = np.linalg.norm(y - yo) / np.linalg.norm(yo)
    _say(f"[net] forward relative L2 error {err:.3e}")
    assert err <= REL
    assert np.array_equal(net_ctx.net_get(), flat)       # the parameters round-trip unchanged


def test_gradient_matches_oracle(torch, R, net_ctx):
    flat = w.net_init(9)
    net_ctx.net_set(flat, CENTRE, SCALE, TAU)
    rng = np.random.default_rng(2)
    X = rng.uniform(-1.2, 1.2, size=(1000, 3))     # not a multiple of 64: a ragged workgroup
    f = rng.uniform(-0.02, 0.02, size=1000)
    _say("[net] gradient 1000")
    g, loss = net_ctx.net_gradient(dev(torch, X), dev(torch, f))
    torch.cuda.synchronize()
    g = host(g)
    P = oracle_params(flat)
    U = (X - np.array(CENTRE)) * SCALE
    yo, cache = M.forward(P, U)
    G = M.backward(P, cache, yo, f / TAU)
    assert abs(loss - M.loss(yo, f / TAU)) <= REL * M.loss(yo, f / TAU)
    off = 0
    for l, (gW, gb) in enumerate(G):
        for ref in (gW.reshape(-1), gb):
            got = g[off:off + ref.size]
            off += ref.size
            rel = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30)
            _say(f"[net] layer {l + 1} block of {ref.size}: relative L2 {rel:.3e}")
            assert rel <= REL, (l, rel)
    assert off == R.RBF_NET_PARAMS


def test_adam_step_and_training(torch, R, net_ctx):
    flat = w.net_init(10)
    net_ctx.net_set(flat, CENTRE, SCALE, TAU)
    rng = np.random.default_rng(3)
    X = rng.uniform(-1, 1, size=(4096, 3))
    f = 0.01 * np.tanh(3 * (np.linalg.norm(X, axis=1) - 0.7))     # a smooth signed field
    lr = 1e-3
    _say("[net] one Adam step")
    net_ctx.net_train(dev(torch, X), dev(torch, f), 4096, 1, lr)
    after = net_ctx.net_get().astype(np.float64)
    step = after - flat.astype(np.float64)
    # the first Adam step moves every parameter by lr g / (|g| + eps) <= lr
    assert np.abs(step).max() <= lr * (1 + 1e-3)
    P = oracle_params(flat)
    U = (X - np.array(CENTRE)) * SCALE
    yo, cache = M.forward(P, U)
    G = np.concatenate([np.concatenate([gW.reshape(-1), gb]) for gW, gb in M.backward(P, cache, yo, f / TAU)])
    big = np.abs(G) > 0.1 * np.abs(G).max()
    assert np.all(np.sign(step[big]) == -np.sign(G[big]))
    assert np.allclose(np.abs(step[big]), lr, rtol=1e-3)
    _say("[net] 40 epochs")
    first = net_ctx.net_gradient(dev(torch, X), dev(torch, f))[1]
    last = net_ctx.net_train(dev(torch, X), dev(torch, f), 512, 40, lr)
    torch.cuda.synchronize()
    _say(f"[net] loss {first:.3e} -> {last:.3e}")
    assert last < 0.1 * first


def _exact_support(X, rc, g):
    from scipy.spatial import cKDTree
    nx, ny, nz = g.dims
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    nodes = np.stack([g.origin[0] + i * g.h[0], g.origin[1] + j * g.h[1], g.origin[2] + k * g.h[2]], -1)
    nodes = nodes.transpose(2, 1, 0, 3).reshape(-1, 3)          # x fastest
    d, _ = cKDTree(X).query(nodes, distance_upper_bound=rc * (1 + 1e-9))
    near = np.isfinite(d).reshape(nz, ny, nx)
    bx, by, bz = -(-nx // 4), -(-ny // 2), -(-nz // 2)
    sup = np.zeros((bz, by, bx), dtype=bool)
    zz, yy, xx = np.nonzero(near)
    sup[zz // 2, yy // 2, xx // 4] = True
    return nodes, sup.reshape(-1)


def test_culled_grid(torch, R):
    c = w.torus(n=6000, seed=1, R=0.1732, r=0.0606)
    eps, sigma, rc = 0.005, 0.02, 0.08
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), eps, sigma, rc)
    try:
        g = w.Grid.around(c.points, 48)
        cube_c = np.array(g.origin) + 0.5 * (np.array(g.dims) - 1) * np.array(g.h)
        scale = 2.0 / ((np.array(g.dims).max() - 1) * np.array(g.h).max())
        X, b = o.extended_centres(c.points, c.normals, eps)
        nodes, sup = _exact_support(X, rc, g)
        # a seeded network whose output changes sign over the grid: its last
        # bias moved by the oracle's median prediction on the support nodes
        flat = w.net_init(11)
        U = (nodes - cube_c) * scale
        node_sup = np.repeat(np.repeat(np.repeat(sup.reshape(-(-g.dims[2] // 2), -(-g.dims[1] // 2), -(-g.dims[0] // 4)),
                                                 2, 0), 2, 1), 4, 2)[:g.dims[2], :g.dims[1], :g.dims[0]].reshape(-1)
        flat[-1] = np.float32(flat[-1] - np.median(M.forward(oracle_params(flat), U[node_sup])[0]))
        ctx.net_set(flat, cube_c, scale, TAU)
        coef = np.random.default_rng(5).uniform(-1, 1, len(X))
        cw = dev(torch, coef)
        _say("[net] culled grid 48^3")
        plain = host(ctx.eval_grid(cw, g.origin, g.h, g.dims, prec=R.RBF_FP32))
        y = host(ctx.net_forward(dev(torch, nodes)))
        yo, _ = M.forward(oracle_params(flat), U)
        delta = 3 * REL * np.sqrt(np.mean(yo ** 2))
        e_val = 4 * delta
        out, st = ctx.eval_grid_culled(cw, g.origin, g.h, g.dims, e_val)
        out = host(out)
        torch.cuda.synchronize()
        _say(f"[net] support {st.support_bricks} kept {st.kept_bricks}")
        assert 0 < st.kept_bricks < st.support_bricks
        # every node is the exact sum, or tau * y (culled support), bit for bit
        culled_val = (np.float32(TAU) * y.astype(np.float32)).astype(np.float64)
        assert np.all((out == plain) | (out == culled_val))
        exact_only = (out == plain) & (out != culled_val)
        culled_only = (out == culled_val) & (out != plain)
        nx, ny, nz = g.dims
        bid = ((np.arange(nz)[:, None, None] // 2) * (-(-ny // 2)) + (np.arange(ny)[None, :, None] // 2)) \
            * (-(-nx // 4)) + np.arange(nx)[None, None, :] // 4
        bid = bid.reshape(-1)
        nb = sup.size
        kept_b = np.zeros(nb, dtype=bool)
        np.logical_or.at(kept_b, bid, exact_only)
        culled_b = np.zeros(nb, dtype=bool)
        np.logical_or.at(culled_b, bid, culled_only)
        assert not np.any(kept_b & culled_b & sup)          # a support brick is one or the other
        # The oracle's decisions with every prediction moved by up to delta.
        # The library's support (bricks near occupied cells) contains the
        # exact one (a node within the cutoff of a centre) and lies within
        # about twice the cutoff of the centres: signed neighbours are taken
        # from the exact support for what must be kept, from the wider one for
        # what may be.
        _, sup_wide = _exact_support(X, 2.5 * rc, g)
        amb = np.abs(yo) <= delta
        lo = M.brick_cull(np.where(amb, 0.0, yo), sup, g.dims, e_val - delta)
        hi = (M.brick_cull(np.where(amb, -0.5 * delta, yo), sup_wide, g.dims, e_val + delta)
              | M.brick_cull(np.where(amb, 0.5 * delta, yo), sup_wide, g.dims, e_val + delta))
        must = lo & sup
        assert not np.any(culled_b[must]), np.nonzero(must & culled_b)[0][:10]
        assert not np.any(kept_b & sup & ~hi), np.nonzero(kept_b & sup & ~hi)[0][:10]
        _say(f"[net] oracle: must keep {must.sum()}, may keep {(hi & sup).sum()} of {sup.sum()} support bricks")
    finally:
        ctx.close()


@pytest.mark.parametrize("dims", [(1, 1, 1), (5, 3, 3), (9, 2, 7)])
def test_culled_grid_small_shapes_and_no_cutoff(torch, R, dims):
    """No cutoff (every brick in the support) and ragged or single-node
    grids: every node is the exact sum or tau * y, bit for bit."""
    c = w.sphere(200, 4)
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), 0.05, 0.2, math.inf)
    try:
        X, _ = o.extended_centres(c.points, c.normals, 0.05)
        origin, h = (-1.1, -1.0, -0.9), (2.2 / max(dims[0] - 1, 1), 2.0 / max(dims[1] - 1, 1), 1.8 / max(dims[2] - 1, 1))
        flat = w.net_init(12)
        ctx.net_set(flat, (0.0, 0.0, 0.0), 0.8, TAU)
        cw = dev(torch, np.random.default_rng(6).uniform(-1, 1, len(X)))
        _say(f"[net] culled grid {dims} without cutoff")
        plain = host(ctx.eval_grid(cw, origin, h, dims, prec=R.RBF_FP32))
        out, st = ctx.eval_grid_culled(cw, origin, h, dims, 0.05)
        out = host(out)
        nx, ny, nz = dims
        i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
        nodes = np.stack([origin[0] + i * h[0], origin[1] + j * h[1], origin[2] + k * h[2]], -1)
        nodes = nodes.transpose(2, 1, 0, 3).reshape(-1, 3)
        y = host(ctx.net_forward(dev(torch, nodes)))
        torch.cuda.synchronize()
        culled_val = (np.float32(TAU) * y.astype(np.float32)).astype(np.float64)
        assert np.all((out == plain) | (out == culled_val))
        nb = (-(-nx // 4)) * (-(-ny // 2)) * (-(-nz // 2))
        assert st.support_bricks == nb and 0 <= st.kept_bricks <= nb
    finally:
        ctx.close()


def test_training_edge_cases(torch, R, net_ctx):
    flat = w.net_init(13)
    net_ctx.net_set(flat, CENTRE, SCALE, TAU)
    X = np.random.default_rng(7).uniform(-1, 1, size=(100, 3))
    f = np.random.default_rng(8).uniform(-0.01, 0.01, size=100)
    assert net_ctx.net_train(dev(torch, X), dev(torch, f), 64, 0, 1e-3) == 0.0      # no epochs: no change
    assert np.array_equal(net_ctx.net_get(), flat)
    loss = net_ctx.net_train(dev(torch, X), dev(torch, f), 4096, 3, 1e-3)        # batch above n
    assert math.isfinite(loss)
    with pytest.raises(R.RbfError):
        net_ctx.net_train(dev(torch, X), dev(torch, f), 0, 1, 1e-3)
    with pytest.raises(R.RbfError):
        net_ctx.net_set(np.full(R.RBF_NET_PARAMS, np.nan, dtype=np.float32), CENTRE, SCALE, TAU)
