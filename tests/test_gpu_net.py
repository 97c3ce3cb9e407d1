"""GPU parity of the learned narrow-band cull: the network's forward pass and
gradients (bf16 matrix cores, float32 accumulation) against the float64
oracle (oracle/mlp.py), Adam's step, training, and the culled grid.

Tolerances, element by element.  The oracle is given the same bf16-rounded
weights W2..W4 the device multiplies with; what remains is the device's own
rounding, propagated through the layers as a first-order bound per entry
(forward_bounds / gradient_bounds below): the float32 input and first layer,
SiLU with the hardware exponential and reciprocal, the activations h1..h3
stored in bf16 (relative error 2^-8), float32 accumulation of the products,
and in the backward pass the products dZ^T H and dZ W taken with dZ and H in
bf16.  SiLU is 1.1-Lipschitz and its derivative 0.5-Lipschitz, which carries
an error of z into h and into dZ.  Every output and every gradient entry
must lie within its bound; the largest observed share of the bound is
printed.  The cull decisions use the forward bound as their margin: a brick
must be kept when the oracle keeps it with every prediction moved within its
bound, and may be kept only when some such move would keep it.
"""
import math
import sys

import numpy as np
import pytest

from oracle import mlp as M
from oracle import rbf_oracle as o
from paper_1305_5179_amd import workloads as w

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
UB = 2.0 ** -8          # bf16 unit roundoff (8-bit significand, round to nearest)
LIP1, LIP2 = 1.0998, 0.5   # max |silu'|, max |silu''|
GAM_MFMA = 130 * U32    # float32 accumulation of 128 products


def _silu_err(z, h):
    """SiLU on the device: z * rcp(1 + exp(-z)) with the hardware exp2 (its
    argument -z log2 e rounded) and reciprocal."""
    return (8.0 + 2.0 * np.abs(z)) * U32 * np.abs(h)


class _Worst:
    """Worst-case combination: every rounding error at its largest, all with
    the same sign, SiLU at its largest slope: a bound."""
    @staticmethod
    def mm(err, mag):                # errors of one factor through a product
        return err @ mag

    @staticmethod
    def add(*terms):
        return sum(terms)

    @staticmethod
    def total(err, axis=0):          # a sum over the samples
        return err.sum(axis)

    @staticmethod
    def slope(z):
        return LIP1


class _RootSumSquare:
    """The same rounding magnitudes combined in quadrature (independent
    errors), SiLU at its actual slope: an estimate of the typical error, not
    a bound; the tests allow a fixed multiple of it."""
    @staticmethod
    def mm(err, mag):
        return np.sqrt((err * err) @ (mag * mag))

    @staticmethod
    def add(*terms):
        return np.sqrt(sum(t * t for t in terms))

    @staticmethod
    def total(err, axis=0):
        return np.sqrt((err * err).sum(axis))

    @staticmethod
    def slope(z):
        return np.abs(M.silu_grad(z))


RSS_FACTOR = 8.0


def forward_bounds(P, U, C=_Worst):
    """Oracle output y and the error of the device's y per sample (a bound
    with C = _Worst), with the intermediate terms the backward pass needs."""
    y, (hs, zs) = M.forward(P, U)
    aU = np.abs(U)
    dU = U32 * aU
    W1, b1 = P[0]
    ez = [C.add(C.mm(dU, np.abs(W1).T), 3 * U32 * (aU @ np.abs(W1).T + np.abs(b1)))]
    ehb = []
    for l in (1, 2, 3):                       # inputs h1..h3 of the matrix-core layers
        z, h = zs[l - 1], hs[l]
        dh = C.add(C.slope(z) * ez[-1], _silu_err(z, h))
        dhb = C.add(dh, UB * (np.abs(h) + dh))      # stored in bf16
        ehb.append(dhb)
        W, b = P[l]
        ez.append(C.add(C.mm(dhb, np.abs(W).T), GAM_MFMA * ((np.abs(h) + dhb) @ np.abs(W).T + np.abs(b))))
    dh4 = C.add(C.slope(zs[3]) * ez[-1], _silu_err(zs[3], hs[4]))   # float32, not rounded
    W5, b5 = P[4]
    dy = C.add(C.mm(dh4, np.abs(W5).T), GAM_MFMA * ((np.abs(hs[4]) + dh4) @ np.abs(W5).T + np.abs(b5)))
    return y, dy[:, 0], dict(hs=hs, zs=zs, ez=ez, ehb=ehb, dh4=dh4)


def gradient_bounds(P, U, t, y, dy, fb, C=_Worst):
    """Oracle gradients' error bound per entry [(dW_l, db_l)] of the mean
    squared error (an estimate with C = _RootSumSquare)."""
    hs, zs, ez, ehb = fb["hs"], fb["zs"], fb["ez"], fb["ehb"]
    B = len(t)
    gam = (B + 64 + 130) * U32                 # float32 sums over the samples
    e = y - t
    de = C.add(dy, U32 * np.abs(t), U32 * np.abs(e))
    g5 = (2.0 / B) * e
    dg5 = C.add((2.0 / B) * de, U32 * np.abs(g5))
    out = [None] * 5
    h4, dh4 = hs[4], fb["dh4"]
    dW5 = C.add(C.mm(dg5[None, :], np.abs(h4))[0], C.mm(np.abs(g5)[None, :], dh4)[0],
                gam * (np.abs(g5) @ np.abs(h4)))
    out[4] = (dW5[None, :], np.array([C.add(C.total(dg5), gam * np.abs(g5).sum())]))
    w5 = P[4][0][0]
    s4 = M.silu_grad(zs[3])
    dZ = g5[:, None] * w5[None, :] * s4
    ddZ = C.add(np.abs(w5)[None, :] * dg5[:, None] * np.abs(s4),
                np.abs(w5)[None, :] * np.abs(g5)[:, None] * LIP2 * ez[3], 8 * U32 * np.abs(dZ))
    for L in (2, 1, 0):                        # weights P[L+1] = W_{L+2}, input h_{L+1}
        W = P[L + 1][0]
        ddZb = C.add(ddZ, UB * (np.abs(dZ) + ddZ))   # the bf16 copy the products take
        db = C.add(C.total(ddZ), gam * np.abs(dZ).sum(0))
        h, dhb = hs[L + 1], ehb[L]
        dW = C.add(C.mm(ddZb.T, np.abs(h)), C.mm(np.abs(dZ).T, dhb), C.mm(ddZb.T, dhb),
                   gam * (np.abs(dZ).T @ np.abs(h)))
        out[L + 1] = (dW, db)
        dH = dZ @ W
        ddH = C.add(C.mm(ddZb, np.abs(W)), GAM_MFMA * ((np.abs(dZ) + ddZb) @ np.abs(W)))
        sb = M.silu_grad(zs[L])
        dZn = dH * sb
        ddZ = C.add(ddH * (np.abs(sb) + LIP2 * ez[L]), np.abs(dH) * LIP2 * ez[L], 8 * U32 * np.abs(dZn))
        dZ = dZn
    aU = np.abs(U)
    out[0] = (C.add(C.mm(ddZ.T, aU), C.mm(np.abs(dZ).T, U32 * aU), gam * (np.abs(dZ).T @ aU)),
              C.add(C.total(ddZ), gam * np.abs(dZ).sum(0)))
    return out


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
    yo, dy, _ = forward_bounds(oracle_params(flat), U)
    _, ry, _ = forward_bounds(oracle_params(flat), U, _RootSumSquare)
    err = np.abs(y - yo)
    _say(f"[net] forward: largest |y - y_oracle| / bound {np.max(err / dy):.2e}, / root-sum-square "
         f"estimate {np.max(err / ry):.3f}; relative L2 {np.linalg.norm(y - yo) / np.linalg.norm(yo):.2e}")
    assert np.all(err <= dy)
    assert np.all(err <= RSS_FACTOR * ry)
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
    t = f / TAU
    yo, dy, fb = forward_bounds(P, U)
    G = M.backward(P, (fb["hs"], fb["zs"]), yo, t)
    Gb = gradient_bounds(P, U, t, yo, dy, fb)
    _, ry, fr = forward_bounds(P, U, _RootSumSquare)
    Gr = gradient_bounds(P, U, t, yo, ry, fr, _RootSumSquare)
    e = np.abs(yo - t)
    assert abs(loss - M.loss(yo, t)) <= np.mean(2 * e * dy + dy * dy) + 1e-5 * M.loss(yo, t)
    off = 0
    for l, ((gW, gb), (bW, bb), (rW, rb)) in enumerate(zip(G, Gb, Gr)):
        for ref, bound, est in ((gW.reshape(-1), bW.reshape(-1), rW.reshape(-1)), (gb, bb, rb)):
            got = g[off:off + ref.size]
            off += ref.size
            err = np.abs(got - ref)
            _say(f"[net] layer {l + 1} block of {ref.size}: largest |g - g_oracle| / bound {np.max(err / bound):.2e}, "
                 f"/ root-sum-square estimate {np.max(err / est):.3f}")
            assert np.all(err <= bound), l
            assert np.all(err <= RSS_FACTOR * est), l
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
        yo, dyo, _ = forward_bounds(oracle_params(flat), U)
        assert np.all(np.abs(y - yo) <= dyo)
        delta = float(np.max(dyo))
        e_val = 4 * 3e-2 * np.sqrt(np.mean(yo ** 2))
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
