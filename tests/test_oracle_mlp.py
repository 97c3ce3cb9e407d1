"""Pins of the learned-cull oracle (CPU only): SiLU closed forms, gradients
against central finite differences, the first Adam step in closed form, and
the brick cull against a plain loop over nodes."""
import itertools
import math

import numpy as np

from oracle import mlp as M


def test_silu_closed_forms():
    assert M.silu(np.array(0.0)) == 0.0
    assert abs(M.silu(np.array(1.0)) - 1.0 / (1.0 + math.exp(-1.0))) < 1e-16
    assert abs(M.silu(np.array(40.0)) - 40.0) < 1e-12
    assert abs(M.silu(np.array(-40.0))) < 1e-15
    assert M.silu_grad(np.array(0.0)) == 0.5
    z = np.linspace(-6, 6, 25)
    h = 1e-6
    fd = (M.silu(z + h) - M.silu(z - h)) / (2 * h)
    assert np.abs(fd - M.silu_grad(z)).max() < 1e-9


def _params(rng, sizes):
    return [(rng.normal(size=(o, i)) / math.sqrt(i), rng.normal(size=o) * 0.1)
            for i, o in zip(sizes[:-1], sizes[1:])]


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    for sizes in ([3, 5, 4, 1], [3, 128, 128, 128, 128, 1]):
        P = M.init_params(*zip(*_params(rng, sizes)))
        U = rng.uniform(-1, 1, size=(6, 3))
        t = rng.normal(size=6)
        y, cache = M.forward(P, U)
        G = M.backward(P, cache, y, t)
        for l in range(len(P)):
            W, b = P[l]
            idx = [tuple(rng.integers(0, s) for s in W.shape) for _ in range(4)]
            for ij in idx:
                h = 1e-6
                Wp = [(w.copy(), bb.copy()) for w, bb in P]
                Wm = [(w.copy(), bb.copy()) for w, bb in P]
                Wp[l][0][ij] += h
                Wm[l][0][ij] -= h
                fd = (M.loss(M.forward(Wp, U)[0], t) - M.loss(M.forward(Wm, U)[0], t)) / (2 * h)
                assert abs(fd - G[l][0][ij]) <= 1e-6 * max(1.0, abs(fd)), (sizes, l, ij, fd, G[l][0][ij])
            k = int(rng.integers(0, b.size))
            Bp = [(w.copy(), bb.copy()) for w, bb in P]
            Bm = [(w.copy(), bb.copy()) for w, bb in P]
            Bp[l][1][k] += 1e-6
            Bm[l][1][k] -= 1e-6
            fd = (M.loss(M.forward(Bp, U)[0], t) - M.loss(M.forward(Bm, U)[0], t)) / 2e-6
            assert abs(fd - G[l][1][k]) <= 1e-6 * max(1.0, abs(fd))


def test_first_adam_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(1)
    P = [(rng.normal(size=(4, 3)), rng.normal(size=4))]
    G = [(rng.normal(size=(4, 3)), np.array([0.5, -2.0, 1e-3, -1e-4]))]
    state = [(np.zeros((4, 3)), np.zeros((4, 3)), np.zeros(4), np.zeros(4))]
    lr, eps = 1e-3, 1e-8
    out = M.adam_step(P, G, state, 1, lr, eps=eps)
    # m_hat = g, v_hat = g^2 after one step: the move is lr * g / (|g| + eps)
    assert np.allclose(P[0][0] - out[0][0], lr * G[0][0] / (np.abs(G[0][0]) + eps), rtol=1e-12, atol=0)
    assert np.allclose(P[0][1] - out[0][1], lr * G[0][1] / (np.abs(G[0][1]) + eps), rtol=1e-12, atol=0)


def _cull_by_loops(y, support, dims, e_val, reach=3):
    nx, ny, nz = dims
    bx, by = -(-nx // 4), -(-ny // 2)

    def brick(i, j, k):
        return (k // 2) * by * bx + (j // 2) * bx + i // 4

    def val(i, j, k):
        return y[(k * ny + j) * nx + i]

    keep = [False] * len(support)
    for i, j, k in itertools.product(range(nx), range(ny), range(nz)):
        b = brick(i, j, k)
        if not support[b]:
            continue
        v = val(i, j, k)
        hit = abs(v) < e_val
        for di, dj, dk in itertools.product(range(-reach, reach + 1), repeat=3):
            a, bb, c = i + di, j + dj, k + dk
            if hit or not (0 <= a < nx and 0 <= bb < ny and 0 <= c < nz):
                continue
            if support[brick(a, bb, c)] and val(a, bb, c) * v < 0:
                hit = True
        if hit:
            keep[b] = True
    return np.array(keep)


def test_brick_cull_matches_a_node_loop():
    rng = np.random.default_rng(2)
    for dims, slope in (((10, 6, 5), (1.0, 0.3, -0.2)), ((16, 8, 8), (1.0, 0.3, -0.2)),
                        ((8, 8, 16), (0.1, -0.2, 1.0)), ((8, 12, 6), (0.0, 1.0, 0.1))):
        nx, ny, nz = dims
        nb = (-(-nx // 4)) * (-(-ny // 2)) * (-(-nz // 2))
        # a smooth field with a zero level set across the longest axis, plus
        # noise, and a random support
        x, yv, z = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
        f = slope[0] * (x - nx / 2.3) + slope[1] * (yv - ny / 2.3) + slope[2] * (z - nz / 2.3)
        f = f.transpose(2, 1, 0).reshape(-1) + rng.normal(scale=0.05, size=nx * ny * nz)
        support = rng.uniform(size=nb) < 0.8
        for e_val in (0.0, 0.5):
            got = M.brick_cull(f, support, dims, e_val)
            want = _cull_by_loops(f, support, dims, e_val)
            assert np.array_equal(got, want), (dims, e_val)
            assert not np.any(got & ~support)
        if max(dims) >= 16:   # bricks more than 3 steps from the zero set: something is culled
            assert M.brick_cull(f, support, dims, 0.0).sum() < support.sum()


def test_brick_cull_threshold_is_strict():
    """|y| == e_val is not below the held-out error: nothing is kept on a
    field of one sign whose smallest value equals e_val."""
    dims = (8, 4, 4)
    y = np.full(8 * 4 * 4, 2.0)
    y[37] = 0.5
    support = np.ones(2 * 2 * 2, dtype=bool)
    assert not M.brick_cull(y, support, dims, 0.5).any()
    assert M.brick_cull(y, support, dims, 0.5000001).sum() == 1
