"""CPU oracle of the learned narrow-band cull (FP64).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The GPU library
never calls it, links it or shares code with it.

Sec. II.A.3 evaluates the interpolant only in a narrow volume around the
surface, M_ext^eps = {x : d(x, M) <= eps}, since the zero level set away
from M is an artefact.  The learned variant replaces the distance test by a
small network that predicts the interpolant from the position, trained on
(position, interpolant) pairs the interpolant itself supplies; the exact sum
is kept where the network's sign may be wrong.  Readings (design notes):

  * Network: u -> 128 -> 128 -> 128 -> 128 -> 1, SiLU after every hidden
    layer (silu(z) = z / (1 + exp(-z))), u = (x - centre) * scale the
    position normalised to the grid cube, output y ~ f(x) / tau.
  * Loss: mean over the batch of (y - t)^2, t = f / tau.
  * Adam (Kingma and Ba): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
    theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
  * Cull, on bricks of 4 x 2 x 2 grid nodes: a support brick (one with a
    centre within the cutoff of its node box) is kept when one of its nodes
    has |y| < e_val, or has a support node with the opposite sign of y within
    3 grid steps along every axis; kept bricks get the exact sum, the other
    support bricks tau * y, nodes outside the support 0.
"""
from __future__ import annotations

import numpy as np

__all__ = ["silu", "silu_grad", "forward", "backward", "loss", "adam_step", "init_params",
           "brick_cull"]

WIDTH = 128
LAYERS = 4          # hidden layers


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    """d silu / dz = s (1 + z (1 - s)), s = 1 / (1 + exp(-z))."""
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(W_list, b_list):
    """Parameters as float64 arrays: [(W1, b1), ..., (W5, b5)], W_l of shape
    (out, in).  The initial values are inputs (drawn by the caller)."""
    return [(np.asarray(W, dtype=np.float64).copy(), np.asarray(b, dtype=np.float64).copy())
            for W, b in zip(W_list, b_list)]


def forward(params, U):
    """y (B,) and the cache of pre-activations z_l and activations h_l."""
    h = np.asarray(U, dtype=np.float64)
    hs, zs = [h], []
    for l, (W, b) in enumerate(params):
        z = h @ W.T + b
        zs.append(z)
        if l < len(params) - 1:
            h = silu(z)
            hs.append(h)
        else:
            h = z
    return h[:, 0], (hs, zs)


def loss(y, t):
    return float(np.mean((y - t) ** 2))


def backward(params, cache, y, t):
    """Gradients [(dW_l, db_l)] of the mean squared error."""
    hs, zs = cache
    B = y.shape[0]
    g = (2.0 / B) * (y - t)[:, None]                 # dL/dz of the output layer
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        grads[l] = (g.T @ hs[l], g.sum(axis=0))
        if l > 0:
            g = (g @ W) * silu_grad(zs[l - 1])
    return grads


def adam_step(params, grads, state, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); state = [(mW, vW, mb, vb)], updated."""
    out = []
    for l, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        mW, vW, mb, vb = state[l]
        mW = b1 * mW + (1 - b1) * gW
        vW = b2 * vW + (1 - b2) * gW * gW
        mb = b1 * mb + (1 - b1) * gb
        vb = b2 * vb + (1 - b2) * gb * gb
        c1, c2 = 1.0 - b1 ** t, 1.0 - b2 ** t
        W = W - lr * (mW / c1) / (np.sqrt(vW / c2) + eps)
        b = b - lr * (mb / c1) / (np.sqrt(vb / c2) + eps)
        state[l] = (mW, vW, mb, vb)
        out.append((W, b))
    return out


def brick_cull(y, support, dims, e_val, reach=3):
    """Kept bricks of the learned cull.

    y: network output at every node (x fastest), support: bool per brick
    (bricks of 4 x 2 x 2 nodes, x fastest), dims: nodes per axis.  A node
    belongs to the support when its brick does.  Returns a bool per brick."""
    nx, ny, nz = (int(d) for d in dims)
    bx, by, bz = -(-nx // 4), -(-ny // 2), -(-nz // 2)
    sup_b = np.asarray(support, dtype=bool).reshape(bz, by, bx)
    Y = np.asarray(y, dtype=np.float64).reshape(nz, ny, nx)
    # node support
    node_sup = np.repeat(np.repeat(np.repeat(sup_b, 2, axis=0), 2, axis=1), 4, axis=2)[:nz, :ny, :nx]
    pos = node_sup & (Y > 0)
    neg = node_sup & (Y < 0)
    near = node_sup & (np.abs(Y) < e_val)
    # a node sees an opposite sign within `reach` steps along every axis
    def dilate(m):
        out = np.zeros_like(m)
        for dz in range(-reach, reach + 1):
            for dy in range(-reach, reach + 1):
                for dx in range(-reach, reach + 1):
                    src = m[max(0, dz):nz + min(0, dz), max(0, dy):ny + min(0, dy), max(0, dx):nx + min(0, dx)]
                    out[max(0, -dz):nz + min(0, -dz), max(0, -dy):ny + min(0, -dy), max(0, -dx):nx + min(0, -dx)] |= src
        return out
    keep_node = near | (pos & dilate(neg)) | (neg & dilate(pos))
    keep_b = np.zeros((bz, by, bx), dtype=bool)
    zz, yy, xx = np.nonzero(keep_node)
    keep_b[zz // 2, yy // 2, xx // 4] = True
    return (keep_b & sup_b).reshape(-1)
