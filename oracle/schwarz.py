"""CPU oracle of the overlapping Schwarz preconditioner (FP64).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The GPU library
never calls it, links it or shares code with it.

Sec. III.A of the paper splits the domain of the cloud into overlapping
subdomains Omega_i with non-overlapping parts, solves the restricted systems
A_i x_i = b_i, and combines the local solutions: added up everywhere
(additive Schwarz) or kept only on the non-overlapping parts (restricted
additive Schwarz), used as a preconditioner of GMRES.  The paper leaves the
subdomains, the overlap and the local matrices open; the readings here
(each listed in the design notes):

  * Cores (the non-overlapping parts).  An octree over the surface points:
    the root cube has corner lo = the componentwise minimum of the points and
    side = the largest extent of their bounding box; a point's finest cell is
    q = floor((p - lo) / (side / 1024)) per axis, clamped to 0..1023 (10
    levels).  A cell is split into its eight children while it holds more
    than `cap` surface points; every leaf with points is a core, and a core
    holds the three centres of each of its points (rows i, N + i, 2N + i).
    A finest-level leaf with more than `cap` points (coincident points) is
    cut into runs of `cap` points by increasing index.
  * Overlap.  Omega_i adds the k = ceil(pct |core_i| / 100) centres outside
    core_i nearest to it: the distance of a centre to a core is its smallest
    squared distance (dx*dx + dy*dy) + dz*dz to a core centre, ties by index.
  * Local matrix.  The Gaussian of Omega_i without truncation plus shift * I
    (the truncated restriction is indefinite for the configurations of the
    paper, and the shift is what keeps the local inverses bounded).
  * cap follows from the largest block: the largest p with
    3p + ceil(3p pct / 100) <= max_block.
  * Small leaves merged (min_block > 0).  The leaves are taken in the
    octree's depth-first order (children by the digit bx + 2 by + 4 bz of
    their cell, the runs of a finest cell by index) and consecutive leaves
    are joined into one core: the core being built is closed before the next
    leaf when its block (3p centres plus their overlap) already reaches
    min_block or when the next leaf would take it above cap points.  The
    domain split then follows the density along the curve, as the paper's
    subdomains of uneven size, without tiny blocks.
"""
from __future__ import annotations


import numpy as np

__all__ = ["overlap_count", "core_cap", "block_size", "octree_cores", "merge_leaves", "core_centres", "overlap",
           "subdomains", "local_matrix", "schwarz_apply", "schwarz_matrix"]


def _phi(r2, sigma):
    return np.exp(-r2 / (2.0 * sigma * sigma))


def _sqdist(a, b):
    d = a[:, None, :] - b[None, :, :]
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]


def overlap_count(ncore: int, pct: int) -> int:
    """k = ceil(pct * ncore / 100) in integers."""
    return (ncore * pct + 99) // 100


def core_cap(max_block: int, pct: int) -> int:
    """Surface points per core: the largest p with 3p + ceil(3p pct/100) <= max_block."""
    p = max_block // 3
    while p > 1 and 3 * p + overlap_count(3 * p, pct) > max_block:
        p -= 1
    return max(p, 1)


def block_size(points: int, pct: int) -> int:
    """Centres of a subdomain whose core holds `points` surface points."""
    return 3 * points + overlap_count(3 * points, pct)


def octree_cores(P: np.ndarray, cap: int) -> list[np.ndarray]:
    """Leaves of the octree over the surface points P (N x 3), each as the
    sorted array of its point indices."""
    P = np.asarray(P, dtype=np.float64)
    lo = P.min(axis=0)
    side = float((P.max(axis=0) - lo).max())
    if not side > 0.0:
        side = 1.0
    fine = side / 1024.0
    q = np.floor((P - lo) / fine)
    q = np.clip(q, 0, 1023).astype(np.int64)
    leaves: list[np.ndarray] = []

    def visit(idx: np.ndarray, level: int):
        if idx.size <= cap or level == 10:
            idx = np.sort(idx)
            for a in range(0, idx.size, cap):
                leaves.append(idx[a:a + cap])
            return
        bit = 9 - level                     # the children split on this bit of q
        child = ((q[idx, 0] >> bit) & 1) + 2 * ((q[idx, 1] >> bit) & 1) + 4 * ((q[idx, 2] >> bit) & 1)
        for c in range(8):
            sub = idx[child == c]
            if sub.size:
                visit(sub, level + 1)

    visit(np.arange(P.shape[0]), 0)
    return leaves


def merge_leaves(leaves: list[np.ndarray], cap: int, min_block: int, pct: int) -> list[np.ndarray]:
    """Consecutive leaves (in the order octree_cores returns them) joined
    into cores of at least min_block centres with their overlap where the
    cap allows; min_block <= 0 keeps every leaf."""
    if min_block <= 0:
        return list(leaves)
    out: list[np.ndarray] = []
    cur: list[np.ndarray] = []
    npts = 0
    for leaf in leaves:
        if cur and (block_size(npts, pct) >= min_block or npts + leaf.size > cap):
            out.append(np.sort(np.concatenate(cur)))
            cur, npts = [], 0
        cur.append(leaf)
        npts += leaf.size
    if cur:
        out.append(np.sort(np.concatenate(cur)))
    return out


def core_centres(points: np.ndarray, n: int) -> np.ndarray:
    """The three centres of each surface point of a core (rows i, N+i, 2N+i)."""
    points = np.asarray(points, dtype=np.int64)
    return np.concatenate([points, points + n, points + 2 * n])


def overlap(X: np.ndarray, core: np.ndarray, k: int) -> np.ndarray:
    """The k centres outside `core` nearest to it (squared distance to the
    nearest core centre; ties by index), nearest first."""
    X = np.asarray(X, dtype=np.float64)
    outside = np.setdiff1d(np.arange(X.shape[0]), core)
    if k <= 0 or outside.size == 0:
        return np.zeros(0, dtype=np.int64)
    d = _sqdist(X[outside], X[core]).min(axis=1)
    order = np.lexsort((outside, d))
    return outside[order[:k]]


def subdomains(points: np.ndarray, X: np.ndarray, max_block: int = 192, pct: int = 10, min_block: int = 0):
    """[(core centres, overlap centres)] for the surface points `points`
    (N x 3) and the centres X (3N x 3, paper order)."""
    n = np.asarray(points).shape[0]
    cap = core_cap(max_block, pct)
    out = []
    for leaf in merge_leaves(octree_cores(points, cap), cap, min_block, pct):
        core = core_centres(leaf, n)
        out.append((core, overlap(X, core, overlap_count(core.size, pct))))
    return out


def local_matrix(X: np.ndarray, members: np.ndarray, sigma: float, shift: float) -> np.ndarray:
    """Untruncated Gaussian on the members plus shift * I."""
    Y = np.asarray(X, dtype=np.float64)[members]
    return _phi(_sqdist(Y, Y), sigma) + shift * np.eye(members.size)


def schwarz_apply(X, subs, sigma: float, shift: float, r: np.ndarray, restricted: bool = False) -> np.ndarray:
    """z = sum_i R_i^T A_i^{-1} R_i r (additive), or with only the core rows of
    every local solution (restricted).  Local systems by LAPACK gesv."""
    r = np.asarray(r, dtype=np.float64)
    z = np.zeros_like(r)
    for core, ov in subs:
        mem = np.concatenate([core, ov])
        y = np.linalg.solve(local_matrix(X, mem, sigma, shift), r[mem])
        if restricted:
            z[core] += y[:core.size]
        else:
            np.add.at(z, mem, y)
    return z


def schwarz_matrix(X, subs, sigma: float, shift: float, restricted: bool = False) -> np.ndarray:
    """The preconditioner as a dense matrix (small inputs only)."""
    m = np.asarray(X).shape[0]
    M = np.zeros((m, m))
    for core, ov in subs:
        mem = np.concatenate([core, ov])
        inv = np.linalg.inv(local_matrix(X, mem, sigma, shift))
        rows = core.size if restricted else mem.size
        for a in range(rows):
            M[mem[a], mem] += inv[a]
    return M
