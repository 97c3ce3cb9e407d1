"""Pins of the Schwarz preconditioner oracle (CPU only).

Each check is tied to something other than the oracle's own code: the
definition of an octree leaf restated as counts over all points, the overlap
as an order property checked with plain loops, closed forms of tiny local
matrices, the exact inverse that a single subdomain or block-diagonal
clusters must give, the symmetry of the additive form, and GMRES converging
in one step with the exact inverse as its preconditioner."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import schwarz as S

SIGMA = 0.05


def test_core_cap_values():
    assert S.core_cap(192, 10) == 58      # 174 + 18 = 192; 59 points would need 195
    assert S.core_cap(192, 0) == 64
    assert S.core_cap(30, 50) == 6        # 18 + 9 = 27; 7 points would need 32
    assert S.overlap_count(174, 10) == 18
    assert S.overlap_count(30, 10) == 3   # exact integers: no 3.0000000000000004 surprise
    assert S.overlap_count(0, 10) == 0


def _cloud(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(n // 2, 3)) * 0.05 + np.array([0.3, 0.1, -0.2])
    b = rng.uniform(-1, 1, size=(n - n // 2 - 6, 3))
    dup = np.repeat(a[:1], 6, axis=0)    # coincident points: a finest cell above the cap
    P = np.concatenate([a, b, dup])
    # a neighbour of the coincident points in the adjacent finest cell that
    # shares their cell on the next coarser level
    lo = P.min(0)
    fine = (P.max(0) - lo).max() / 1024
    q = np.floor((a[0] - lo) / fine)
    nb = a[0].copy()
    nb[0] = lo[0] + (float(int(q[0]) ^ 1) + 0.5) * fine
    return np.concatenate([P, nb[None, :]])


@pytest.mark.parametrize("cap", [5, 20])
def test_octree_leaves_match_the_definition(cap):
    """A leaf is a cell with at most `cap` points whose parent holds more
    (the root when it holds at most `cap`), or a run of a finest cell."""
    P = _cloud(400, 3)
    leaves = S.octree_cores(P, cap)
    allpts = np.sort(np.concatenate(leaves))
    assert np.array_equal(allpts, np.arange(len(P)))               # a partition
    lo = P.min(0)
    side = (P.max(0) - lo).max()
    q = np.clip(np.floor((P - lo) / (side / 1024)), 0, 1023).astype(np.int64)
    for leaf in leaves:
        assert 1 <= leaf.size <= cap
        first = leaf[0]
        # the leaf's level: the first level whose cell (of the first point) holds <= cap points
        for level in range(11):
            sh = 10 - level
            cell = [i for i in range(len(P)) if all((q[i, d] >> sh) == (q[first, d] >> sh) for d in range(3))]
            if len(cell) <= cap or level == 10:
                break
        assert all(i in cell for i in leaf)
        if len(cell) <= cap:
            assert sorted(cell) == sorted(leaf.tolist())           # the whole cell
            if level > 0:                                           # and its parent held more
                sh = 11 - level
                parent = [i for i in range(len(P))
                          if all((q[i, d] >> sh) == (q[first, d] >> sh) for d in range(3))]
                assert len(parent) > cap
        else:
            # finest cell above the cap: runs of `cap` points in index order
            runs = [sorted(cell)[a:a + cap] for a in range(0, len(cell), cap)]
            assert sorted(leaf.tolist()) in runs


def _morton_full_depth(qcell, level):
    """The depth-first position of a cell at `level`: its coordinates' bits
    interleaved (x lowest), padded to the finest level."""
    key = 0
    for b in range(level):
        bit = level - 1 - b
        digit = ((qcell[0] >> bit) & 1) + 2 * ((qcell[1] >> bit) & 1) + 4 * ((qcell[2] >> bit) & 1)
        key = key * 8 + digit
    return key << (3 * (10 - level))


@pytest.mark.parametrize("cap", [5, 20])
def test_leaves_come_in_depth_first_order(cap):
    """octree_cores returns its leaves in increasing Morton order of their
    cells (x the lowest bit), the runs of one finest cell by index: the
    order in which leaves are merged."""
    P = _cloud(400, 3)
    leaves = S.octree_cores(P, cap)
    lo = P.min(0)
    side = (P.max(0) - lo).max()
    q = np.clip(np.floor((P - lo) / (side / 1024)), 0, 1023).astype(np.int64)
    keys = []
    for leaf in leaves:
        # the leaf's level: the coarsest cell of its first point holding only leaf points
        first = leaf[0]
        for level in range(11):
            sh = 10 - level
            cell = [i for i in range(len(P)) if all((q[i, d] >> sh) == (q[first, d] >> sh) for d in range(3))]
            if set(cell) <= set(leaf.tolist()) or level == 10:
                break
        keys.append((_morton_full_depth(q[first] >> (10 - level), level), int(leaf[0])))
    assert keys == sorted(keys)


def _merge_by_definition(leaves, cap, min_block, pct):
    """Greedy runs of consecutive leaves, restated: a run grows while its
    block is below min_block and the next leaf fits under the cap."""
    runs, i = [], 0
    while i < len(leaves):
        j = i + 1
        pts = leaves[i].size
        while j < len(leaves) and 3 * pts + -(-(3 * pts * pct) // 100) < min_block and pts + leaves[j].size <= cap:
            pts += leaves[j].size
            j += 1
        runs.append((i, j))
        i = j
    return runs


@pytest.mark.parametrize("cap,min_block,pct", [(20, 64, 10), (20, 30, 0), (5, 200, 10), (50, 16, 25)])
def test_merged_cores_are_greedy_runs_of_leaves(cap, min_block, pct):
    P = _cloud(400, 3)
    leaves = S.octree_cores(P, cap)
    merged = S.merge_leaves(leaves, cap, min_block, pct)
    runs = _merge_by_definition(leaves, cap, min_block, pct)
    assert len(merged) == len(runs)
    for core, (i, j) in zip(merged, runs):
        assert np.array_equal(core, np.sort(np.concatenate(leaves[i:j])))
        assert core.size <= cap
    assert np.array_equal(np.sort(np.concatenate(merged)), np.arange(len(P)))
    # fewer, larger cores than leaves whenever small leaves exist
    small = [l for l in leaves if S.block_size(l.size, pct) < min_block]
    if len(small) > 1:
        assert len(merged) < len(leaves)


def test_merge_off_keeps_the_leaves():
    P = _cloud(400, 3)
    leaves = S.octree_cores(P, 20)
    merged = S.merge_leaves(leaves, 20, 0, 10)
    assert len(merged) == len(leaves) and all(np.array_equal(a, b) for a, b in zip(merged, leaves))
    X, _ = O.extended_centres(P, P, 0.01)
    subs = S.subdomains(P, X, max_block=66, pct=10)
    assert len(subs) == len(leaves)


def test_overlap_is_the_k_nearest():
    rng = np.random.default_rng(5)
    X = rng.uniform(size=(90, 3))
    X[41] = X[40]                       # a tie in distance, broken by index
    core = np.array([0, 1, 2, 3, 4, 5, 6])

    def dist(j):
        best = math.inf
        for c in core:
            dx, dy, dz = X[j, 0] - X[c, 0], X[j, 1] - X[c, 1], X[j, 2] - X[c, 2]
            best = min(best, (dx * dx + dy * dy) + dz * dz)
        return best

    # k ends between the two tied centres: only the lower index is taken
    ranked = sorted((dist(j), j) for j in range(len(X)) if j not in core)
    k = [j for _, j in ranked].index(40) + 1
    ov = S.overlap(X, core, k)
    assert ov.size == k and not set(ov) & set(core)
    assert 40 in ov and 41 not in ov
    chosen = [(dist(j), j) for j in ov]
    rest = [(dist(j), j) for j in range(len(X)) if j not in core and j not in ov]
    assert max(chosen) < min(rest)
    assert chosen == sorted(chosen)     # nearest first


def test_local_matrix_two_points():
    X = np.array([[0.0, 0.0, 0.0], [0.03, 0.04, 0.0]])
    A = S.local_matrix(X, np.array([0, 1]), SIGMA, 0.25)
    e = math.exp(-0.0025 / (2 * SIGMA * SIGMA))
    assert np.allclose(A, [[1.25, e], [e, 1.25]], rtol=0, atol=1e-15)


def _sphere(n, seed):
    rng = np.random.default_rng(seed)
    g = rng.normal(size=(n, 3))
    p = g / np.linalg.norm(g, axis=1)[:, None]
    return p, p.copy()


def test_single_subdomain_is_the_shifted_inverse():
    P, N = _sphere(30, 1)
    X, _ = O.extended_centres(P, N, 0.02)
    subs = S.subdomains(P, X, max_block=200, pct=0)
    assert len(subs) == 1 and subs[0][0].size == 90
    shift = 0.1
    r = np.random.default_rng(2).uniform(-1, 1, 90)
    z = S.schwarz_apply(X, subs, 0.3, shift, r)
    A = O.interpolation_matrix(X, 0.3) + shift * np.eye(90)
    assert np.linalg.norm(A @ z - r) <= 1e-10 * np.linalg.norm(r)


def test_restricted_is_exact_on_separated_clusters():
    """Clusters 40 sigma apart: the Gaussian between them underflows to 0, the
    matrix is block diagonal and every core is one cluster, so the restricted
    form with overlap is the exact inverse."""
    rng = np.random.default_rng(7)
    corners = np.array([[0, 0, 0], [1, 1, 0], [0, 1, 1], [1, 0, 1]], dtype=float) * 80 * SIGMA
    P = np.concatenate([c + rng.uniform(-SIGMA, SIGMA, size=(12, 3)) for c in corners])
    Nrm = rng.normal(size=P.shape)
    X, _ = O.extended_centres(P, Nrm, 0.2 * SIGMA)
    assert S.core_cap(44, 20) == 12                     # 36 + 8 = 44: one cluster per core
    subs = S.subdomains(P, X, max_block=44, pct=20)
    assert len(subs) == 4 and all(c.size == 36 for c, _ in subs)
    assert all(o.size == 8 for _, o in subs)
    shift = 0.05
    A = O.interpolation_matrix(X, SIGMA) + shift * np.eye(len(X))
    x = rng.uniform(-1, 1, len(X))
    z = S.schwarz_apply(X, subs, SIGMA, shift, A @ x, restricted=True)
    assert np.allclose(z, x, rtol=0, atol=1e-9 * np.abs(x).max())
    # the additive form adds the overlap rows' partial solutions: not exact
    z_add = S.schwarz_apply(X, subs, SIGMA, shift, A @ x, restricted=False)
    assert np.abs(z_add - x).max() > 1e-3


def test_additive_form_is_symmetric():
    P, N = _sphere(40, 4)
    X, _ = O.extended_centres(P, N, 0.02)
    subs = S.subdomains(P, X, max_block=30, pct=30)
    assert len(subs) > 3
    M = S.schwarz_matrix(X, subs, 0.3, 0.1)
    assert np.abs(M - M.T).max() <= 1e-9 * np.abs(M).max()
    r = np.random.default_rng(3).uniform(-1, 1, len(X))
    assert np.allclose(M @ r, S.schwarz_apply(X, subs, 0.3, 0.1, r), rtol=1e-9, atol=1e-12)
    Mr = S.schwarz_matrix(X, subs, 0.3, 0.1, restricted=True)
    assert np.allclose(Mr @ r, S.schwarz_apply(X, subs, 0.3, 0.1, r, restricted=True), rtol=1e-9, atol=1e-12)


def test_preconditioned_gmres_with_the_exact_inverse_takes_one_step():
    P, N = _sphere(20, 6)
    X, _ = O.extended_centres(P, N, 0.05)
    A = O.interpolation_matrix(X, 0.4)
    Ainv = np.linalg.inv(A)
    b = np.random.default_rng(1).uniform(-1, 1, len(X))
    res = O.gmres(lambda v: A @ v, b, restart=10, tol=1e-10, apply_M=lambda v: Ainv @ v)
    assert res.converged and res.iters == 1
    assert np.linalg.norm(A @ res.x - b) <= 1e-9 * np.linalg.norm(b)
    plain = O.gmres(lambda v: A @ v, b, restart=10, tol=1e-6, max_iters=40)
    ident = O.gmres(lambda v: A @ v, b, restart=10, tol=1e-6, max_iters=40, apply_M=lambda v: v)
    assert np.array_equal(plain.x, ident.x)
