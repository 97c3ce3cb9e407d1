"""GPU parity at the full sizes of the scan-like metaball workload (2,000,000
points, 6,000,000 centres, sigma 0.01, cutoff 4 sigma, 512^3 grid) and of the
torus workload with solved weights: sampled operator rows and grid nodes,
computed one by one by the C cell-list oracle (pinned in
test_oracle_cells.py), and the operator's exact nonzero count.

Tolerances as in test_gpu_parity.py: float64 |d| <= 1e-13 sum_j |A_ij x_j|;
float32 |d| <= 64 u32 max(1, (r_c / 4 sigma)^2) sum_j |A_ij x_j| (derived in
the design notes), with a tighter tripwire at 16 u32 (the largest ratio
observed on any parity case is below 6 u32), so that a several-fold loss of
accuracy fails even inside the derived bound."""
import math
import sys

import numpy as np
import pytest

from oracle import rbf_oracle as o
from oracle.cells import CellOracle, max_threads
from paper_1305_5179_amd import workloads as w

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
TOL64 = 1e-13
TRIPWIRE32 = 16 * U32


def tol32(sigma, cutoff):
    return 64 * U32 * max(1.0, (cutoff / (4 * sigma)) ** 2)


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


def dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def band_node_indices(g, points, cutoff, k, rng):
    """k grid nodes near the cloud, chosen from the inputs alone: the node
    nearest to a cloud point moved by a uniform offset in the cutoff ball."""
    P = w.band_samples(points, cutoff, k, seed=int(rng.integers(1 << 30)))
    ijk = np.rint((P - np.asarray(g.origin)) / np.asarray(g.h)).astype(np.int64)
    ijk = np.clip(ijk, 0, np.asarray(g.dims) - 1)
    return ijk[:, 0] + g.dims[0] * (ijk[:, 1] + g.dims[1] * ijk[:, 2])


@pytest.fixture(scope="module")
def metaballs_full(torch, R):
    cfg = w.METABALLS_2M
    _say("[metaballs 2M] generating the cloud")
    c = w.metaballs(cfg["n"], cfg["seed"])
    X, _ = o.extended_centres(c.points, c.normals, cfg["eps"])
    _say("[metaballs 2M] setup")
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), cfg["eps"], cfg["sigma"], cfg["cutoff"])
    L = CellOracle(X, cfg["cutoff"])
    yield dict(c=c, X=X, ctx=ctx, L=L, cfg=cfg)
    ctx.close()
    L.close()


def test_metaballs_full_pair_count_is_exact(metaballs_full):
    """The lists hold every pair inside the cutoff exactly once: useful pairs
    = nnz(A), counted by the oracle over all 6M rows."""
    t = metaballs_full
    st = t["ctx"].stats()
    nnz = t["L"].count(threads=max_threads())
    _say(f"[metaballs 2M pairs] device {st.useful_pairs}  oracle {nnz}  examined/useful "
         f"{st.examined_pairs / st.useful_pairs:.3f}")
    assert st.n_centres == 6_000_000
    assert st.useful_pairs == nnz


@pytest.mark.parametrize("prec", [0, 1])
def test_metaballs_full_operator_sampled_rows(metaballs_full, torch, prec):
    t = metaballs_full
    X, cfg, L = t["X"], t["cfg"], t["L"]
    x = w.random_vector(X.shape[0], seed=4)
    y = host(t["ctx"].matvec(dev(torch, x), prec=prec))
    rows = np.random.default_rng(51).choice(X.shape[0], 400, replace=False)
    ref = L.matvec_rows(x, cfg["sigma"], rows=rows, threads=max_threads())
    scale = L.matvec_rows(np.abs(x), cfg["sigma"], rows=rows, threads=max_threads())
    ratio = np.max(np.abs(y[rows] - ref) / scale)
    _say(f"[metaballs 2M operator prec={prec}] max ratio {ratio / U32:.2f} u32")
    assert ratio <= (tol32(cfg["sigma"], cfg["cutoff"]) if prec == 0 else TOL64)
    if prec == 0:
        assert ratio <= TRIPWIRE32


def test_metaballs_full_grid_sampled_nodes(metaballs_full, torch, R):
    """The 512^3 grid (134M nodes) in float32: sampled band nodes and random
    nodes against the oracle; nodes with no centre within the cutoff are 0."""
    t = metaballs_full
    X, cfg, L = t["X"], t["cfg"], t["L"]
    g = w.Grid.around(t["c"].points, cfg["grid_n"])
    coef = np.random.default_rng(52).uniform(-1, 1, X.shape[0])
    out = t["ctx"].eval_grid(dev(torch, coef), g.origin, g.h, g.dims, prec=R.RBF_FP32)
    rng = np.random.default_rng(53)
    idx = np.concatenate([band_node_indices(g, t["c"].points, cfg["cutoff"], 400, rng),
                          rng.choice(g.size, 100, replace=False)])
    got = host(out[dev(torch, idx).long()])
    del out
    nodes = o.grid_nodes(g.origin, g.h, g.dims, idx)
    ref = L.evaluate(coef, nodes, cfg["sigma"], threads=max_threads())
    scale = L.evaluate(np.abs(coef), nodes, cfg["sigma"], threads=max_threads())
    err = np.abs(got - ref)
    ratio = np.max(err[scale > 0] / scale[scale > 0])
    _say(f"[metaballs 2M grid] nodes with a centre in reach {np.sum(scale > 0)} of {idx.size}, "
         f"max ratio {ratio / U32:.2f} u32")
    assert np.sum(scale > 0) >= 350
    assert np.all(err <= tol32(cfg["sigma"], cfg["cutoff"]) * scale + U32 * np.abs(ref) + 1e-300)
    assert np.all(got[scale == 0] == 0)
    assert ratio <= TRIPWIRE32


def test_torus_grid_with_solved_weights(torch, R):
    """The 256^3 torus grid with the chosen pipeline's weights (three
    refinement steps): per node |d| within the derived float32 bound, and the
    share of sampled nodes meeting the 1e-6 absolute gate reported (the
    float32 evaluation of terms summing to sum_j |c_j phi_j| ~ 1e2 cannot
    meet 1e-6 everywhere)."""
    cfg = w.TORUS_200K
    c = w.torus(cfg["n"], cfg["seed"])
    X, _ = o.extended_centres(c.points, c.normals, cfg["eps"])
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), cfg["eps"], cfg["sigma"], cfg["cutoff"])
    try:
        coef, info = ctx.solve(tol=1e-8, restart=30, max_iters=90, max_outer=3)
        g = w.Grid.around(c.points, cfg["grid_n"])
        out = ctx.eval_grid(coef, g.origin, g.h, g.dims, prec=R.RBF_FP32)
        rng = np.random.default_rng(61)
        idx = np.concatenate([band_node_indices(g, c.points, cfg["cutoff"], 400, rng),
                              rng.choice(g.size, 100, replace=False)])
        got = host(out[dev(torch, idx).long()])
        cw = host(coef)
    finally:
        ctx.close()
    L = CellOracle(X, cfg["cutoff"])
    nodes = o.grid_nodes(g.origin, g.h, g.dims, idx)
    ref = L.evaluate(cw, nodes, cfg["sigma"], threads=max_threads())
    scale = L.evaluate(np.abs(cw), nodes, cfg["sigma"], threads=max_threads())
    L.close()
    err = np.abs(got - ref)
    inside = scale > 0
    share = np.mean(err[inside] <= 1e-6)
    ratio = np.max(err[inside] / scale[inside])
    _say(f"[torus grid, solved weights] resid {info.rel_resid:.2e}; nodes in reach {inside.sum()}; "
         f"max |d| {err.max():.2e}; median sum|c phi| {np.median(scale[inside]):.3g}; "
         f"share within 1e-6 {share:.3f}; max ratio {ratio / U32:.2f} u32")
    assert np.all(err <= tol32(cfg["sigma"], cfg["cutoff"]) * scale + U32 * np.abs(ref) + 1e-300)
    assert np.all(got[~inside] == 0)
    assert ratio <= TRIPWIRE32
