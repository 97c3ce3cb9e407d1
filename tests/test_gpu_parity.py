"""GPU parity: the HIP path, called through the C ABI, against the CPU
oracle on the same seeded inputs.

Tolerances (derived in the design notes):
  * centres: exact float64 equality (same operations, no contraction);
  * float64 operator / evaluation: |d| <= 1e-13 * sum_j |A_ij x_j|;
  * float32 operator / evaluation: |d| <= 64 u sum_j |A_ij x_j| (u = 2^-24),
    plus exact truncation decisions, checked separately at the cutoff;
  * solve: relative weight error <= 1e-5 on well-conditioned systems.
"""
import math
import sys

import numpy as np
import pytest

from oracle import rbf_oracle as o
from paper_1305_5179_amd import workloads as w

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
TOL64 = 1e-13
TOL32 = 64 * U32


def tol32(sigma, cutoff):
    """float32 tolerance relative to sum_j |A_ij x_j|.  A term's relative
    error grows with its scaled squared distance d = k r^2 (the exponent's
    absolute error is a few u d), so with a cutoff the bound scales with
    T = k r_c^2: 64 u up to r_c = 4 sigma, in proportion beyond."""
    if not math.isfinite(cutoff):
        return TOL32
    return TOL32 * max(1.0, (cutoff / (4 * sigma)) ** 2)


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


def abs_sums(X, x, rows, sigma, cutoff, targets=None):
    """sum_j |A_ij x_j| for the given rows (targets default to centres)."""
    T = X if targets is None else targets
    out = np.empty(len(rows))
    for t, i in enumerate(rows):
        r2 = o.sqdist(T[i:i + 1], X)[0]
        k = o.phi(r2, sigma)
        if math.isfinite(cutoff):
            k = np.where(r2 <= cutoff * cutoff, k, 0.0)
        out[t] = np.dot(k, np.abs(x))
    return out


CASES = {
    # name: (cloud factory, eps, sigma, cutoff)
    "one_point": (lambda: w.Cloud(np.array([[0.1, 0.2, 0.3]]), np.array([[0.0, 0.0, 2.0]]), "one"), 0.05, 0.1, math.inf),
    "five_points_cut": (lambda: w.sphere(5, seed=9), 0.1, 0.3, 0.9),
    "lattice_dense": (lambda: w.lattice_cloud(6, 6, 0.1, jitter=0.2), 0.05, 0.04, math.inf),
    "sphere333_dense": (lambda: w.sphere(333, seed=7), 0.02, 0.2, math.inf),
    "sphere333_cut": (lambda: w.sphere(333, seed=7), 0.02, 0.15, 0.45),
    "torus_patch_cut": (lambda: w.patch(w.torus(), 1701, seed=3), 0.005, 0.02, 0.08),
    # cutoff 12 sigma: too wide for the expanded form, so every group takes
    # the direct differences with the lane masks
    "sphere333_wide": (lambda: w.sphere(333, seed=7), 0.02, 0.05, 0.6),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request, torch, R):
    name = request.param
    make, eps, sigma, cutoff = CASES[name]
    c = make()
    _say(f"[case {name}] n={c.n} eps={eps} sigma={sigma} cutoff={cutoff}")
    X, b = o.extended_centres(c.points, c.normals, eps)
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), eps, sigma, cutoff)
    yield dict(name=name, cloud=c, eps=eps, sigma=sigma, cutoff=cutoff, X=X, b=b, ctx=ctx)
    ctx.close()


def test_centres_equal_oracle(case, torch):
    Xg, bg = case["ctx"].centres()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(Xg), case["X"])
    np.testing.assert_array_equal(host(bg), case["b"])


def test_pair_count_equals_oracle_nonzeros(case):
    """The lists hold every pair inside the cutoff exactly once."""
    st = case["ctx"].stats()
    A = o.interpolation_matrix(case["X"], case["sigma"], case["cutoff"])
    assert st.useful_pairs == np.count_nonzero(A)
    assert st.examined_pairs >= st.useful_pairs


@pytest.mark.parametrize("prec", [0, 1])
def test_operator_matches_oracle(case, torch, R, prec):
    X, sigma, cutoff = case["X"], case["sigma"], case["cutoff"]
    x = w.random_vector(X.shape[0], seed=4)
    y = host(case["ctx"].matvec(dev(torch, x), prec=prec))
    ref = o.matvec(X, x, sigma, cutoff)
    scale = abs_sums(X, x, range(X.shape[0]), sigma, cutoff)
    tol = tol32(sigma, cutoff) if prec == 0 else TOL64
    ratio = np.max(np.abs(y - ref) / scale)
    _say(f"[{case['name']} prec={prec}] max |dy| / sum|Ax| = {ratio:.3e} (u32 units {ratio / U32:.2f})")
    assert ratio <= tol


@pytest.mark.parametrize("prec", [0, 1])
def test_point_evaluation_matches_oracle(case, torch, R, prec):
    X, sigma, cutoff = case["X"], case["sigma"], case["cutoff"]
    rng = np.random.default_rng(21)
    coef = rng.uniform(-2, 2, X.shape[0])
    lo, hi = X.min(0) - 3 * sigma, X.max(0) + 3 * sigma
    pts = rng.uniform(lo, hi, size=(97, 3))
    pts = np.concatenate([pts, X[:5] + 1e-3, [[1e3, 1e3, 1e3]]])   # near centres, and far away
    f = host(case["ctx"].eval_points(dev(torch, coef), dev(torch, pts), prec=prec))
    ref = o.evaluate(X, coef, pts, sigma, cutoff)
    scale = abs_sums(X, coef, range(pts.shape[0]), sigma, cutoff, targets=pts)
    tol = tol32(sigma, cutoff) if prec == 0 else TOL64
    np.testing.assert_array_less(np.abs(f - ref), tol * scale + 1e-300)
    assert f[-1] == 0.0 or not math.isfinite(cutoff)


@pytest.mark.parametrize("prec", [0, 1])
def test_grid_evaluation_matches_oracle(case, torch, R, prec):
    X, sigma, cutoff = case["X"], case["sigma"], case["cutoff"]
    rng = np.random.default_rng(22)
    coef = rng.uniform(-2, 2, X.shape[0])
    g = w.Grid.around(X, 9)
    g = w.Grid(g.origin, g.h, (9, 7, 11))   # ragged 4x2x2 bricks on every axis
    out = host(case["ctx"].eval_grid(dev(torch, coef), g.origin, g.h, g.dims, prec=prec))
    nodes = o.grid_nodes(g.origin, g.h, g.dims)
    ref = o.evaluate(X, coef, nodes, sigma, cutoff)
    scale = abs_sums(X, coef, range(nodes.shape[0]), sigma, cutoff, targets=nodes)
    tol = tol32(sigma, cutoff) if prec == 0 else TOL64
    err = np.abs(out - ref)
    # float32 output: add its own rounding
    bound = tol * scale + (U32 * np.abs(ref) if prec == 0 else 0) + 1e-300
    assert np.all(err <= bound), float(np.max(err / bound))
    if math.isfinite(cutoff):
        assert np.all(out[scale == 0] == 0.0)


def _brick_form(sigma, cutoff, h):
    """Whether a float32 grid takes the list-free brick sums: the library's
    range condition on the product form's exponents (scaled units)."""
    sk = math.sqrt(math.log2(math.e) / (2 * sigma * sigma))
    diag = math.sqrt((3 * h[0]) ** 2 + h[1] ** 2 + h[2] ** 2)
    umax = sk * (cutoff + diag) * (1 + 1e-6)
    return umax * umax + 2 * umax * sk * (3 * h[0] + h[1] + h[2]) <= 64


@pytest.mark.parametrize("name", ["torus_patch_cut", "sphere333_cut"])
def test_grid_brick_sums_match_oracle(name, torch, R):
    """Float32 grids fine enough for the list-free brick sums: every node
    against the oracle, bricks ragged on every axis, nodes without a centre
    within the cutoff exactly zero, and the same values on a second call."""
    make, eps, sigma, cutoff = CASES[name]
    c = make()
    X, _ = o.extended_centres(c.points, c.normals, eps)
    h = (0.5 * sigma, 0.45 * sigma, 0.55 * sigma)
    assert _brick_form(sigma, cutoff, h)
    lo = X.min(axis=0) - 0.6 * cutoff
    span = X.max(axis=0) + 0.6 * cutoff - lo
    dims = [int(math.ceil(span[d] / h[d])) + 1 for d in range(3)]
    dims = [d + (1 - d % 4) % 4 if i == 0 else d + (1 - d % 2) for i, d in enumerate(dims)]   # ragged bricks
    g = w.Grid(tuple(float(v) for v in lo), h, tuple(dims))
    _say(f"[brick grid {name}] dims {dims}")
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), eps, sigma, cutoff)
    try:
        coef = np.random.default_rng(23).uniform(-2, 2, X.shape[0])
        out = host(ctx.eval_grid(dev(torch, coef), g.origin, g.h, g.dims, prec=0))
        again = host(ctx.eval_grid(dev(torch, coef), g.origin, g.h, g.dims, prec=0))
    finally:
        ctx.close()
    nodes = o.grid_nodes(g.origin, g.h, g.dims)
    ref = o.evaluate(X, coef, nodes, sigma, cutoff)
    scale = abs_sums(X, coef, range(nodes.shape[0]), sigma, cutoff, targets=nodes)
    err = np.abs(out - ref)
    bound = tol32(sigma, cutoff) * scale + U32 * np.abs(ref) + 1e-300
    band = scale > 0
    _say(f"[brick grid {name}] band nodes {band.sum()} of {g.size}, max err/bound {np.max(err / bound):.3f}, "
         f"max err {np.max(err[band] / scale[band]) / U32:.2f} u32 of sum |terms|")
    assert band.sum() > 1000 and (~band).sum() > 1000
    assert np.all(err <= bound)
    assert np.all(out[~band] == 0.0)
    assert np.array_equal(out, again)


def test_grid_brick_sums_edge_cases(torch, R):
    """List-free brick sums on degenerate grids: a zero spacing on one axis
    (every node of a row at the same place), a single node, and a grid out
    of reach of every centre (all exact zeros)."""
    make, eps, sigma, cutoff = CASES["torus_patch_cut"]
    c = make()
    X, _ = o.extended_centres(c.points, c.normals, eps)
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), eps, sigma, cutoff)
    try:
        coef = np.random.default_rng(24).uniform(-2, 2, X.shape[0])
        cen = X.mean(axis=0)
        grids = [
            w.Grid(tuple(float(v) for v in cen - 0.05), (0.5 * sigma, 0.0, 0.5 * sigma), (21, 5, 19)),
            w.Grid(tuple(float(v) for v in X[7]), (0.5 * sigma,) * 3, (1, 1, 1)),
            w.Grid(tuple(float(v) for v in X.max(axis=0) + 2 * cutoff), (0.5 * sigma,) * 3, (9, 7, 5)),
        ]
        for g in grids:
            assert _brick_form(sigma, cutoff, g.h)
            out = host(ctx.eval_grid(dev(torch, coef), g.origin, g.h, g.dims, prec=0))
            nodes = o.grid_nodes(g.origin, g.h, g.dims)
            ref = o.evaluate(X, coef, nodes, sigma, cutoff)
            scale = abs_sums(X, coef, range(nodes.shape[0]), sigma, cutoff, targets=nodes)
            bound = tol32(sigma, cutoff) * scale + U32 * np.abs(ref) + 1e-300
            _say(f"[brick edge] dims {g.dims} h {g.h}: band {int((scale > 0).sum())}, "
                 f"max err/bound {np.max(np.abs(out - ref) / bound):.3f}")
            assert np.all(np.abs(out - ref) <= bound)
            assert np.all(out[scale == 0] == 0.0)
        assert np.count_nonzero(out) == 0   # the last grid is out of reach
    finally:
        ctx.close()


def test_cutoff_decision_is_the_float64_one(torch, R):
    """Pairs within a few ulps of the cutoff: the float32 kernel must take the
    float64 decision (inclusive) on both sides of it."""
    rc = 0.08
    sigma = 0.02
    base = np.array([0.0, 0.0, 0.0])
    # centre 0 and centre 1 exactly rc apart along x (r^2 == rc^2 in float64
    # for these values); centre 2 one ulp beyond along y.
    pts = np.array([base, base + [rc, 0, 0], base + [0, np.nextafter(rc, 1.0), 0], base + [0, 0, 0.5]])
    nrm = np.tile([0.0, 0.0, 1.0], (4, 1))
    eps = 0.3   # off-surface points far from everything else
    X, _ = o.extended_centres(pts, nrm, eps)
    ctx = R.Rbf(dev(torch, pts), dev(torch, nrm), eps, sigma, rc)
    x = np.zeros(X.shape[0])
    x[1] = 1.0
    x[2] = 10.0
    for prec in (0, 1):
        y = host(ctx.matvec(dev(torch, x), prec=prec))
        ref = o.matvec(X, x, sigma, rc)
        assert (o.sqdist(X[0:1], X[1:2])[0, 0] <= rc * rc) and (o.sqdist(X[0:1], X[2:3])[0, 0] > rc * rc)
        assert abs(y[0] - ref[0]) <= 1e-6 * abs(ref[0]), (prec, y[0], ref[0])
        assert ref[0] == pytest.approx(math.exp(-rc * rc / (2 * sigma * sigma)))
    ctx.close()


def test_solve_well_conditioned_matches_lu(torch, R):
    c = w.lattice_cloud(7, 6, 0.1, jitter=0.25)
    eps, sigma = 0.05, 0.045
    X, b = o.extended_centres(c.points, c.normals, eps)
    assert np.linalg.cond(o.interpolation_matrix(X, sigma)) < 1e4
    ref, _ = o.solve_direct(X, b, sigma)
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), eps, sigma)
    for mode in (R.RBF_SOLVE_IR_FP32, R.RBF_SOLVE_PLAIN_FP64):
        coef, info = ctx.solve(tol=1e-12, mode=mode, restart=30)
        cg = host(coef)
        _say(f"[solve mode={mode}] status={info.status} iters={info.iters} outer={info.outer} "
             f"resid={info.rel_resid:.2e}")
        assert info.status == R.RBF_OK
        assert info.rel_resid <= 1e-12
        assert o.relative_residual(X, cg, b, sigma) <= 1e-11
        assert np.linalg.norm(cg - ref) / np.linalg.norm(ref) <= 1e-5
    ctx.close()


def test_default_rhs_equals_explicit_rhs(torch, R):
    """A solve without b builds the system's right-hand side (0 on the
    surface, +eps / -eps off it, Sec. II.B) on the device; it must give the
    same coefficients, to the bit, as the oracle's b passed explicitly."""
    make, eps, sigma, cutoff = CASES["torus_patch_cut"]
    c = make()
    X, b = o.extended_centres(c.points, c.normals, eps)
    for mode in (R.RBF_SOLVE_IR_FP32, R.RBF_SOLVE_PLAIN_FP64):
        out = []
        for explicit in (False, True):
            ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), eps, sigma, cutoff)
            try:
                kw = dict(tol=1e-10, mode=mode, restart=30, max_iters=60, max_outer=2)
                coef, info = ctx.solve(b=dev(torch, b), **kw) if explicit else ctx.solve(**kw)
                out.append((host(coef), info.rel_resid, info.iters))
            finally:
                ctx.close()
        _say(f"[default rhs mode={mode}] iters {out[0][2]} resid {out[0][1]:.3e}")
        assert np.array_equal(out[0][0], out[1][0])
        assert out[0][1] == out[1][1] and out[0][2] == out[1][2]


def test_gmres_iterates_match_oracle(torch, R):
    """After exactly k steps from zero, the device GMRES iterate equals the
    oracle's GMRES(k) iterate (same Krylov space, same minimiser)."""
    c = w.patch(w.torus(20000, seed=1), 300, seed=4)
    eps, sigma, rc = 0.01, 0.03, 0.12
    X, b = o.extended_centres(c.points, c.normals, eps)
    A = o.interpolation_matrix(X, sigma, rc)
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), eps, sigma, rc)
    for k in (1, 5, 17):
        ref = o.gmres(lambda v: A @ v, b, restart=k, max_iters=k, tol=0.0)
        coef, info = ctx.solve(tol=0.0, mode=R.RBF_SOLVE_PLAIN_FP64, restart=k, max_iters=k, max_outer=1)
        cg = host(coef)
        assert info.iters == k and info.status == R.RBF_ENOCONV
        rel = np.linalg.norm(cg - ref.x) / np.linalg.norm(ref.x)
        _say(f"[gmres k={k}] |c - c_oracle|/|c_oracle| = {rel:.2e} resid gpu {info.rel_resid:.6e} "
             f"oracle {ref.history[-1]:.6e}")
        assert rel <= 1e-9
        assert abs(info.rel_resid - ref.history[-1]) <= 1e-9 * ref.history[-1]
    ctx.close()


def test_solve_limits_and_resume(torch, R):
    c = w.lattice_cloud(5, 5, 0.1, jitter=0.2)
    eps, sigma = 0.05, 0.05
    X, b = o.extended_centres(c.points, c.normals, eps)
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), eps, sigma)
    c1, i1 = ctx.solve(tol=1e-14, mode=R.RBF_SOLVE_PLAIN_FP64, restart=4, max_iters=4)
    assert i1.status == R.RBF_ENOCONV and i1.iters == 4
    # resume from the stopped iterate; the history starts at its residual
    c2, i2 = ctx.solve(x0=c1.clone(), tol=1e-12, mode=R.RBF_SOLVE_PLAIN_FP64, restart=10)
    assert i2.status == R.RBF_OK
    assert i2.history[0] == pytest.approx(i1.rel_resid, rel=1e-12)
    ctx.close()


def test_solve_modes_alternate_on_one_context(torch, R):
    """The refinement's inner solve keeps its Krylov basis in float32 in the
    same storage the plain method uses in float64: alternating the modes on
    one context gives, bit for bit, what fresh contexts give."""
    make, eps, sigma, cutoff = CASES["torus_patch_cut"]
    c = make()
    P, N = dev(torch, c.points), dev(torch, c.normals)
    kw = dict(tol=1e-12, restart=20, max_iters=40)
    plain, ir = R.RBF_SOLVE_PLAIN_FP64, R.RBF_SOLVE_IR_FP32

    def fresh(mode):
        ctx = R.Rbf(P, N, eps, sigma, cutoff)
        try:
            x, info = ctx.solve(mode=mode, **kw)
            return host(x), info.rel_resid
        finally:
            ctx.close()

    ref_plain, ref_ir = fresh(plain), fresh(ir)
    ctx = R.Rbf(P, N, eps, sigma, cutoff)
    try:
        seq = []
        for mode in (plain, ir, plain, ir):
            x, info = ctx.solve(mode=mode, **kw)
            seq.append((host(x), info.rel_resid))
    finally:
        ctx.close()
    _say(f"[modes] plain {ref_plain[1]:.3e} refined {ref_ir[1]:.3e}")
    for (x, r), ref in zip(seq, (ref_plain, ref_ir, ref_plain, ref_ir)):
        assert np.array_equal(x, ref[0]) and r == ref[1]
    assert ref_ir[1] < 0.1 and ref_plain[1] < 0.1


# ---------------------------------------------------------------------------
# The sphere workload (2,000 points, no cutoff) at full size.
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def sphere_small(torch, R):
    cfg = w.SPHERE_SMALL
    c = w.sphere(cfg["n"], cfg["seed"])
    X, b = o.extended_centres(c.points, c.normals, cfg["eps"])
    coef, rel = o.solve_direct(X, b, cfg["sigma"])
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), cfg["eps"], cfg["sigma"], cfg["cutoff"])
    yield dict(c=c, X=X, b=b, coef=coef, ctx=ctx, cfg=cfg)
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_sphere_operator(sphere_small, torch, prec):
    s = sphere_small
    X, cfg = s["X"], s["cfg"]
    x = w.random_vector(X.shape[0], seed=4)
    y = host(s["ctx"].matvec(dev(torch, x), prec=prec))
    ref = o.matvec(X, x, cfg["sigma"])
    scale = abs_sums(X, x, range(X.shape[0]), cfg["sigma"], math.inf)
    ratio = np.max(np.abs(y - ref) / scale)
    _say(f"[sphere operator prec={prec}] max ratio {ratio / U32:.2f} u32")
    assert ratio <= (TOL32 if prec == 0 else TOL64)


def test_sphere_grid_with_oracle_weights(sphere_small, torch):
    """The grid tolerance of 1e-6 absolute, given the oracle's (LU) weights."""
    s = sphere_small
    cfg = s["cfg"]
    g = cfg["grid"]()
    f32 = host(s["ctx"].eval_grid(dev(torch, s["coef"]), g.origin, g.h, g.dims, prec=0))
    f64 = host(s["ctx"].eval_grid(dev(torch, s["coef"]), g.origin, g.h, g.dims, prec=1))
    ref = o.evaluate_grid(s["X"], s["coef"], g.origin, g.h, g.dims, cfg["sigma"])
    e32, e64 = np.max(np.abs(f32 - ref)), np.max(np.abs(f64 - ref))
    _say(f"[sphere grid] max |f32 - f| = {e32:.3e}  max |f64 - f| = {e64:.3e}")
    assert e32 <= 1e-6
    assert e64 <= 1e-12


# ---------------------------------------------------------------------------
# The torus workload (200,000 points, 600,000 centres, cutoff 4 sigma) at
# full size: sampled rows and nodes the oracle computes one by one.
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def torus_full(torch, R):
    cfg = w.TORUS_200K
    c = w.torus(cfg["n"], cfg["seed"])
    X, b = o.extended_centres(c.points, c.normals, cfg["eps"])
    _say("[torus] setup")
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), cfg["eps"], cfg["sigma"], cfg["cutoff"])
    yield dict(c=c, X=X, b=b, ctx=ctx, cfg=cfg)
    ctx.close()


def test_torus_stats(torus_full):
    st = torus_full["ctx"].stats()
    _say(f"[torus stats] groups={st.n_groups} entries={st.list_entries} useful={st.useful_pairs} "
         f"examined={st.examined_pairs} inflation={st.examined_pairs / st.useful_pairs:.3f} cells={st.n_cells}")
    assert st.n_centres == 600_000
    assert 4.5e8 < st.useful_pairs < 6.0e8


@pytest.mark.parametrize("prec", [0, 1])
def test_torus_operator_sampled_rows(torus_full, torch, prec):
    t = torus_full
    X, cfg = t["X"], t["cfg"]
    x = w.random_vector(X.shape[0], seed=4)
    y = host(t["ctx"].matvec(dev(torch, x), prec=prec))
    rows = np.random.default_rng(31).choice(X.shape[0], 400, replace=False)
    ref = o.matvec_rows(X, x, rows, cfg["sigma"], cfg["cutoff"])
    scale = abs_sums(X, x, rows, cfg["sigma"], cfg["cutoff"])
    ratio = np.max(np.abs(y[rows] - ref) / scale)
    _say(f"[torus operator prec={prec}] max ratio {ratio / U32:.2f} u32")
    assert ratio <= (TOL32 if prec == 0 else TOL64)


def test_torus_grid_sampled_nodes(torus_full, torch):
    t = torus_full
    X, cfg = t["X"], t["cfg"]
    g = w.Grid.around(t["c"].points, cfg["grid_n"])
    coef = np.random.default_rng(32).uniform(-1, 1, X.shape[0])
    out = host(t["ctx"].eval_grid(dev(torch, coef), g.origin, g.h, g.dims, prec=0))
    rng = np.random.default_rng(33)
    nz = np.flatnonzero(out)
    idx = np.concatenate([rng.choice(nz, 300, replace=False), rng.choice(g.size, 100, replace=False)])
    nodes = o.grid_nodes(g.origin, g.h, g.dims, idx)
    ref = o.evaluate(X, coef, nodes, cfg["sigma"], cfg["cutoff"])
    scale = abs_sums(X, coef, range(len(idx)), cfg["sigma"], cfg["cutoff"], targets=nodes)
    err = np.abs(out[idx] - ref)
    bound = TOL32 * scale + U32 * np.abs(ref) + 1e-300
    _say(f"[torus grid] band nodes {nz.size}, max err/bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound)
    assert np.all(out[idx][scale == 0] == 0)


# ---------------------------------------------------------------------------
# The metaball workload's geometry (hole, position noise, sigma 0.01, cutoff
# 4 sigma) at 100,000 points: sampled operator rows, sampled grid nodes and
# the pair count of sampled rows.
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def metaballs_100k(torch, R):
    cfg = dict(w.METABALLS_2M)
    c = w.metaballs(100_000, cfg["seed"])
    X, b = o.extended_centres(c.points, c.normals, cfg["eps"])
    _say("[metaballs 100k] setup")
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), cfg["eps"], cfg["sigma"], cfg["cutoff"])
    yield dict(c=c, X=X, b=b, ctx=ctx, cfg=cfg)
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_metaballs_operator_sampled_rows(metaballs_100k, torch, prec):
    t = metaballs_100k
    X, cfg = t["X"], t["cfg"]
    x = w.random_vector(X.shape[0], seed=4)
    y = host(t["ctx"].matvec(dev(torch, x), prec=prec))
    rows = np.random.default_rng(41).choice(X.shape[0], 400, replace=False)
    ref = o.matvec_rows(X, x, rows, cfg["sigma"], cfg["cutoff"])
    scale = abs_sums(X, x, rows, cfg["sigma"], cfg["cutoff"])
    ratio = np.max(np.abs(y[rows] - ref) / scale)
    _say(f"[metaballs operator prec={prec}] max ratio {ratio / U32:.2f} u32")
    assert ratio <= (tol32(cfg["sigma"], cfg["cutoff"]) if prec == 0 else TOL64)


def test_metaballs_pair_count_of_sampled_rows(metaballs_100k):
    """The useful pairs of the whole operator against the oracle's count on
    sampled rows, scaled: the row counts vary, so only a loose band."""
    t = metaballs_100k
    X, cfg = t["X"], t["cfg"]
    st = t["ctx"].stats()
    rows = np.random.default_rng(42).choice(X.shape[0], 300, replace=False)
    r2 = np.stack([o.sqdist(X[i:i + 1], X)[0] for i in rows])
    per_row = np.sum(r2 <= cfg["cutoff"] ** 2, axis=1)
    est = per_row.mean() * X.shape[0]
    _say(f"[metaballs pairs] device {st.useful_pairs}  sampled estimate {est:.4g}")
    assert 0.8 * est < st.useful_pairs < 1.25 * est


def test_metaballs_grid_sampled_nodes(metaballs_100k, torch):
    t = metaballs_100k
    X, cfg = t["X"], t["cfg"]
    g = w.Grid.around(t["c"].points, 128)
    coef = np.random.default_rng(43).uniform(-1, 1, X.shape[0])
    out = host(t["ctx"].eval_grid(dev(torch, coef), g.origin, g.h, g.dims, prec=0))
    rng = np.random.default_rng(44)
    nz = np.flatnonzero(out)
    idx = np.concatenate([rng.choice(nz, 300, replace=False), rng.choice(g.size, 100, replace=False)])
    nodes = o.grid_nodes(g.origin, g.h, g.dims, idx)
    ref = o.evaluate(X, coef, nodes, cfg["sigma"], cfg["cutoff"])
    scale = abs_sums(X, coef, range(len(idx)), cfg["sigma"], cfg["cutoff"], targets=nodes)
    err = np.abs(out[idx] - ref)
    bound = tol32(cfg["sigma"], cfg["cutoff"]) * scale + U32 * np.abs(ref) + 1e-300
    _say(f"[metaballs grid] band nodes {nz.size}, max err/bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound)
    assert np.all(out[idx][scale == 0] == 0)


# ---------------------------------------------------------------------------
# Density measures (Sec. IV: separation distance, fill distance, h_max).
# ---------------------------------------------------------------------------
def test_density_matches_paper_halton_example(torch, R):
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "halton25.json")))
    P = np.stack([w.halton(25, 2, 1), w.halton(25, 3, 1), np.zeros(25)], axis=1)
    nrm = np.tile([0.0, 0.0, 1.0], (25, 1))
    ctx = R.Rbf(dev(torch, P), dev(torch, nrm), 0.01, 0.1, 0.5)
    s = np.linspace(0.0, 1.0, 1501)
    gx, gy = np.meshgrid(s, s)
    S = np.stack([gx.ravel(), gy.ravel(), np.zeros(gx.size)], axis=1)
    d = ctx.density(dev(torch, S))
    q, hmax, h = d.q, d.h_max, d.h_fill
    half_unit = 0.5 * 10.0 ** (-g["printed_digits"])
    assert abs(q - g["q"]) <= half_unit and abs(h - g["h"]) <= half_unit
    assert q == o.separation_distance(P)
    assert hmax == o.h_max(P)
    assert h == o.fill_distance(P, S)
    # the sigma choices of eqs. h1 and h2 with the sampled fill distance
    assert d.h == h
    assert d.sigma_sep == 2.0 * o.separation_distance(P)
    assert d.sigma_fill == math.sqrt(2.0) * o.fill_distance(P, S)
    ctx.close()


def test_density_matches_oracle_on_a_patch(case):
    c = case["cloud"]
    d = case["ctx"].density()
    q, hmax, hf = d.q, d.h_max, d.h_fill
    if c.n < 2:
        assert math.isnan(q) and math.isnan(hmax) and math.isnan(d.sigma_sep)
        return
    assert q == o.separation_distance(c.points)
    assert hmax == o.h_max(c.points)
    assert math.isnan(hf)
    # without a domain sample the fill distance is estimated by eq. hmax
    assert d.h == math.sqrt(2.0) * o.h_max(c.points)
    assert d.sigma_sep == 2.0 * q
    assert d.sigma_fill == math.sqrt(2.0) * (math.sqrt(2.0) * o.h_max(c.points))


def test_measured_alu_rates_are_physical(torch, R):
    """The issue-rate probe behind the pair roofline, against the chip's unit
    counts: VOP2 float32 FMAs at most 32 lanes per SIMD per cycle at 2.5 GHz
    (the published float32 vector rate) and at least 16 lanes at 1 GHz; the
    DPP form, an exponential and the mixes no faster than the VOP2 FMA; the
    pair kernel's chunk bodies no faster than one exponential per pair step
    and the masked body (one more instruction per step) no faster than the
    inner one."""
    r = R.measure_rates()
    simds = r.compute_units * 4
    _say(f"[rates] CUs {r.compute_units} fma {r.fma_per_s:.3e}/s dpp fma {r.dpp_fma_per_s:.3e}/s "
         f"exp {r.exp_per_s:.3e}/s exp+3fma {r.exp_3fma_per_s:.3e}/s exp+7fma {r.exp_7fma_per_s:.3e}/s "
         f"inner steps {r.inner_pair_steps_per_s:.3e}/s masked steps {r.masked_pair_steps_per_s:.3e}/s")
    assert r.compute_units > 0
    assert simds * 16 * 1.0e9 <= r.fma_per_s <= simds * 32 * 2.5e9
    assert 0 < r.dpp_fma_per_s <= r.fma_per_s * 1.05
    assert 0 < r.exp_per_s <= r.fma_per_s * 1.05
    assert 0 < r.exp_7fma_per_s < r.exp_3fma_per_s < r.exp_per_s
    assert 0 < r.masked_pair_steps_per_s <= r.inner_pair_steps_per_s * 1.05
    assert r.inner_pair_steps_per_s <= r.exp_per_s * 1.05
