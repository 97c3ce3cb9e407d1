"""GPU parity of the Schwarz preconditioner: the HIP path, called through the
C ABI, against the CPU oracle (oracle/schwarz.py) on the same seeded inputs.

  * subdomains (octree cores, k-nearest overlaps): bit-exact integer sets,
    the overlap in its nearest-first order;
  * z = M^{-1} r: the device inverts each block in float64 and keeps the
    inverse in float32, so |z_gpu - z_oracle|_j <= 4 u32 sum_i sum_b
    |(A_i + shift I)^{-1}_{jb}| |r_b| (the oracle's own inverses give the
    bound) plus a float64 term; with `half` in float16, every entry rounded
    once (relative 2^-11, absolute 2^-25 below the normal range), and the
    products and sums in float32 (at most n u32 <= 2^-14 relative for blocks
    up to 1024), so |z_gpu - z_oracle|_j <= 2 u16 sum_i sum_b (|inv_{jb}| +
    2^-13) |r_b|;
  * the preconditioned solve: the float64 residual the library reports is
    the oracle's, and on a small well-conditioned system the weights match
    LU to 1e-5.
"""
import math
import sys

import numpy as np
import pytest

from oracle import rbf_oracle as o
from oracle import schwarz as S
from paper_1305_5179_amd import workloads as w

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


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


def _clustered(n, seed):
    """Clusters, a sparse background and coincident points (finest-level
    leaves above the cap, and cores whose overlap needs the full search)."""
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(n // 2, 3)) * 0.03 + np.array([0.2, -0.1, 0.05])
    b = rng.uniform(-1, 1, size=(n - n // 2 - 80, 3))
    dup = np.repeat(a[:1], 80, axis=0)
    P = np.concatenate([a, b, dup])
    N = rng.normal(size=P.shape)
    return w.Cloud(P, N, "clustered")


CLOUDS = {
    "sphere2000": (lambda: w.sphere(2000, 0), 0.01, 0.05, math.inf),
    "torus6000": (lambda: w.torus(n=6000, seed=1, R=0.1732, r=0.0606), 0.005, 0.02, 0.08),
    "clustered1500": (lambda: _clustered(1500, 9), 0.01, 0.05, 0.2),
}

OPTS = {
    "default": dict(),
    "restricted30": dict(restricted=1, overlap_pct=30),
    "small_blocks": dict(max_block=40, overlap_pct=20),
    # blocks above the LDS order (swept in global memory), with and without
    # the merge of small leaves; mixed sizes in one launch
    "large_merged": dict(max_block=1024, min_block=64),
    "mixed_restricted": dict(max_block=600, min_block=200, restricted=1),
    # the inverses in float16 (rows of even length; odd blocks occur)
    "default_half": dict(half=1),
    "restricted_half": dict(restricted=1, overlap_pct=30, half=1),
    "large_half": dict(max_block=1024, min_block=64, half=1),
}
U16 = 2.0 ** -11


def _subs_key(subs):
    return {int(np.min(core)): (np.sort(core), np.asarray(ov)) for core, ov in subs}


@pytest.fixture(scope="module")
def built(torch, R):
    cache = {}

    def get(name, optname):
        key = (name, optname)
        if key not in cache:
            make, eps, sigma, cutoff = CLOUDS[name]
            c = make()
            _say(f"[schwarz] setup {name} {optname}")
            ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), eps, sigma, cutoff)
            info = ctx.schwarz_setup(**OPTS[optname])
            torch.cuda.synchronize()
            X, _ = o.extended_centres(c.points, c.normals, eps)
            cache[key] = (c, ctx, info, X, sigma, cutoff)
        return cache[key]
    yield get
    for v in cache.values():
        v[1].close()


def _oracle_opts(optname):
    d = dict(max_block=192, overlap_pct=10, restricted=0, shift=0.3, min_block=0)
    d.update(OPTS[optname])
    d.pop("half", None)
    return d


@pytest.mark.parametrize("name", list(CLOUDS))
@pytest.mark.parametrize("optname", list(OPTS))
def test_subdomains_are_the_oracles(built, name, optname):
    c, ctx, info, X, sigma, cutoff = built(name, optname)
    oo = _oracle_opts(optname)
    gpu = ctx.schwarz_subdomains()
    assert info.retries == 0 and info.n_sub == len(gpu)
    assert info.max_members <= oo["max_block"]
    cap = S.core_cap(oo["max_block"], oo["overlap_pct"])
    leaves = S.merge_leaves(S.octree_cores(c.points, cap), cap, oo["min_block"], oo["overlap_pct"])
    n = len(c.points)
    cores = {int(np.min(S.core_centres(l, n))): np.sort(S.core_centres(l, n)) for l in leaves}
    g = _subs_key(gpu)
    assert sorted(g) == sorted(cores)
    for k0, core in cores.items():
        assert np.array_equal(g[k0][0], core), k0
    # every centre in exactly one core
    allc = np.sort(np.concatenate([core for core, _ in gpu]))
    assert np.array_equal(allc, np.arange(3 * n))
    # overlaps: all of them on small clouds, a seeded sample otherwise
    keys = sorted(cores)
    nkeys = 60 if oo["max_block"] <= 192 else 16
    if len(keys) > nkeys:
        keys = list(np.random.default_rng(4).choice(keys, nkeys, replace=False))
    for k0 in keys:
        core = cores[k0]
        want = S.overlap(X, core, min(S.overlap_count(core.size, oo["overlap_pct"]), len(X) - core.size))
        assert np.array_equal(g[k0][1], want), (k0, g[k0][1][:8], want[:8])


def _apply_bound(X, subs, sigma, shift, r, restricted, floor=0.0):
    """sum_i sum_b (|inv_i[j, b]| + floor) |r_b| over the subdomains i holding j."""
    B = np.zeros(len(X))
    for core, ov in subs:
        mem = np.concatenate([core, ov])
        inv = np.abs(np.linalg.inv(S.local_matrix(X, mem, sigma, shift))) + floor
        rows = core.size if restricted else mem.size
        B[mem[:rows]] += inv[:rows] @ np.abs(r[mem])
    return B


@pytest.mark.parametrize("name", ["sphere2000", "clustered1500"])
@pytest.mark.parametrize("optname", list(OPTS))
def test_apply_matches_the_oracle(torch, built, name, optname):
    c, ctx, info, X, sigma, cutoff = built(name, optname)
    oo = _oracle_opts(optname)
    subs = S.subdomains(c.points, X, oo["max_block"], oo["overlap_pct"], oo["min_block"])
    r = np.random.default_rng(11).uniform(-1, 1, len(X))
    _say(f"[schwarz] apply {name} {optname}")
    z = host(ctx.schwarz_apply(dev(torch, r)))
    torch.cuda.synchronize()
    want = S.schwarz_apply(X, subs, sigma, oo["shift"], r, restricted=bool(oo["restricted"]))
    half = OPTS[optname].get("half", 0) == 1
    B = _apply_bound(X, subs, sigma, oo["shift"], r, bool(oo["restricted"]), floor=2.0 ** -13 if half else 0.0)
    err = np.abs(z - want)
    tol = (2 * U16 if half else 4 * U32) * B + 1e-12 * np.abs(want).max()
    assert np.all(np.isfinite(z))
    worst = int(np.argmax(err / tol))
    _say(f"[schwarz] apply {name} {optname}: max err / bound {(err / tol).max():.3f}")
    assert np.all(err <= tol), (worst, err[worst], tol[worst], (err / (U32 * B)).max())


@pytest.mark.parametrize("max_block", [192, 1024])
def test_apply_small_shift_and_torus_sample(torch, R, max_block):
    """A 1e-6 shift (inverse entries in the 1e5 range, ill-conditioned local
    blocks): the float32 bound still holds element by element; torus patch,
    sampled rows; blocks up to 192 and up to 1024 centres."""
    make, eps, sigma, cutoff = CLOUDS["torus6000"]
    c = make()
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), eps, sigma, cutoff)
    try:
        _say(f"[schwarz] torus6000 shift 1e-6 max_block {max_block}")
        info = ctx.schwarz_setup(shift=1e-6, max_block=max_block)
        assert info.retries == 0
        X, _ = o.extended_centres(c.points, c.normals, eps)
        subs = S.subdomains(c.points, X, max_block=max_block)      # the oracle's own decomposition
        r = np.random.default_rng(12).uniform(-1, 1, len(X))
        z = host(ctx.schwarz_apply(dev(torch, r)))
        torch.cuda.synchronize()
        # the rows of a seeded sample of cores; a centre's value sums the
        # local solutions of every subdomain that holds it
        holders = {}
        for i, (core, ov) in enumerate(subs):
            for j in np.concatenate([core, ov]):
                holders.setdefault(int(j), []).append(i)
        solved = {}

        def local(h):
            if h not in solved:
                hc, ho = subs[h]
                mem = np.concatenate([hc, ho])
                A = S.local_matrix(X, mem, sigma, 1e-6)
                solved[h] = (mem, np.linalg.solve(A, r[mem]), np.abs(np.linalg.inv(A)) @ np.abs(r[mem]))
            return solved[h]

        for i in np.random.default_rng(13).choice(len(subs), min(25, len(subs)), replace=False):
            core = subs[i][0]
            want = np.zeros(core.size)
            bound = np.zeros(core.size)
            for t, j in enumerate(core):
                for h in holders[int(j)]:
                    mem, y, b = local(h)
                    pos = int(np.nonzero(mem == j)[0][0])
                    want[t] += y[pos]
                    bound[t] += b[pos]
            err = np.abs(z[core] - want)
            assert np.all(err <= 4 * U32 * bound + 1e-10 * np.abs(want).max()), (i, err.max(), bound.max())
    finally:
        ctx.close()


@pytest.mark.parametrize("half", [0, 1])
def test_preconditioned_solve_small_well_conditioned(torch, R, half):
    """A small sphere with sigma below the spacing: the preconditioned IR
    solve reaches 1e-12 and its weights match LU to 1e-5 (with float32 or
    float16 local inverses: the preconditioner changes, the residual the
    solver stops on is the float64 one)."""
    c = w.sphere(300, 3)
    eps, sigma = 0.08, 0.06
    X, b = o.extended_centres(c.points, c.normals, eps)
    A = o.interpolation_matrix(X, sigma)
    assert np.linalg.cond(A) < 1e4
    c_lu = np.linalg.solve(A, b)
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), eps, sigma, math.inf)
    try:
        ctx.schwarz_setup(max_block=60, overlap_pct=20, half=half)
        for mode in (R.RBF_SOLVE_IR_FP32, R.RBF_SOLVE_PLAIN_FP64):
            _say(f"[schwarz] solve sphere300 mode {mode}")
            cw, res = ctx.solve(tol=1e-12, mode=mode, precond=R.RBF_PRECOND_SCHWARZ, max_iters=3000)
            torch.cuda.synchronize()
            cg = host(cw)
            assert res.status == R.RBF_OK, res
            assert np.linalg.norm(cg - c_lu) <= 1e-5 * np.linalg.norm(c_lu)
            assert o.relative_residual(X, cg, b, sigma) <= 1e-11
    finally:
        ctx.close()


def test_preconditioned_solve_torus_patch(torch, R, built):
    """Torus patch at the paper's density: the reported residual is the
    oracle's, and the additive form reaches 1e-3 in fewer operator
    applications than no preconditioner."""
    c, ctx, info, X, sigma, cutoff = built("torus6000", "default")
    b = o.extended_centres(c.points, c.normals, 0.005)[1]
    out = {}
    for pre in (R.RBF_PRECOND_NONE, R.RBF_PRECOND_SCHWARZ):
        _say(f"[schwarz] solve torus6000 precond {pre}")
        cw, res = ctx.solve(tol=1e-3, precond=pre, max_iters=600)
        torch.cuda.synchronize()
        cg = host(cw)
        rel = o.relative_residual(X, cg, b, sigma, cutoff)
        assert abs(rel - res.rel_resid) <= 1e-6 * max(rel, 1e-12) + 1e-13, (rel, res.rel_resid)
        out[pre] = (res.status, res.iters, rel)
    _say(f"[schwarz] torus6000 to 1e-3: {out}")
    assert out[R.RBF_PRECOND_SCHWARZ][0] == R.RBF_OK
    assert out[R.RBF_PRECOND_SCHWARZ][1] < out[R.RBF_PRECOND_NONE][1]


def test_setup_rejects_bad_options(torch, R):
    c = w.sphere(50, 1)
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), 0.01, 0.05, math.inf)
    try:
        for bad in (dict(max_block=2), dict(max_block=1025), dict(overlap_pct=-1), dict(overlap_pct=101),
                    dict(restricted=2), dict(half=2), dict(shift=-1.0), dict(shift=float("nan")),
                    dict(max_block=3, overlap_pct=10), dict(min_block=-1), dict(max_block=100, min_block=101),
                    dict(tune=2)):
            with pytest.raises(R.RbfError) as e:
                ctx.schwarz_setup(**bad)
            assert e.value.status == R.RBF_EINVAL, bad
        with pytest.raises(R.RbfError):
            ctx.solve(precond=R.RBF_PRECOND_SCHWARZ)    # none set up
        info = ctx.schwarz_setup(max_block=6, overlap_pct=0)   # two points per core
        assert info.max_members <= 6
    finally:
        ctx.close()


def test_one_point(torch, R):
    """One point: one subdomain of its three centres, no room for overlap."""
    P = np.array([[0.1, 0.2, 0.3]])
    N = np.array([[0.0, 0.0, 1.0]])
    ctx = R.Rbf(dev(torch, P), dev(torch, N), 0.05, 0.1, math.inf)
    try:
        info = ctx.schwarz_setup()
        assert info.n_sub == 1 and info.n_members == 3
        X, _ = o.extended_centres(P, N, 0.05)
        r = np.array([1.0, -2.0, 0.5])
        z = host(ctx.schwarz_apply(dev(torch, r)))
        want = np.linalg.solve(S.local_matrix(X, np.arange(3), 0.1, 0.3), r)
        assert np.allclose(z, want, rtol=1e-6, atol=0)
    finally:
        ctx.close()


def test_restricted_solve_and_setup_twice(torch, R):
    """The restricted form preconditions the solve too, and a second setup
    replaces the first."""
    c = w.sphere(300, 3)
    eps, sigma = 0.08, 0.06
    X, b = o.extended_centres(c.points, c.normals, eps)
    c_lu = np.linalg.solve(o.interpolation_matrix(X, sigma), b)
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), eps, sigma, math.inf)
    try:
        ctx.schwarz_setup(max_block=60, overlap_pct=20)
        info = ctx.schwarz_setup(max_block=90, overlap_pct=30, restricted=1)
        assert info.max_members <= 90
        _say("[schwarz] restricted solve sphere300")
        cw, res = ctx.solve(tol=1e-12, precond=R.RBF_PRECOND_SCHWARZ, max_iters=3000)
        torch.cuda.synchronize()
        assert res.status == R.RBF_OK, res
        assert np.linalg.norm(host(cw) - c_lu) <= 1e-5 * np.linalg.norm(c_lu)
    finally:
        ctx.close()


@pytest.mark.parametrize("name", ["sphere2000", "clustered1500"])
def test_large_blocks_are_used(built, name):
    """The large configurations do put blocks above the LDS order (192) in
    the launch, and one launch per cloud holds blocks of both kinds (the
    LDS sweep and the global-memory sweep side by side)."""
    c, ctx, info, X, sigma, cutoff = built(name, "large_merged")
    gpu = ctx.schwarz_subdomains()
    sizes = np.array([core.size + ov.size for core, ov in gpu])
    _say(f"[schwarz] {name} large_merged: {len(gpu)} blocks, sizes {sizes.min()}..{sizes.max()}, "
         f"factor {info.factor_ms:.2f} ms, apply {info.apply_threads} x {info.apply_blocks}")
    assert sizes.max() > 192 and sizes.max() <= 1024
    assert info.min_members == sizes.min() and info.max_members == sizes.max()
    mixed = {"sphere2000": "mixed_restricted", "clustered1500": "large_merged"}[name]
    c2, ctx2, info2, *_ = built(name, mixed)
    sizes2 = np.array([core.size + ov.size for core, ov in ctx2.schwarz_subdomains()])
    assert sizes2.max() > 192 and sizes2.min() <= 192


def test_launch_shape_does_not_change_the_result(torch, R):
    """Every row of W r is formed by one lane in a fixed order, so the tuned
    and the fixed launch shapes give the same bits (additive and restricted)."""
    make, eps, sigma, cutoff = CLOUDS["sphere2000"]
    c = make()
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), eps, sigma, cutoff)
    try:
        r = dev(torch, np.random.default_rng(21).uniform(-1, 1, 3 * len(c.points)))
        for restricted in (0, 1):
            out = []
            for tune in (0, 1):
                _say(f"[schwarz] sphere2000 max_block 700 restricted {restricted} tune {tune}")
                info = ctx.schwarz_setup(max_block=700, restricted=restricted, tune=tune)
                out.append(host(ctx.schwarz_apply(r)))
                torch.cuda.synchronize()
                if tune == 0:
                    # the covering workgroup size, one workgroup per task
                    assert info.apply_threads in (128, 256, 512)
                    if not restricted:
                        need = info.max_members
                        assert info.apply_threads == (128 if need <= 128 else 256 if need <= 256 else 512)
            assert np.array_equal(out[0], out[1])
    finally:
        ctx.close()


def _k_nearest_outside(X, core, k):
    """The k centres outside `core` nearest to it by the oracle's distance:
    candidates from a k-d tree on the core (scipy), then the exact float64
    (dx dx + dy dy) + dz dz to every core centre, ties by index."""
    from scipy.spatial import cKDTree
    tree = cKDTree(X[core])
    d, _ = tree.query(X, k=1)
    d[core] = np.inf
    cand = np.argsort(d, kind="stable")[:k + 64]
    dd = X[cand][:, None, :] - X[core][None, :, :]
    exact = ((dd[..., 0] * dd[..., 0] + dd[..., 1] * dd[..., 1]) + dd[..., 2] * dd[..., 2]).min(axis=1)
    order = np.lexsort((cand, exact))
    return cand[order[:k]]


def test_torus200k_2048_subdomains(torch, R):
    """The torus workload split into about 2,000 subdomains of 64..1024
    centres (blocks up to 1024, small octree leaves merged up to 64): cores
    equal to the oracle's, overlaps of sampled cores the k nearest, and the
    apply's rows of sampled cores against float64 local solves of every
    subdomain holding them."""
    cfg = w.TORUS_200K
    c = w.torus(cfg["n"], cfg["seed"])
    X, _ = o.extended_centres(c.points, c.normals, cfg["eps"])
    n = len(c.points)
    ctx = R.Rbf(dev(torch, c.points), dev(torch, c.normals), cfg["eps"], cfg["sigma"], cfg["cutoff"])
    try:
        _say("[schwarz] torus200k max_block 1024 min_block 64: setup")
        info = ctx.schwarz_setup(max_block=1024, min_block=64)
        torch.cuda.synchronize()
        gpu = ctx.schwarz_subdomains()
        sizes = np.array([a.size + b.size for a, b in gpu])
        _say(f"[schwarz] torus200k: {len(gpu)} subdomains, sizes {sizes.min()}..{sizes.max()} "
             f"(median {int(np.median(sizes))}), factor {info.factor_ms:.1f} ms, retries {info.retries}, "
             f"apply {info.apply_threads} x {info.apply_blocks}")
        assert 1500 <= len(gpu) <= 2500 and sizes.max() <= 1024 and sizes.min() >= 64
        cap = S.core_cap(1024, 10)
        leaves = S.merge_leaves(S.octree_cores(c.points, cap), cap, 64, 10)
        cores = {int(np.min(S.core_centres(l, n))): np.sort(S.core_centres(l, n)) for l in leaves}
        g = _subs_key(gpu)
        assert sorted(g) == sorted(cores)
        for k0, core in cores.items():
            assert np.array_equal(g[k0][0], core), k0
        rng = np.random.default_rng(31)
        for k0 in rng.choice(sorted(cores), 8, replace=False):
            core = cores[int(k0)]
            want = _k_nearest_outside(X, core, S.overlap_count(core.size, 10))
            assert np.array_equal(g[int(k0)][1], want), k0
        r = rng.uniform(-1, 1, len(X))
        z = host(ctx.schwarz_apply(dev(torch, r)))
        torch.cuda.synchronize()
        members = [np.concatenate([a, b]) for a, b in gpu]
        for i in rng.choice(len(gpu), 6, replace=False):
            core = gpu[i][0]
            want = np.zeros(core.size)
            bound = np.zeros(core.size)
            for h, mem in enumerate(members):
                pos = np.nonzero(np.isin(mem, core))[0]
                if pos.size == 0:
                    continue
                A = S.local_matrix(X, mem, cfg["sigma"], 0.3)
                y = np.linalg.solve(A, r[mem])
                b = np.abs(np.linalg.inv(A)) @ np.abs(r[mem])
                idx = np.searchsorted(np.sort(core), mem[pos])
                order = np.argsort(core)
                want[order[idx]] += y[pos]
                bound[order[idx]] += b[pos]
            err = np.abs(z[core] - want)
            assert np.all(err <= 4 * U32 * bound + 1e-12 * np.abs(want).max()), (i, err.max(), bound.max())
    finally:
        ctx.close()
