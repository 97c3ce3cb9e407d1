"""Contexts used from several host threads at once, each thread on its own
stream: every result equals, bit for bit, the same calls made one after
another on the main thread.  The library's host state that calls share or
keep per thread (the caching allocator, the pinned read-back slots, the
error text, the temporary-memory stream) must keep concurrent calls apart;
the device work itself is deterministic, so any mix-up shows as a changed
bit.  Workloads: a torus patch with a cutoff (lists, masks, the brick grid,
a refinement solve, the Schwarz preconditioner and a preconditioned solve)
and a small sphere without one (dense lists)."""
import sys
import threading

import numpy as np
import pytest

from paper_1305_5179_amd import workloads as w

pytestmark = pytest.mark.gpu

CASES = [
    ("torus_patch", lambda: w.patch(w.torus(), 1701, seed=3), 0.005, 0.02, 0.08, 48),
    ("sphere_dense", lambda: w.sphere(333, seed=7), 0.02, 0.2, float("inf"), 24),
]


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


def _work(torch, R, case):
    """Setup, both matvecs, a short refinement solve and the grid, on the
    current stream; host copies of every output."""
    _, make, eps, sigma, cutoff, gn = case
    c = make()
    dev = torch.device("cuda", 0)
    pts = torch.as_tensor(c.points, device=dev).contiguous()
    nrm = torch.as_tensor(c.normals, device=dev).contiguous()
    ctx = R.Rbf(pts, nrm, eps, sigma, cutoff)
    try:
        x = torch.as_tensor(w.random_vector(ctx.m, seed=4), device=dev)
        y32 = ctx.matvec(x, prec=R.RBF_FP32)
        y64 = ctx.matvec(x, prec=R.RBF_FP64)
        coef, info = ctx.solve(tol=1e-10, restart=20, max_iters=60, max_outer=3)
        g = w.Grid.around(c.points, gn)
        f = ctx.eval_grid(coef, g.origin, g.h, g.dims, prec=R.RBF_FP32)
        out = dict(y32=y32.cpu().numpy(), y64=y64.cpu().numpy(), coef=coef.cpu().numpy(),
                   grid=f.cpu().numpy(), iters=info.iters, resid=info.rel_resid, status=info.status)
        if cutoff != float("inf"):
            # the Schwarz preconditioner (float16 inverses: the launch-shape
            # tuner times candidates, but every shape gives the same bits)
            ctx.schwarz_setup(max_block=96, half=1)
            z = ctx.schwarz_apply(x)
            pc, pinfo = ctx.solve(tol=1e-10, restart=20, max_iters=60, max_outer=3,
                                  precond=R.RBF_PRECOND_SCHWARZ)
            out.update(z=z.cpu().numpy(), pcoef=pc.cpu().numpy(), piters=pinfo.iters, presid=pinfo.rel_resid)
        torch.cuda.current_stream().synchronize()
        return out
    finally:
        ctx.close()


def _same(a, b, label):
    for k in a:
        if isinstance(a[k], np.ndarray):
            assert a[k].shape == b[k].shape, (label, k)
            assert np.array_equal(a[k], b[k]), (label, k, np.max(np.abs(a[k] - b[k])))
        else:
            assert a[k] == b[k], (label, k, a[k], b[k])


def test_concurrent_contexts_on_own_streams(torch, R):
    _say("[threads] sequential reference runs")
    ref = [_work(torch, R, case) for case in CASES]
    # four threads: each case twice, all at once, every thread on a stream
    # of its own (created by the thread, default priority)
    jobs = [CASES[i % len(CASES)] for i in range(4)]
    results = [None] * len(jobs)
    errors = []
    start = threading.Barrier(len(jobs))

    def run(i):
        try:
            s = torch.cuda.Stream()
            start.wait(timeout=60)
            with torch.cuda.stream(s):
                results[i] = _work(torch, R, jobs[i])
        except Exception as e:   # reported by the main thread
            errors.append((i, repr(e)))

    _say("[threads] four threads, two cases each twice")
    threads = [threading.Thread(target=run, args=(i,), daemon=True) for i in range(len(jobs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads), "a thread did not finish"
    assert not errors, errors
    for i, job in enumerate(jobs):
        _same(ref[i % len(CASES)], results[i], f"{job[0]} (thread {i})")
    _say("[threads] every output equal to the sequential run, bit for bit")
