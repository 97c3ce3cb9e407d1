"""The C ABI: the library loads, exports every function include/rbf.h
declares, and rejects bad arguments with a status (never an abort).  These
run without a GPU: argument checks come before any device work, and with no
device the library answers RBF_EDEVICE."""
import ctypes as C
import math
import os
import re
import subprocess

import pytest

from paper_1305_5179_amd import rbf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbf.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rbf_[a-z_0-9]+)\s*\(", text)))


def _gpu_present():
    return os.path.exists("/dev/kfd")


def test_header_declarations_match_binding_list():
    assert _declared_functions() == sorted(rbf.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = rbf.load_library()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    nm = subprocess.run(["nm", "-D", "--defined-only", rbf.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (rbf_[a-z_0-9]+)$", nm, flags=re.M))
    assert set(_declared_functions()) <= exported
    # nothing else leaks out under the rbf_ prefix
    assert exported == set(_declared_functions())


def test_default_solve_options():
    o = rbf.default_opts()
    assert (o.tol, o.restart, o.max_outer, o.max_iters, o.mode, o.precond, o.basis, o.graph) == \
        (1e-8, 30, 1000, 30000, 1, 0, rbf.RBF_FP32, 1)
    assert C.sizeof(rbf.SolveOpts) == 40
    assert rbf.load_library().rbf_default_solve_opts(None) == rbf.RBF_EINVAL


def test_default_schwarz_options():
    o = rbf.SchwarzOpts()
    lib = rbf.load_library()
    assert lib.rbf_default_schwarz_opts(C.byref(o)) == rbf.RBF_OK
    assert (o.max_block, o.overlap_pct, o.restricted, o.min_block, o.shift, o.tune, o.half) == (192, 10, 0, 0, 0.3, 1, 0)
    assert lib.rbf_default_schwarz_opts(None) == rbf.RBF_EINVAL


def test_schwarz_entry_points_reject_null_context():
    lib = rbf.load_library()
    o = rbf.SchwarzOpts()
    lib.rbf_default_schwarz_opts(C.byref(o))
    assert lib.rbf_schwarz_setup(None, C.byref(o), None) == rbf.RBF_EINVAL
    p = C.c_void_p(0x1000)
    assert lib.rbf_schwarz_apply(None, p, p, None) == rbf.RBF_EINVAL
    info = rbf.SchwarzInfo()
    assert lib.rbf_schwarz_get_info(None, C.byref(info)) == rbf.RBF_EINVAL
    assert lib.rbf_schwarz_subdomains(None, None, None, None) == rbf.RBF_EINVAL


@pytest.mark.parametrize("n,eps,sigma,cutoff,msg", [
    (0, 0.01, 0.05, math.inf, "n must be positive"),
    (-3, 0.01, 0.05, math.inf, "n must be positive"),
    (10, 0.0, 0.05, math.inf, "off_surface_eps"),
    (10, float("nan"), 0.05, math.inf, "off_surface_eps"),
    (10, math.inf, 0.05, math.inf, "off_surface_eps"),
    (10, 0.01, -1.0, math.inf, "sigma"),
    (10, 0.01, float("nan"), math.inf, "sigma"),
    (10, 0.01, 0.05, 0.0, "cutoff"),
    (10, 0.01, 0.05, -1.0, "cutoff"),
    (10, 0.01, 0.05, float("nan"), "cutoff"),
])
def test_setup_rejects_bad_scalars(n, eps, sigma, cutoff, msg):
    lib = rbf.load_library()
    out = C.c_void_p(0x1234)
    p = C.c_void_p(0x1000)
    st = lib.rbf_setup(p, p, n, eps, sigma, cutoff, None, C.byref(out))
    assert st == rbf.RBF_EINVAL
    assert out.value is None
    assert msg in lib.rbf_last_error(None).decode()


def test_setup_null_out_pointer():
    lib = rbf.load_library()
    assert lib.rbf_setup(None, None, 10, 0.01, 0.05, 1.0, None, None) == rbf.RBF_EINVAL


@pytest.mark.skipif(_gpu_present(), reason="checks the no-device path")
def test_setup_without_device_is_edevice():
    lib = rbf.load_library()
    out = C.c_void_p()
    p = C.c_void_p(0x1000)
    assert lib.rbf_setup(p, p, 10, 0.01, 0.05, math.inf, None, C.byref(out)) == rbf.RBF_EDEVICE
    assert "device" in lib.rbf_last_error(None).decode()


def test_null_context_calls_are_einval():
    lib = rbf.load_library()
    v = C.c_void_p(0x1000)
    assert lib.rbf_matvec(None, v, v, 0, None) == rbf.RBF_EINVAL
    assert lib.rbf_solve(None, None, None, v, None, None, None) == rbf.RBF_EINVAL
    g = rbf.make_grid((0, 0, 0), (1, 1, 1), (2, 2, 2))
    assert lib.rbf_eval_grid(None, v, C.byref(g), v, 0, None) == rbf.RBF_EINVAL
    assert lib.rbf_eval_points(None, v, v, 3, v, 0, None) == rbf.RBF_EINVAL
    assert lib.rbf_centres(None, v, v, None) == rbf.RBF_EINVAL
    assert lib.rbf_get_stats(None, None) == rbf.RBF_EINVAL
    assert lib.rbf_count_grid_pairs(None, C.byref(g), None, None, None) == rbf.RBF_EINVAL
    d = rbf.DensityInfo()
    assert lib.rbf_density(None, None, 0, C.byref(d), None) == rbf.RBF_EINVAL
    H = (C.c_double * 6)()
    k = C.c_int()
    assert lib.rbf_arnoldi(None, v, 2, 1, 1, v, H, C.byref(k), None) == rbf.RBF_EINVAL
    lib.rbf_destroy(None)
    assert lib.rbf_last_error(None)


def test_binding_refuses_host_tensors():
    import torch
    with pytest.raises(TypeError):
        rbf._ptr(torch.zeros(3, dtype=torch.float64))


@pytest.mark.gpu
def test_binding_checks_sizes_shapes_and_devices():
    """The C side cannot check array lengths behind raw pointers: the binding
    refuses wrongly sized or shaped tensors before calling it."""
    import numpy as np
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1305_5179_amd import workloads as w
    c = w.sphere(50, seed=1)
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")  # noqa: E731
    with pytest.raises(ValueError):
        rbf.Rbf(d(c.points).reshape(-1), d(c.normals), 0.01, 0.2, 0.6)      # points not (n, 3)
    with pytest.raises(ValueError):
        rbf.Rbf(d(c.points), d(c.normals[:-1]), 0.01, 0.2, 0.6)             # normals of n - 1 rows
    ctx = rbf.Rbf(d(c.points), d(c.normals), 0.01, 0.2, 0.6)
    m = ctx.m
    good, short = torch.zeros(m, dtype=torch.float64, device="cuda"), torch.zeros(m - 1, dtype=torch.float64,
                                                                               device="cuda")
    with pytest.raises(ValueError):
        ctx.matvec(short)
    with pytest.raises(ValueError):
        ctx.matvec(good, short)
    with pytest.raises(ValueError):
        ctx.solve(b=short)
    with pytest.raises(ValueError):
        ctx.solve(x0=short)
    with pytest.raises(ValueError):
        ctx.solve(c=short)
    with pytest.raises(ValueError):
        ctx.eval_grid(short, (0, 0, 0), (0.1, 0.1, 0.1), (4, 4, 4))
    with pytest.raises(ValueError):
        ctx.eval_grid(good, (0, 0, 0), (0.1, 0.1, 0.1), (4, 4, 4),
                      out=torch.zeros(63, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        ctx.eval_points(good, torch.zeros(12, dtype=torch.float64, device="cuda"))   # pts not (k, 3)
    with pytest.raises(ValueError):
        ctx.eval_points(good, torch.zeros((4, 3), dtype=torch.float64, device="cuda"),
                        out=torch.zeros(3, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        ctx.density(torch.zeros(9, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        ctx.arnoldi(short, 3)
    with pytest.raises(TypeError):
        ctx.matvec(torch.zeros(m, dtype=torch.float32, device="cuda"))
    with pytest.raises(TypeError):
        ctx.matvec(torch.zeros(m, dtype=torch.float64))                    # host tensor
    # a well-formed call still works after the refusals
    y = ctx.matvec(good)
    torch.cuda.synchronize()
    assert float(torch.abs(y).max()) == 0.0
    ctx.close()
