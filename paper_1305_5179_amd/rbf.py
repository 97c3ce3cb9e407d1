"""ctypes binding of librbf (include/rbf.h).

Argument marshalling only: every step runs in the HIP library.  Arrays are
torch tensors on the GPU (float64, contiguous); calls are enqueued on the
current torch stream.  The library must have been built
(``python -m paper_1305_5179_amd.build``); loading raises when it is missing.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbf.so")

RBF_OK, RBF_EINVAL, RBF_ENOMEM, RBF_EDEVICE, RBF_ENOCONV, RBF_EBREAKDOWN = 0, -1, -2, -3, -4, -5
RBF_FP32, RBF_FP64 = 0, 1
RBF_SOLVE_PLAIN_FP64, RBF_SOLVE_IR_FP32 = 0, 1
RBF_PRECOND_NONE, RBF_PRECOND_SCHWARZ = 0, 1
STATUS_NAMES = {0: "RBF_OK", -1: "RBF_EINVAL", -2: "RBF_ENOMEM", -3: "RBF_EDEVICE",
                -4: "RBF_ENOCONV", -5: "RBF_EBREAKDOWN"}

# Every symbol include/rbf.h declares.
EXPORTS = ["rbf_default_solve_opts", "rbf_setup", "rbf_centres", "rbf_matvec", "rbf_solve",
           "rbf_eval_grid", "rbf_eval_points", "rbf_density", "rbf_get_stats", "rbf_count_grid_pairs",
           "rbf_profile_begin", "rbf_profile_end", "rbf_destroy", "rbf_last_error",
           "rbf_default_schwarz_opts", "rbf_schwarz_setup", "rbf_schwarz_apply", "rbf_schwarz_get_info",
           "rbf_schwarz_subdomains", "rbf_net_set", "rbf_net_get", "rbf_net_forward", "rbf_net_gradient",
           "rbf_net_train", "rbf_eval_grid_culled", "rbf_arnoldi", "rbf_eval_grid_noalloc",
           "rbf_measure_rates"]
RBF_NET_PARAMS = 50177


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int), ("max_outer", C.c_int),
                ("max_iters", C.c_int), ("mode", C.c_int), ("precond", C.c_int), ("basis", C.c_int),
                ("graph", C.c_int)]


class SchwarzOpts(C.Structure):
    _fields_ = [("max_block", C.c_int), ("overlap_pct", C.c_int), ("restricted", C.c_int),
                ("min_block", C.c_int), ("shift", C.c_double), ("tune", C.c_int), ("half", C.c_int)]


class SchwarzInfo(C.Structure):
    _fields_ = [("n_sub", C.c_int64), ("n_members", C.c_int64), ("max_members", C.c_int64),
                ("inverse_bytes", C.c_int64), ("retries", C.c_int), ("max_shift", C.c_double),
                ("min_members", C.c_int64), ("apply_threads", C.c_int), ("apply_blocks", C.c_int),
                ("factor_ms", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("outer", C.c_int), ("rel_resid", C.c_double), ("status", C.c_int),
                ("n_history", C.c_int), ("history", C.POINTER(C.c_double)),
                ("history_ms", C.POINTER(C.c_double))]


class DensityInfo(C.Structure):
    _fields_ = [("q", C.c_double), ("h_max", C.c_double), ("h_fill", C.c_double), ("h", C.c_double),
                ("sigma_sep", C.c_double), ("sigma_fill", C.c_double)]


class Grid(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("h", C.c_double * 3), ("dims", C.c_int64 * 3)]


class Stats(C.Structure):
    _fields_ = [("n_points", C.c_int64), ("n_centres", C.c_int64), ("n_groups", C.c_int64),
                ("list_entries", C.c_int64), ("useful_pairs", C.c_int64), ("examined_pairs", C.c_int64),
                ("n_cells", C.c_int64), ("cell_size", C.c_double), ("sigma", C.c_double),
                ("cutoff", C.c_double), ("eps", C.c_double), ("inner_entries", C.c_int64)]


class Profile(C.Structure):
    """Arrays indexed [kind][prec]: kind 0 = operator, 1 = evaluation."""
    _fields_ = [("launches", (C.c_int64 * 2) * 2), ("kernel_ms", (C.c_double * 2) * 2),
                ("useful_pairs", (C.c_int64 * 2) * 2), ("examined_pairs", (C.c_int64 * 2) * 2)]


class Rates(C.Structure):
    _fields_ = [("compute_units", C.c_int), ("fma_per_s", C.c_double), ("exp_per_s", C.c_double),
                ("exp_3fma_per_s", C.c_double), ("exp_7fma_per_s", C.c_double), ("dpp_fma_per_s", C.c_double),
                ("inner_pair_steps_per_s", C.c_double), ("masked_pair_steps_per_s", C.c_double)]


class CullStats(C.Structure):
    _fields_ = [("support_bricks", C.c_int64), ("kept_bricks", C.c_int64), ("useful_pairs", C.c_int64),
                ("examined_pairs", C.c_int64)]


class RbfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library() -> C.CDLL:
    """Load librbf.so and declare its prototypes."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1305_5179_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i64, dbl, i32 = C.c_void_p, C.c_int64, C.c_double, C.c_int
    lib.rbf_default_solve_opts.argtypes = [C.POINTER(SolveOpts)]
    lib.rbf_setup.argtypes = [vp, vp, i64, dbl, dbl, dbl, vp, C.POINTER(vp)]
    lib.rbf_centres.argtypes = [vp, vp, vp, vp]
    lib.rbf_matvec.argtypes = [vp, vp, vp, i32, vp]
    lib.rbf_solve.argtypes = [vp, vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
    lib.rbf_eval_grid.argtypes = [vp, vp, C.POINTER(Grid), vp, i32, vp]
    lib.rbf_eval_points.argtypes = [vp, vp, vp, i64, vp, i32, vp]
    lib.rbf_density.argtypes = [vp, vp, i64, C.POINTER(DensityInfo), vp]
    lib.rbf_arnoldi.argtypes = [vp, vp, i32, i32, i32, vp, C.POINTER(dbl), C.POINTER(i32), vp]
    lib.rbf_eval_grid_noalloc.argtypes = [vp, vp, C.POINTER(Grid), vp, vp]
    lib.rbf_get_stats.argtypes = [vp, C.POINTER(Stats)]
    lib.rbf_count_grid_pairs.argtypes = [vp, C.POINTER(Grid), C.POINTER(i64), C.POINTER(i64), vp]
    lib.rbf_profile_begin.argtypes = []
    lib.rbf_profile_end.argtypes = [C.POINTER(Profile)]
    lib.rbf_measure_rates.argtypes = [C.POINTER(Rates), vp]
    lib.rbf_default_schwarz_opts.argtypes = [C.POINTER(SchwarzOpts)]
    lib.rbf_schwarz_setup.argtypes = [vp, C.POINTER(SchwarzOpts), vp]
    lib.rbf_schwarz_apply.argtypes = [vp, vp, vp, vp]
    lib.rbf_schwarz_get_info.argtypes = [vp, C.POINTER(SchwarzInfo)]
    lib.rbf_schwarz_subdomains.argtypes = [vp, C.POINTER(i64), C.POINTER(C.c_int32), C.POINTER(i64)]
    lib.rbf_net_set.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(dbl), dbl, dbl, vp]
    lib.rbf_net_get.argtypes = [vp, C.POINTER(C.c_float), vp]
    lib.rbf_net_forward.argtypes = [vp, vp, i64, vp, vp]
    lib.rbf_net_gradient.argtypes = [vp, vp, vp, i64, vp, C.POINTER(dbl), vp]
    lib.rbf_net_train.argtypes = [vp, vp, vp, i64, i32, i32, dbl, C.POINTER(dbl), vp]
    lib.rbf_eval_grid_culled.argtypes = [vp, vp, C.POINTER(Grid), vp, dbl, C.POINTER(CullStats), vp]
    lib.rbf_destroy.argtypes = [vp]
    lib.rbf_destroy.restype = None
    lib.rbf_last_error.argtypes = [vp]
    lib.rbf_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("rbf_destroy", "rbf_last_error"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def profile_begin() -> None:
    st = load_library().rbf_profile_begin()
    if st != RBF_OK:
        raise RbfError(st, load_library().rbf_last_error(None).decode())


def profile_end() -> Profile:
    p = Profile()
    st = load_library().rbf_profile_end(C.byref(p))
    if st != RBF_OK:
        raise RbfError(st, load_library().rbf_last_error(None).decode())
    return p


def measure_rates() -> Rates:
    """Issue rates of the device's vector ALU (rbf_measure_rates), on the
    current stream."""
    r = Rates()
    st = load_library().rbf_measure_rates(C.byref(r), _stream())
    if st != RBF_OK:
        raise RbfError(st, load_library().rbf_last_error(None).decode())
    return r


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    load_library().rbf_default_solve_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def make_grid(origin, h, dims) -> Grid:
    g = Grid()
    for d in range(3):
        g.origin[d] = float(origin[d])
        g.h[d] = float(h[d])
        g.dims[d] = int(dims[d])
    return g


@dataclass
class SolveResult:
    status: int
    iters: int
    outer: int
    rel_resid: float
    history: list
    history_ms: list


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype_name: str = "float64", numel: int | None = None, rows3: bool = False, device=None,
         name: str = "tensor"):
    """Device address of a torch tensor after the checks the C side cannot
    make from a raw pointer: a CUDA (HIP) tensor of the given dtype,
    contiguous, on the context's device, with `numel` elements or, with
    rows3, of shape (k, 3)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a CUDA (HIP) torch tensor")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise TypeError(f"{name}: expected dtype {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if device is not None and t.device != device:
        raise ValueError(f"{name}: tensor is on {t.device}, the context on {device}")
    if rows3 and (t.dim() != 2 or t.shape[1] != 3):
        raise ValueError(f"{name}: expected shape (k, 3), got {tuple(t.shape)}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


class Rbf:
    """A context: extended centre set, neighbour structure and solver storage."""

    def __init__(self, points, normals, eps: float, sigma: float, cutoff: float = math.inf):
        lib = load_library()
        self._lib = lib
        self.ctx = C.c_void_p()
        n = int(points.shape[0])
        self.device = points.device
        pp = _ptr(points, rows3=True, name="points")
        pn = _ptr(normals, rows3=True, numel=3 * n, device=self.device, name="normals")
        st = lib.rbf_setup(pp, pn, n, float(eps), float(sigma), float(cutoff), _stream(), C.byref(self.ctx))
        if st != RBF_OK:
            raise RbfError(st, lib.rbf_last_error(None).decode())
        self.n = n
        self.m = 3 * n

    def _check(self, st):
        if st != RBF_OK:
            raise RbfError(st, self._lib.rbf_last_error(self.ctx).decode())

    def _vec(self, t, name, dtype_name="float64", numel=None):
        """Checked address of a length-3n (or `numel`) vector on the context's device."""
        return _ptr(t, dtype_name, numel=self.m if numel is None else numel, device=self.device, name=name)

    def close(self):
        if self.ctx:
            self._lib.rbf_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def centres(self):
        import torch
        X = torch.empty((self.m, 3), dtype=torch.float64, device=self.device)
        b = torch.empty(self.m, dtype=torch.float64, device=self.device)
        self._check(self._lib.rbf_centres(self.ctx, _ptr(X), _ptr(b), _stream()))
        return X, b

    def matvec(self, x, y=None, prec: int = RBF_FP32):
        import torch
        if y is None:
            y = torch.empty_like(x)
        self._check(self._lib.rbf_matvec(self.ctx, self._vec(x, "x"), self._vec(y, "y"), int(prec), _stream()))
        return y

    def solve(self, b=None, x0=None, c=None, **opts) -> tuple:
        import torch
        if c is None:
            c = torch.empty(self.m, dtype=torch.float64, device=self.device)
        o = default_opts(**opts)
        info = SolveInfo()
        st = self._lib.rbf_solve(self.ctx, self._vec(b, "b") if b is not None else None,
                                 self._vec(x0, "x0") if x0 is not None else None, self._vec(c, "c"), C.byref(o),
                                 C.byref(info), _stream())
        if st not in (RBF_OK, RBF_ENOCONV):
            raise RbfError(st, self._lib.rbf_last_error(self.ctx).decode())
        hist = [info.history[i] for i in range(info.n_history)]
        hms = [info.history_ms[i] for i in range(info.n_history)]
        return c, SolveResult(st, info.iters, info.outer, info.rel_resid, hist, hms)

    def eval_grid(self, c, origin, h, dims, prec: int = RBF_FP32, out=None):
        import torch
        g = make_grid(origin, h, dims)
        total = int(dims[0]) * int(dims[1]) * int(dims[2])
        dt = torch.float32 if prec == RBF_FP32 else torch.float64
        if out is None:
            out = torch.empty(total, dtype=dt, device=self.device)
        self._check(self._lib.rbf_eval_grid(self.ctx, self._vec(c, "c"), C.byref(g),
                                            self._vec(out, "out", "float32" if prec == RBF_FP32 else "float64",
                                                      total),
                                            int(prec), _stream()))
        return out

    def eval_points(self, c, pts, prec: int = RBF_FP32, out=None):
        import torch
        k = int(pts.shape[0])
        if out is None:
            out = torch.empty(k, dtype=torch.float64, device=self.device)
        pp = _ptr(pts, rows3=True, device=self.device, name="pts")
        self._check(self._lib.rbf_eval_points(self.ctx, self._vec(c, "c"), pp, k, self._vec(out, "out", numel=k),
                                              int(prec), _stream()))
        return out

    def density(self, samples=None) -> DensityInfo:
        """q, h_max, h_fill (NaN without samples), h and the sigma choices of
        eqs. h1 / h2 for the cloud (rbf_density)."""
        d = DensityInfo()
        ns = 0 if samples is None else int(samples.shape[0])
        ps = _ptr(samples, rows3=True, device=self.device, name="samples") if samples is not None else None
        self._check(self._lib.rbf_density(self.ctx, ps, ns, C.byref(d), _stream()))
        return d

    def arnoldi(self, v0, m: int, op_prec: int = RBF_FP64, basis: int = RBF_FP64):
        """m Arnoldi steps of the solver from v0 (rbf_arnoldi): (V (m+1) x 3n,
        H (m+1) x m as numpy, steps)."""
        import numpy as np
        import torch
        V = torch.empty((m + 1, self.m), dtype=torch.float64, device=self.device)
        H = np.zeros((m + 1) * m, dtype=np.float64)
        k = C.c_int()
        self._check(self._lib.rbf_arnoldi(self.ctx, self._vec(v0, "v0"), int(m), int(op_prec), int(basis),
                                          _ptr(V, device=self.device, name="V"),
                                          H.ctypes.data_as(C.POINTER(C.c_double)), C.byref(k), _stream()))
        return V, H.reshape(m + 1, m), k.value

    def stats(self) -> Stats:
        s = Stats()
        self._check(self._lib.rbf_get_stats(self.ctx, C.byref(s)))
        return s

    def schwarz_setup(self, **opts) -> SchwarzInfo:
        """Build the Schwarz preconditioner (rbf_schwarz_setup); returns its sizes."""
        o = SchwarzOpts()
        self._lib.rbf_default_schwarz_opts(C.byref(o))
        for k, v in opts.items():
            setattr(o, k, v)
        self._check(self._lib.rbf_schwarz_setup(self.ctx, C.byref(o), _stream()))
        return self.schwarz_info()

    def schwarz_info(self) -> SchwarzInfo:
        info = SchwarzInfo()
        self._check(self._lib.rbf_schwarz_get_info(self.ctx, C.byref(info)))
        return info

    def schwarz_apply(self, r, z=None):
        import torch
        if z is None:
            z = torch.empty_like(r)
        self._check(self._lib.rbf_schwarz_apply(self.ctx, self._vec(r, "r"), self._vec(z, "z"), _stream()))
        return z

    def schwarz_subdomains(self) -> list:
        """[(core centres, overlap centres)] as numpy int64 arrays (paper indices)."""
        import numpy as np
        info = self.schwarz_info()
        offs = np.zeros(info.n_sub + 1, dtype=np.int64)
        ncore = np.zeros(max(info.n_sub, 1), dtype=np.int32)
        mem = np.zeros(max(info.n_members, 1), dtype=np.int64)
        self._check(self._lib.rbf_schwarz_subdomains(
            self.ctx, offs.ctypes.data_as(C.POINTER(C.c_int64)), ncore.ctypes.data_as(C.POINTER(C.c_int32)),
            mem.ctypes.data_as(C.POINTER(C.c_int64))))
        out = []
        for i in range(info.n_sub):
            seg = mem[offs[i]:offs[i + 1]]
            out.append((seg[:ncore[i]].copy(), seg[ncore[i]:].copy()))
        return out

    def net_set(self, params, centre, scale: float, tau: float):
        """Install the cull network (params: RBF_NET_PARAMS float32 values, host)."""
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != RBF_NET_PARAMS:
            raise ValueError(f"expected {RBF_NET_PARAMS} parameters")
        c3 = (C.c_double * 3)(*[float(v) for v in centre])
        self._check(self._lib.rbf_net_set(self.ctx, p.ctypes.data_as(C.POINTER(C.c_float)), c3, float(scale),
                                          float(tau), _stream()))

    def net_get(self):
        import numpy as np
        p = np.zeros(RBF_NET_PARAMS, dtype=np.float32)
        self._check(self._lib.rbf_net_get(self.ctx, p.ctypes.data_as(C.POINTER(C.c_float)), _stream()))
        return p

    def net_forward(self, x, y=None):
        import torch
        k = int(x.shape[0])
        if y is None:
            y = torch.empty(k, dtype=torch.float32, device=self.device)
        self._check(self._lib.rbf_net_forward(self.ctx, _ptr(x, rows3=True, device=self.device, name="x"), k,
                                              self._vec(y, "y", "float32", k), _stream()))
        return y

    def net_gradient(self, x, f):
        import torch
        k = int(x.shape[0])
        g = torch.empty(RBF_NET_PARAMS, dtype=torch.float32, device=self.device)
        loss = C.c_double()
        self._check(self._lib.rbf_net_gradient(self.ctx, _ptr(x, rows3=True, device=self.device, name="x"),
                                               self._vec(f, "f", numel=k), k, _ptr(g, "float32"),
                                               C.byref(loss), _stream()))
        return g, loss.value

    def net_train(self, x, f, batch: int, epochs: int, lr: float) -> float:
        k = int(x.shape[0])
        loss = C.c_double()
        self._check(self._lib.rbf_net_train(self.ctx, _ptr(x, rows3=True, device=self.device, name="x"),
                                            self._vec(f, "f", numel=k), k, int(batch), int(epochs),
                                            float(lr), C.byref(loss), _stream()))
        return loss.value

    def eval_grid_culled(self, c, origin, h, dims, e_val: float, out=None):
        import torch
        g = make_grid(origin, h, dims)
        total = int(dims[0]) * int(dims[1]) * int(dims[2])
        if out is None:
            out = torch.empty(total, dtype=torch.float32, device=self.device)
        st = CullStats()
        self._check(self._lib.rbf_eval_grid_culled(self.ctx, self._vec(c, "c"), C.byref(g),
                                                   self._vec(out, "out", "float32", total),
                                                   float(e_val), C.byref(st), _stream()))
        return out, st

    def count_grid_pairs(self, origin, h, dims):
        g = make_grid(origin, h, dims)
        u, e = C.c_int64(), C.c_int64()
        self._check(self._lib.rbf_count_grid_pairs(self.ctx, C.byref(g), C.byref(u), C.byref(e), _stream()))
        return u.value, e.value

