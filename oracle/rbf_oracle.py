"""CPU oracle for Gaussian-RBF implicit surface reconstruction (FP64).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The GPU library
never calls it, links it or shares code with it.

Every function is the plain definition of what the paper computes, written in
float64 with numpy, in the paper's notation, with no blocking, fusion or
reordering beyond what the definition states.  Library routines serve as
steps where noted (LAPACK ``gesv`` through ``numpy.linalg.solve``).

Paper: Cuomo, Galletti, Giunta, Starace, "Surface Reconstruction from
Scattered Point via RBF Interpolation on GPU" (arXiv 1305.5179).

Readings taken where the paper is silent or inconsistent (each listed with
its justification in the design notes):
  * Kernel: phi(r) = exp(-r^2 / (2 sigma^2)).  The paper's Table I and the
    matrix-entry equation of Sec. III.A carry a 1/(sqrt(2 pi) sigma) factor;
    any constant factor alpha used consistently leaves the interpolant f
    unchanged (the weights scale by 1/alpha), so it is dropped.
  * Off-surface values: 0 on the cloud, +v outside, -v inside (Sec. II.A.2
    uses v = 1 and calls the magnitude arbitrary).  By linearity the weights
    scale with v; the default is v = delta, so f approximates a signed
    distance near the surface.
  * Truncation (Sec. III.A, the finite-bandwidth remark after the
    matrix-entry equation): entries with r^2 > r_c^2 are neglected; the test
    is inclusive, r^2 <= r_c^2, decided in float64 with
    r^2 = (dx*dx + dy*dy) + dz*dz.  r_c = inf means no truncation.
  * Evaluation (Sec. II.B, the evaluation matrix-vector product) uses the same
    truncation, so that f(x_i) = (A c)_i holds exactly at the centres.
  * Normals are normalised here: n_hat = n / sqrt((nx*nx + ny*ny) + nz*nz).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "unit_normals", "extended_centres", "phi", "sqdist", "interpolation_matrix",
    "matvec", "matvec_rows", "solve_direct", "evaluate", "grid_nodes", "evaluate_grid",
    "gmres", "GmresResult", "relative_residual", "separation_distance",
    "fill_distance", "h_max", "interpolant_sign_check",
]


# ---------------------------------------------------------------------------
# Step 1 of the reconstruction algorithm (Alg. 1): the extended data set.
# ---------------------------------------------------------------------------
def unit_normals(normals: np.ndarray) -> np.ndarray:
    """Oriented unit normals n_hat_i = n_i / |n_i| (Sec. II.A.1 marches along
    the normals; the step length is delta only for unit normals)."""
    n = np.asarray(normals, dtype=np.float64)
    s = (n[:, 0] * n[:, 0] + n[:, 1] * n[:, 1]) + n[:, 2] * n[:, 2]
    norm = np.sqrt(s)
    return n / norm[:, None]


def extended_centres(points: np.ndarray, normals: np.ndarray, delta: float,
                     value: float | None = None):
    """Extended set X_ext = X u X_delta^+ u X_delta^- and its data values
    (Sec. II.A.1 and II.A.2).

    Centre i is the point x_i, centre N+i is x_i + delta*n_i ("outside"),
    centre 2N+i is x_i - delta*n_i ("inside").  The values are 0 on the cloud,
    +value outside and -value inside (value defaults to delta).
    Returns (X, b) with X of shape (3N, 3) and b of length 3N.
    """
    p = np.asarray(points, dtype=np.float64)
    nh = unit_normals(normals)
    outside = p + delta * nh
    inside = p - delta * nh
    X = np.concatenate([p, outside, inside], axis=0)
    v = delta if value is None else value
    n = p.shape[0]
    b = np.concatenate([np.zeros(n), np.full(n, v), np.full(n, -v)])
    return X, b


# ---------------------------------------------------------------------------
# The Gaussian kernel and the interpolation operator (Sec. II.B, eq. RBFsys;
# Sec. III.A, eq. matrixEntries with the truncation remark).
# ---------------------------------------------------------------------------
def phi(r2, sigma: float):
    """Gaussian radial function of the squared distance: exp(-r^2 / (2 sigma^2))."""
    return np.exp(-np.asarray(r2, dtype=np.float64) / (2.0 * sigma * sigma))


def sqdist(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Squared distances between the rows of ``a`` (m x 3) and ``b`` (n x 3),
    each as (dx*dx + dy*dy) + dz*dz with dx = a_x - b_x."""
    dx = a[:, None, 0] - b[None, :, 0]
    dy = a[:, None, 1] - b[None, :, 1]
    dz = a[:, None, 2] - b[None, :, 2]
    return (dx * dx + dy * dy) + dz * dz


def _kernel_block(a: np.ndarray, b: np.ndarray, sigma: float, cutoff: float) -> np.ndarray:
    r2 = sqdist(a, b)
    k = phi(r2, sigma)
    if math.isfinite(cutoff):
        k = np.where(r2 <= cutoff * cutoff, k, 0.0)
    return k


def interpolation_matrix(X: np.ndarray, sigma: float, cutoff: float = math.inf) -> np.ndarray:
    """Dense A with A_ij = phi(|x_i - x_j|), truncated at r_c (small N only)."""
    return _kernel_block(X, X, sigma, cutoff)


def matvec_rows(X: np.ndarray, x: np.ndarray, rows, sigma: float,
                cutoff: float = math.inf) -> np.ndarray:
    """(A x)_i for the listed rows i, each summed over all j in index order.
    Brute force: O(len(rows) * 3N) work, so it serves any N for sampled rows."""
    rows = np.asarray(rows, dtype=np.int64)
    out = np.empty(rows.size)
    for t, i in enumerate(rows):
        k = _kernel_block(X[i:i + 1], X, sigma, cutoff)[0]
        out[t] = np.dot(k, x)
    return out


def matvec(X: np.ndarray, x: np.ndarray, sigma: float, cutoff: float = math.inf,
           rows_per_block: int = 256) -> np.ndarray:
    """y = A x for every row (row blocks only bound the memory used)."""
    m = X.shape[0]
    y = np.empty(m)
    for s in range(0, m, rows_per_block):
        k = _kernel_block(X[s:s + rows_per_block], X, sigma, cutoff)
        y[s:s + rows_per_block] = k @ x
    return y


def solve_direct(X: np.ndarray, b: np.ndarray, sigma: float, cutoff: float = math.inf):
    """Weights c with A c = b by LU with partial pivoting (LAPACK gesv).
    Returns (c, relative residual |A c - b| / |b|)."""
    A = interpolation_matrix(X, sigma, cutoff)
    c = np.linalg.solve(A, b)
    return c, float(np.linalg.norm(A @ c - b) / np.linalg.norm(b))


def relative_residual(X, c, b, sigma, cutoff=math.inf) -> float:
    """|b - A c|_2 / |b|_2 with the float64 truncated operator."""
    r = b - matvec(X, c, sigma, cutoff)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


# ---------------------------------------------------------------------------
# Step 3 of Alg. 1: evaluation of the interpolant (Sec. II.B, eq. matxvet).
# ---------------------------------------------------------------------------
def evaluate(X: np.ndarray, c: np.ndarray, pts: np.ndarray, sigma: float,
             cutoff: float = math.inf, rows_per_block: int = 256) -> np.ndarray:
    """P_f(xi_m) = sum_j c_j phi(|xi_m - x_j|) for every evaluation point."""
    pts = np.asarray(pts, dtype=np.float64)
    out = np.empty(pts.shape[0])
    for s in range(0, pts.shape[0], rows_per_block):
        k = _kernel_block(pts[s:s + rows_per_block], X, sigma, cutoff)
        out[s:s + rows_per_block] = k @ c
    return out


def grid_nodes(origin, h, dims, index=None) -> np.ndarray:
    """Coordinates of grid nodes xi_(i,j,k) = origin + (i, j, k) * h, listed
    with i fastest (linear index i + nx*(j + ny*k)); ``index`` selects nodes."""
    nx, ny, nz = (int(d) for d in dims)
    if index is None:
        index = np.arange(nx * ny * nz, dtype=np.int64)
    index = np.asarray(index, dtype=np.int64)
    i = index % nx
    j = (index // nx) % ny
    k = index // (nx * ny)
    return np.stack([origin[0] + i * h[0], origin[1] + j * h[1], origin[2] + k * h[2]], axis=1)


def evaluate_grid(X, c, origin, h, dims, sigma, cutoff=math.inf, index=None) -> np.ndarray:
    """f on the grid nodes (all of them, or the selected linear indices)."""
    return evaluate(X, c, grid_nodes(origin, h, dims, index), sigma, cutoff)


# ---------------------------------------------------------------------------
# GMRES(m), the Krylov method the paper uses for A x = b (Sec. III.A).
# Arnoldi with modified Gram-Schmidt, Givens rotations on the Hessenberg
# matrix, restart after m steps (Saad and Schultz's GMRES).
# ---------------------------------------------------------------------------
@dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    rel_resid: float
    converged: bool
    history: list = field(default_factory=list)   # true relative residual at each restart
    estimates: list = field(default_factory=list)  # |g_{j+1}| / |b| after each step


def gmres(apply_A, b: np.ndarray, x0: np.ndarray | None = None, restart: int = 30,
          max_iters: int = 1000, tol: float = 1e-8, apply_M=None) -> GmresResult:
    """Restarted GMRES.  Stops when the relative residual (the rotated
    right-hand side's last entry inside a cycle, the true residual at a
    restart) is <= tol, or after max_iters operator applications inside
    cycles.  With apply_M, right preconditioning (Sec. III.A uses the
    Schwarz solves as a preconditioner of GMRES): the cycle builds its basis
    on A M, and the correction is M V y."""
    if apply_M is None:
        apply_M = lambda v: v  # noqa: E731
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    res = GmresResult(x=x, iters=0, rel_resid=math.nan, converged=False)
    if bnorm == 0.0:
        res.x[:] = 0.0
        res.rel_resid = 0.0
        res.converged = True
        return res
    m = restart
    while True:
        r = b - apply_A(x)
        beta = float(np.linalg.norm(r))
        res.rel_resid = beta / bnorm
        res.history.append(res.rel_resid)
        if res.rel_resid <= tol:
            res.converged = True
            break
        if res.iters >= max_iters:
            break
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            w = apply_A(apply_M(V[j]))
            res.iters += 1
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            for i in range(j):
                a, bb = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * bb
                H[i + 1, j] = -sn[i] * a + cs[i] * bb
            a, bb = H[j, j], H[j + 1, j]
            rho = math.hypot(a, bb)
            cs[j], sn[j] = (1.0, 0.0) if rho == 0.0 else (a / rho, bb / rho)
            H[j, j] = rho
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            res.estimates.append(abs(g[j + 1]) / bnorm)
            breakdown = H[j, j] == 0.0
            hnext = float(np.linalg.norm(w))
            if hnext > 0.0:
                V[j + 1] = w / hnext
            if abs(g[j + 1]) / bnorm <= tol or res.iters >= max_iters or hnext == 0.0 or breakdown:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        x = x + apply_M(V[:k].T @ y)
        res.x = x
    res.x = x
    return res


# ---------------------------------------------------------------------------
# Density measures and sigma heuristics (Sec. IV: eqs. sepDist, fillDist,
# h1, h2, hmax).
# ---------------------------------------------------------------------------
def separation_distance(P: np.ndarray) -> float:
    """q_X = 1/2 min_{i != j} |x_i - x_j| (brute force over all pairs)."""
    best = math.inf
    for s in range(0, P.shape[0], 512):
        d = sqdist(P[s:s + 512], P)
        rows = np.arange(s, min(s + 512, P.shape[0]))
        d[np.arange(rows.size), rows] = math.inf
        best = min(best, float(d.min()))
    return 0.5 * math.sqrt(best)


def fill_distance(P: np.ndarray, samples: np.ndarray) -> float:
    """h_{X,Omega} = sup_{x in Omega} min_j |x - x_j|, the sup taken over the
    given sample of Omega."""
    best = 0.0
    for s in range(0, samples.shape[0], 512):
        d = sqdist(samples[s:s + 512], P)
        best = max(best, float(np.sqrt(d.min(axis=1)).max()))
    return best


def h_max(P: np.ndarray) -> float:
    """h_max = max_j min_{i != j} |x_i - x_j| (Sec. IV.B)."""
    best = 0.0
    for s in range(0, P.shape[0], 512):
        d = sqdist(P[s:s + 512], P)
        rows = np.arange(s, min(s + 512, P.shape[0]))
        d[np.arange(rows.size), rows] = math.inf
        best = max(best, float(np.sqrt(d.min(axis=1)).max()))
    return best


def interpolant_sign_check(f: np.ndarray, sdf: np.ndarray, tau: float):
    """Sign agreement between f and a signed distance on the nodes where
    |f| > tau; returns (agreeing, counted)."""
    m = np.abs(f) > tau
    return int(np.count_nonzero(np.sign(f[m]) == np.sign(sdf[m]))), int(np.count_nonzero(m))
