"""Seeded synthetic point clouds and test vectors.

This module only produces inputs: surface points with their outward unit
normals, evaluation-grid descriptors and random vectors.  It contains none of
the reconstruction arithmetic (no off-surface points, no kernel, no solve), so
both the CPU oracle and the GPU path can draw their inputs from it.

The shapes stand in for the paper's workloads (Sec. IV: a scattered sphere
cloud, incomplete and noisy clouds, a scanned model); every generator is
deterministic given its seed (``numpy.random.default_rng``).
"""
from __future__ import annotations

import hashlib
import math
import os
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Cloud:
    """A surface point cloud: ``points`` and outward unit ``normals`` (n x 3, float64)."""

    points: np.ndarray
    normals: np.ndarray
    name: str

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.points).tobytes())
        h.update(np.ascontiguousarray(self.normals).tobytes())
        return h.hexdigest()


@dataclass(frozen=True)
class Grid:
    """Regular evaluation grid: node (i, j, k) = origin + (i, j, k) * h, x fastest."""

    origin: tuple
    h: tuple
    dims: tuple

    @property
    def size(self) -> int:
        return int(self.dims[0]) * int(self.dims[1]) * int(self.dims[2])

    @staticmethod
    def cube(lo: float, hi: float, n: int) -> "Grid":
        """n^3 nodes on [lo, hi]^3 with both end points included."""
        h = (hi - lo) / (n - 1)
        return Grid((lo, lo, lo), (h, h, h), (n, n, n))

    @staticmethod
    def around(points: np.ndarray, n: int, scale: float = 1.2) -> "Grid":
        """n^3 cube centred on the bounding-box centre of ``points``; its
        half side is ``scale`` times the largest half extent of the box."""
        lo = points.min(axis=0)
        hi = points.max(axis=0)
        c = 0.5 * (lo + hi)
        half = scale * 0.5 * float(np.max(hi - lo))
        h = 2.0 * half / (n - 1)
        o = c - half
        return Grid((float(o[0]), float(o[1]), float(o[2])), (h, h, h), (n, n, n))


def sphere(n: int = 2000, seed: int = 0) -> Cloud:
    """Points uniform on the unit sphere (normalised Gaussian samples);
    the outward normal of the unit sphere at p is p itself."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3))
    p = g / np.sqrt(np.sum(g * g, axis=1))[:, None]
    return Cloud(p, p.copy(), f"sphere{n}")


def _torus_rows(s: float, R: float, r: float, rng: np.random.Generator):
    nv = max(3, int(round(2.0 * math.pi * r / s)))
    us, vs = [], []
    for k in range(nv):
        v = 2.0 * math.pi * (k + 0.5) / nv
        m = max(3, int(round(2.0 * math.pi * (R + r * math.cos(v)) / s)))
        ju = rng.uniform(-0.25, 0.25, size=m)
        jvv = rng.uniform(-0.25, 0.25, size=m)
        u = 2.0 * math.pi * (np.arange(m) + 0.5 + ju) / m
        vv = 2.0 * math.pi * (k + 0.5 + jvv) / nv
        us.append(u)
        vs.append(vv)
    return np.concatenate(us), np.concatenate(vs)


def torus(n: int = 200_000, seed: int = 1, R: float = 1.0, r: float = 0.35) -> Cloud:
    """Jittered, roughly even ("Poisson-disk-like") samples of a torus.

    Rows equally spaced in the tube angle v; each row holds points equally
    spaced in the ring angle u at the same arc spacing s; every point is
    jittered by up to a quarter cell in u and v.  s is chosen so the count is
    at least n, then a seeded random subset of exactly n points is kept and
    the order shuffled (a scanner delivers no particular order).
    """
    area = 4.0 * math.pi * math.pi * R * r
    s_hi = math.sqrt(area / n) * 1.05
    s_lo = s_hi * 0.9

    def cnt(s):
        nv = max(3, int(round(2.0 * math.pi * r / s)))
        return sum(max(3, int(round(2.0 * math.pi * (R + r * math.cos(2.0 * math.pi * (k + 0.5) / nv)) / s)))
                   for k in range(nv))

    while cnt(s_lo) < n:
        s_lo *= 0.98
    for _ in range(60):
        mid = 0.5 * (s_lo + s_hi)
        if cnt(mid) >= n:
            s_lo = mid
        else:
            s_hi = mid
    rng = np.random.default_rng(seed)
    u, v = _torus_rows(s_lo, R, r, rng)
    keep = np.sort(rng.choice(u.size, size=n, replace=False))
    u, v = u[keep], v[keep]
    order = rng.permutation(n)
    u, v = u[order], v[order]
    cu, su, cv, sv = np.cos(u), np.sin(u), np.cos(v), np.sin(v)
    p = np.stack([(R + r * cv) * cu, (R + r * cv) * su, r * sv], axis=1)
    nrm = np.stack([cv * cu, cv * su, sv], axis=1)
    return Cloud(p, nrm, f"torus{n}")


def torus_sdf(q: np.ndarray, R: float = 1.0, r: float = 0.35) -> np.ndarray:
    """Signed distance to the torus (positive outside)."""
    rho = np.sqrt(q[:, 0] ** 2 + q[:, 1] ** 2)
    return np.sqrt((rho - R) ** 2 + q[:, 2] ** 2) - r


def sphere_sdf(q: np.ndarray) -> np.ndarray:
    """Signed distance to the unit sphere (positive outside)."""
    return np.sqrt(np.sum(q * q, axis=1)) - 1.0


def _metaball_field(x: np.ndarray, c: np.ndarray, s: np.ndarray):
    """F(x) = sum_k exp(-|x - c_k|^2 / (2 s_k^2)) - 1/2 and its gradient."""
    F = np.full(x.shape[0], -0.5)
    G = np.zeros_like(x)
    for ck, sk in zip(c, s):
        d = x - ck
        e = np.exp(-np.sum(d * d, axis=1) / (2.0 * sk * sk))
        F += e
        G -= (e / (sk * sk))[:, None] * d
    return F, G


def _metaball_field_threads(x: np.ndarray, c: np.ndarray, s: np.ndarray, parts: int = 16):
    """_metaball_field over row blocks of x on a thread pool.  Every row's
    values depend on that row alone, so the result is the same, bit for bit,
    as one call over all of x."""
    if x.shape[0] < 65536:
        return _metaball_field(x, c, s)
    from concurrent.futures import ThreadPoolExecutor
    blocks = np.array_split(np.arange(x.shape[0]), parts)
    with ThreadPoolExecutor(max_workers=min(parts, os.cpu_count() or 1)) as ex:
        res = list(ex.map(lambda ix: _metaball_field(x[ix[0]:ix[-1] + 1], c, s), blocks))
    return np.concatenate([r[0] for r in res]), np.concatenate([r[1] for r in res])


def metaballs(n: int = 2_000_000, seed: int = 2, k: int = 12, band: float = 0.1, hole: float = 0.15,
              noise: float = 1e-3, batch: int = 4_000_000) -> Cloud:
    """An incomplete, noisy scan-like cloud: the zero set of a sum of k
    seeded Gaussian metaballs (centres U[-0.5, 0.5]^3, widths U(0.15, 0.30),
    level 1/2).  Candidates uniform in the box with |F| < band are projected
    onto the surface by three Newton steps x <- x - F grad F / |grad F|^2;
    the outward normal is -grad F / |grad F| at the projected point; points
    within `hole` of the first projected point are removed; exactly n are
    kept (in generation order) and N(0, noise^2) is added to each coordinate."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-0.5, 0.5, size=(k, 3))
    s = rng.uniform(0.15, 0.30, size=k)
    lo = c.min(axis=0) - 3.0 * s.max()
    hi = c.max(axis=0) + 3.0 * s.max()
    pts, nrm = [], []
    have = 0
    first = None
    while have < n:
        x = rng.uniform(lo, hi, size=(batch, 3))
        F, _ = _metaball_field_threads(x, c, s)
        x = x[np.abs(F) < band]
        for _ in range(3):
            F, G = _metaball_field_threads(x, c, s)
            x = x - (F / np.sum(G * G, axis=1))[:, None] * G
        F, G = _metaball_field_threads(x, c, s)
        g = np.sqrt(np.sum(G * G, axis=1))
        ok = (np.abs(F) < 1e-9) & (g > 1e-6)
        x, G, g = x[ok], G[ok], g[ok]
        if first is None and x.shape[0]:
            first = x[0].copy()
        keep = np.sum((x - first) ** 2, axis=1) > hole * hole
        x, G, g = x[keep], G[keep], g[keep]
        pts.append(x)
        nrm.append(-G / g[:, None])
        have += x.shape[0]
    p = np.concatenate(pts)[:n]
    q = np.concatenate(nrm)[:n]
    p = p + rng.normal(0.0, noise, size=p.shape)
    return Cloud(p, q, f"metaballs{n}")


def patch(cloud: Cloud, n: int, seed: int = 5) -> Cloud:
    """The n points of ``cloud`` nearest to one of its points chosen at
    random: a compact piece at the cloud's own density."""
    rng = np.random.default_rng(seed)
    c = cloud.points[rng.integers(cloud.n)]
    d = np.sum((cloud.points - c) ** 2, axis=1)
    idx = np.sort(np.argsort(d, kind="stable")[:n])
    return Cloud(cloud.points[idx].copy(), cloud.normals[idx].copy(), f"{cloud.name}_patch{n}")


def random_vector(m: int, seed: int = 4) -> np.ndarray:
    """x_j ~ U(-1, 1): the input vector used to time and check the operator."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=m)


def lattice_cloud(nx: int, ny: int, spacing: float, seed: int = 6, jitter: float = 0.0) -> Cloud:
    """A flat nx x ny patch of the plane z = 0 with normal +z, optionally
    jittered in-plane: a small well-separated test cloud."""
    rng = np.random.default_rng(seed)
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    p = np.zeros((nx * ny, 3))
    p[:, 0] = ii.ravel() * spacing
    p[:, 1] = jj.ravel() * spacing
    if jitter > 0:
        p[:, :2] += rng.uniform(-jitter, jitter, size=(nx * ny, 2)) * spacing
    nrm = np.zeros_like(p)
    nrm[:, 2] = 1.0
    return Cloud(p, nrm, f"plane{nx}x{ny}")


def net_init(seed: int = 8, width: int = 128, layers: int = 4) -> np.ndarray:
    """Initial parameters of the cull network, flat float32 in the library's
    order (W1, b1, W2, b2, W3, b3, W4, b4, w5, b5; W[out][in]): every entry
    uniform in +-1/sqrt(fan_in) of its layer."""
    rng = np.random.default_rng(seed)
    sizes = [3] + [width] * layers + [1]
    out = []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        a = 1.0 / math.sqrt(fan_in)
        out.append(rng.uniform(-a, a, size=fan_out * fan_in))
        out.append(rng.uniform(-a, a, size=fan_out))
    return np.concatenate(out).astype(np.float32)


def net_unflatten(flat: np.ndarray, width: int = 128, layers: int = 4):
    """[(W, b)] views of a flat parameter vector (float64 copies)."""
    sizes = [3] + [width] * layers + [1]
    out, o = [], 0
    flat = np.asarray(flat, dtype=np.float64)
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        W = flat[o:o + fan_out * fan_in].reshape(fan_out, fan_in)
        o += fan_out * fan_in
        b = flat[o:o + fan_out]
        o += fan_out
        out.append((W.copy(), b.copy()))
    return out


def band_samples(points: np.ndarray, radius: float, n: int, seed: int = 3) -> np.ndarray:
    """n positions in the support band: a random cloud point plus a uniform
    offset in the ball of `radius`."""
    rng = np.random.default_rng(seed)
    base = points[rng.integers(0, len(points), n)]
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    r = radius * rng.uniform(size=n) ** (1.0 / 3.0)
    return base + d * r[:, None]


def cull_samples(points: np.ndarray, radius: float, lo, hi, n: int, seed: int = 3) -> np.ndarray:
    """Training positions of the cull network: half of them a random cloud
    point plus a uniform offset in the ball of `radius` (the support of the
    truncated interpolant), half uniform in the box [lo, hi]; shuffled."""
    rng = np.random.default_rng(seed)
    n_band = n // 2
    base = points[rng.integers(0, len(points), n_band)]
    d = rng.normal(size=(n_band, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    r = radius * rng.uniform(size=n_band) ** (1.0 / 3.0)
    band = base + d * r[:, None]
    box = rng.uniform(np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64), size=(n - n_band, 3))
    X = np.concatenate([band, box])
    return X[rng.permutation(n)]


def halton(n: int, base: int, start: int = 1) -> np.ndarray:
    """Radical-inverse (van der Corput) sequence in ``base``, indices start..start+n-1."""
    out = np.empty(n)
    for t in range(n):
        i, f, x = start + t, 1.0, 0.0
        while i > 0:
            f /= base
            x += f * (i % base)
            i //= base
        out[t] = x
    return out


# Named workloads (the solve/evaluation parameters that go with each cloud).
SPHERE_SMALL = dict(n=2000, seed=0, eps=0.01, sigma=0.05, cutoff=math.inf,
                    grid=lambda: Grid.cube(-1.2, 1.2, 32))
TORUS_200K = dict(n=200_000, seed=1, eps=0.005, sigma=0.02, cutoff=0.08, restart=30,
                  grid_n=256, R=1.0, r=0.35)
# The offset is not given for this cloud: eps = sigma / 4 keeps the torus
# workload's ratio and stays above 2.5 times the noise.
METABALLS_2M = dict(n=2_000_000, seed=2, eps=0.0025, sigma=0.01, cutoff=0.04, restart=30,
                    grid_n=512)
