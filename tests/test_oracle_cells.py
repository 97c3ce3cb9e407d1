"""Pins of the C cell-list oracle (oracle/cellsum.c): closed forms, the
operator's invariants (symmetry, unit diagonal, the inclusive truncation
boundary, pair counts) and agreement with the numpy oracle's dense
definitions, itself pinned in test_oracle_pins.py.  No GPU."""
import math

import numpy as np
import pytest

from oracle import rbf_oracle as o
from oracle.cells import CellOracle
from paper_1305_5179_amd import workloads as w


def abs_scale(X, x, sigma, cutoff, T=None):
    """sum_j |A_ij x_j| per row (dense, numpy)."""
    T = X if T is None else T
    r2 = o.sqdist(T, X)
    K = o.phi(r2, sigma)
    if math.isfinite(cutoff):
        K = np.where(r2 <= cutoff * cutoff, K, 0.0)
    return K @ np.abs(x)


CASES = [
    ("sphere_cut", lambda: w.sphere(333, seed=7), 0.02, 0.15, 0.45),
    ("sphere_dense", lambda: w.sphere(200, seed=3), 0.02, 0.2, math.inf),
    ("torus_patch", lambda: w.patch(w.torus(20000, seed=1), 700, seed=3), 0.005, 0.02, 0.08),
    # every centre in one plane: one cell layer along z
    ("planar", lambda: w.lattice_cloud(9, 7, 0.05, jitter=0.3), 0.0, 0.04, 0.12),
]


@pytest.mark.parametrize("name,make,eps,sigma,rc", CASES, ids=[c[0] for c in CASES])
def test_matvec_equals_dense_oracle(name, make, eps, sigma, rc):
    c = make()
    if eps > 0:
        X, _ = o.extended_centres(c.points, c.normals, eps)
    else:
        X = c.points
    x = w.random_vector(X.shape[0], seed=4)
    ref = o.matvec(X, x, sigma, rc)
    L = CellOracle(X, rc)
    y = L.matvec_rows(x, sigma, threads=2)
    A = o.interpolation_matrix(X, sigma, rc)
    assert L.useful == np.count_nonzero(A)
    assert L.examined >= L.useful
    assert L.count(threads=3) == np.count_nonzero(A)
    assert L.count(rows=[0, 5]) == np.count_nonzero(A[[0, 5]])
    assert np.all(np.abs(y - ref) <= 1e-14 * abs_scale(X, x, sigma, rc) + 1e-300)
    # a subset of rows, in any order, equals those rows
    rows = np.random.default_rng(5).permutation(X.shape[0])[:37]
    assert np.array_equal(L.matvec_rows(x, sigma, rows=rows), y[rows])


def test_two_point_closed_form():
    """Two centres at distance d with phi(d) = 1/2: y = (x0 + x1/2, x0/2 + x1);
    beyond the cutoff the off-diagonal term is absent."""
    sigma = 0.1
    d = sigma * math.sqrt(2.0 * math.log(2.0))
    X = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
    x = np.array([3.0, -5.0])
    y = CellOracle(X, 1.0).matvec_rows(x, sigma)
    assert y == pytest.approx([3.0 - 2.5, 1.5 - 5.0], rel=0, abs=4e-16)
    y = CellOracle(X, 0.5 * d).matvec_rows(x, sigma)
    assert np.array_equal(y, x)


def test_truncation_is_inclusive_at_the_cutoff():
    """r^2 = r_c^2 exactly is kept; the next float64 beyond it is not."""
    rc = 0.5
    sigma = 0.25
    X = np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [0.0, np.nextafter(0.5, 1.0), 0.0]])
    x = np.array([0.0, 1.0, 1.0])
    L = CellOracle(X, rc)
    y = L.matvec_rows(x, sigma, rows=[0])
    assert y[0] == math.exp(-0.25 / (2 * sigma * sigma))
    assert L.useful == 2    # (0, 0) and (0, 1)


def test_symmetry_and_unit_diagonal():
    c = w.patch(w.torus(20000, seed=1), 400, seed=8)
    X, _ = o.extended_centres(c.points, c.normals, 0.005)
    L = CellOracle(X, 0.08)
    a, b = w.random_vector(X.shape[0], seed=1), w.random_vector(X.shape[0], seed=2)
    Aa, Ab = L.matvec_rows(a, 0.02), L.matvec_rows(b, 0.02)
    assert abs(b @ Aa - a @ Ab) <= 1e-13 * (np.abs(b) @ np.abs(Aa) + np.abs(a) @ np.abs(Ab))
    for i in (0, 17, X.shape[0] - 1):
        e = np.zeros(X.shape[0])
        e[i] = 1.0
        assert L.matvec_rows(e, 0.02, rows=[i])[0] == 1.0


def test_evaluation_equals_dense_oracle():
    c = w.sphere(333, seed=7)
    X, _ = o.extended_centres(c.points, c.normals, 0.02)
    coef = w.random_vector(X.shape[0], seed=6)
    rng = np.random.default_rng(9)
    pts = np.concatenate([rng.uniform(-1.3, 1.3, (400, 3)),
                          np.array([[5.0, 5.0, 5.0], [-3.0, 0.0, 0.0]]),   # far outside: exactly 0
                          X[:5]])                                             # at centres: f = (A c)_i
    for rc in (0.45, math.inf):
        L = CellOracle(X, rc)
        f = L.evaluate(coef, pts, 0.15, threads=3)
        ref = o.evaluate(X, coef, pts, 0.15, rc)
        assert np.all(np.abs(f - ref) <= 1e-14 * abs_scale(X, coef, 0.15, rc, pts) + 1e-300)
        if math.isfinite(rc):
            assert f[400] == 0.0 and f[401] == 0.0
        assert np.array_equal(f[-5:], L.matvec_rows(coef, 0.15, rows=np.arange(5)))


def test_thread_count_does_not_change_the_sums():
    c = w.patch(w.torus(20000, seed=1), 900, seed=3)
    X, _ = o.extended_centres(c.points, c.normals, 0.005)
    x = w.random_vector(X.shape[0], seed=4)
    L = CellOracle(X, 0.08)
    assert np.array_equal(L.matvec_rows(x, 0.02, threads=1), L.matvec_rows(x, 0.02, threads=5))
