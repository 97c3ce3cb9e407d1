"""The oracle's pins must catch plausible mistakes.  Each case plants one
mistake in the oracle (on the CPU, by replacing one function of the module)
and runs the pin tests; at least one of them must fail."""
import math

import numpy as np
import pytest

from oracle import rbf_oracle as o
import tests.test_oracle_pins as pins

PIN_TESTS = [
    pins.test_extended_set_worked_example,
    pins.test_extended_set_default_values_are_plus_minus_delta,
    pins.test_unit_normals_normalise_every_row,
    pins.test_phi_closed_forms,
    lambda: [pins.test_two_point_operator_along_each_axis(a) for a in range(3)],
    pins.test_cutoff_is_inclusive_and_exact,
    pins.test_operator_symmetric_unit_diagonal_positive_semidefinite,
    pins.test_single_triple_closed_form,
    pins.test_interpolation_conditions_hold,
    pins.test_evaluate_closed_form,
    pins.test_grid_layout_x_fastest_and_endpoints,
    pins.test_gmres_attains_the_krylov_minimum,
    pins.test_gmres_reaches_the_direct_solution_and_never_increases_the_residual,
    pins.test_halton_separation_and_fill_distance_match_the_paper,
    pins.test_density_measures_on_a_lattice,
]


def _phi_no_two(r2, sigma):
    return np.exp(-np.asarray(r2, dtype=np.float64) / (sigma * sigma))


def _sqdist_no_z(a, b):
    dx = a[:, None, 0] - b[None, :, 0]
    dy = a[:, None, 1] - b[None, :, 1]
    return dx * dx + dy * dy


def _sqdist_sign(a, b):
    dx = a[:, None, 0] + b[None, :, 0]
    dy = a[:, None, 1] - b[None, :, 1]
    dz = a[:, None, 2] - b[None, :, 2]
    return (dx * dx + dy * dy) + dz * dz


_orig_centres = o.extended_centres


def _centres_swapped(points, normals, delta, value=None):
    X, b = _orig_centres(points, normals, delta, value)
    n = points.shape[0]
    X = np.concatenate([X[:n], X[2 * n:], X[n:2 * n]])
    return X, b


def _centres_unnormalised(points, normals, delta, value=None):
    p = np.asarray(points, dtype=np.float64)
    nrm = np.asarray(normals, dtype=np.float64)
    X = np.concatenate([p, p + delta * nrm, p - delta * nrm])
    v = delta if value is None else value
    n = p.shape[0]
    return X, np.concatenate([np.zeros(n), np.full(n, v), np.full(n, -v)])


def _kernel_block_strict(a, b, sigma, cutoff):
    r2 = o.sqdist(a, b)
    k = o.phi(r2, sigma)
    if math.isfinite(cutoff):
        k = np.where(r2 < cutoff * cutoff, k, 0.0)
    return k


def _grid_nodes_y_fastest(origin, h, dims, index=None):
    nx, ny, nz = (int(d) for d in dims)
    if index is None:
        index = np.arange(nx * ny * nz, dtype=np.int64)
    index = np.asarray(index, dtype=np.int64)
    j = index % ny
    i = (index // ny) % nx
    k = index // (nx * ny)
    return np.stack([origin[0] + i * h[0], origin[1] + j * h[1], origin[2] + k * h[2]], axis=1)


def _evaluate_transposed_weights(X, c, pts, sigma, cutoff=math.inf, rows_per_block=256):
    return o.__dict__["_orig_evaluate"](X, c[::-1].copy(), pts, sigma, cutoff, rows_per_block)


def _gmres_variant(old, new):
    """GMRES of the oracle with one source line changed."""
    import inspect
    import textwrap
    src = textwrap.dedent(inspect.getsource(o.__dict__["_orig_gmres"]))
    assert old in src
    ns = dict(o.__dict__)
    exec(compile(src.replace(old, new), "<mutated gmres>", "exec"), ns)
    return ns["gmres"]


def _gmres_rotation_sign(*a, **k):
    return _gmres_variant("H[i + 1, j] = -sn[i] * a + cs[i] * b", "H[i + 1, j] = sn[i] * a + cs[i] * b")(*a, **k)


def _gmres_orthogonalisation_sign(*a, **k):
    return _gmres_variant("w = w - H[i, j] * V[i]", "w = w + H[i, j] * V[i]")(*a, **k)


def _gmres_residual_update(*a, **k):
    return _gmres_variant("g[j + 1] = -sn[j] * g[j]", "g[j + 1] = sn[j] * g[j]")(*a, **k)


def _gmres_back_substitution(*a, **k):
    return _gmres_variant("y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]",
                          "y[i] = (g[i] + np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]")(*a, **k)


MUTATIONS = {
    "phi without the factor 2": ("phi", _phi_no_two),
    "distance without z": ("sqdist", _sqdist_no_z),
    "distance with a sign error": ("sqdist", _sqdist_sign),
    "outside and inside swapped": ("extended_centres", _centres_swapped),
    "normals not normalised": ("extended_centres", _centres_unnormalised),
    "strict cutoff": ("_kernel_block", _kernel_block_strict),
    "grid y fastest": ("grid_nodes", _grid_nodes_y_fastest),
    "weights reversed in evaluation": ("evaluate", _evaluate_transposed_weights),
    "GMRES: old rotations applied with a wrong sign": ("gmres", _gmres_rotation_sign),
    "GMRES: projection added instead of subtracted": ("gmres", _gmres_orthogonalisation_sign),
    "GMRES: residual estimate with a wrong sign": ("gmres", _gmres_residual_update),
    "GMRES: back substitution with a wrong sign": ("gmres", _gmres_back_substitution),
}


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_pins_catch_planted_mistake(name, monkeypatch):
    attr, fake = MUTATIONS[name]
    monkeypatch.setitem(o.__dict__, "_orig_evaluate", o.evaluate)
    monkeypatch.setitem(o.__dict__, "_orig_gmres", o.gmres)
    monkeypatch.setattr(o, attr, fake)
    caught = []
    for t in PIN_TESTS:
        try:
            t()
        except Exception as e:   # an assertion or a numerical failure
            caught.append((getattr(t, "__name__", "lambda"), type(e).__name__))
    assert caught, f"no pin caught: {name}"
