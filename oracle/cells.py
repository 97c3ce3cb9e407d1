"""ctypes wrapper of the C cell-list oracle (cellsum.c): the truncated
Gaussian operator rows and the interpolant at points, float64, on any number
of host threads.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It computes the same
definitions as ``rbf_oracle.matvec_rows`` / ``rbf_oracle.evaluate`` (Sec. II.B
eqs. RBFsys and matxvet, Sec. III.A eq. matrixEntries), in time proportional
to the pairs within one cell of each query rather than to all pairs; the
tests pin it to those functions.  Build it with ``python -m oracle.build``.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle_cells.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m oracle.build`")
        lib = C.CDLL(LIB_PATH)
        vp, i64, dbl, i32 = C.c_void_p, C.c_int64, C.c_double, C.c_int
        lib.oracle_cells_new.argtypes = [vp, i64, dbl]
        lib.oracle_cells_new.restype = vp
        lib.oracle_cells_free.argtypes = [vp]
        lib.oracle_cells_free.restype = None
        lib.oracle_cells_matvec.argtypes = [vp, vp, dbl, vp, i64, vp, i32, C.POINTER(i64), C.POINTER(i64)]
        lib.oracle_cells_matvec.restype = None
        lib.oracle_cells_eval.argtypes = [vp, vp, dbl, vp, i64, vp, i32, C.POINTER(i64), C.POINTER(i64)]
        lib.oracle_cells_eval.restype = None
        lib.oracle_cells_count.argtypes = [vp, vp, i64, i32]
        lib.oracle_cells_count.restype = i64
        lib.oracle_cells_max_threads.argtypes = []
        lib.oracle_cells_max_threads.restype = i32
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().oracle_cells_max_threads())


class CellOracle:
    """The centres X (m x 3) bucketed by cells of side >= cutoff."""

    def __init__(self, X: np.ndarray, cutoff: float = math.inf):
        lib = _load()
        self.X = np.ascontiguousarray(X, dtype=np.float64)
        self.m = self.X.shape[0]
        self._h = lib.oracle_cells_new(self.X.ctypes.data, self.m, float(cutoff))
        if not self._h:
            raise MemoryError("oracle cell list")
        self.useful = self.examined = 0

    def close(self):
        if self._h:
            _load().oracle_cells_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def matvec_rows(self, x: np.ndarray, sigma: float, rows=None, threads: int = 1) -> np.ndarray:
        """(A x)_i for the given rows (all when None); the pair counts of the
        call go to self.useful / self.examined."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.shape == (self.m,)
        r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
        if r is not None:
            assert r.size == 0 or (r.min() >= 0 and r.max() < self.m)
        n = self.m if r is None else r.size
        y = np.empty(n, dtype=np.float64)
        u, e = C.c_int64(), C.c_int64()
        _load().oracle_cells_matvec(self._h, x.ctypes.data, float(sigma), None if r is None else r.ctypes.data,
                                    n, y.ctypes.data, int(threads), C.byref(u), C.byref(e))
        self.useful, self.examined = u.value, e.value
        return y

    def count(self, rows=None, threads: int = 1) -> int:
        """Pairs inside the truncation of the given rows (all when None): the
        nonzeros of A in those rows."""
        r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
        n = self.m if r is None else r.size
        return int(_load().oracle_cells_count(self._h, None if r is None else r.ctypes.data, n, int(threads)))

    def evaluate(self, c: np.ndarray, pts: np.ndarray, sigma: float, threads: int = 1) -> np.ndarray:
        """f(p) = sum_j c_j phi(|p - x_j|), truncated, at the points pts (k x 3)."""
        c = np.ascontiguousarray(c, dtype=np.float64)
        assert c.shape == (self.m,)
        P = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        out = np.empty(P.shape[0], dtype=np.float64)
        u, e = C.c_int64(), C.c_int64()
        _load().oracle_cells_eval(self._h, c.ctypes.data, float(sigma), P.ctypes.data, P.shape[0], out.ctypes.data,
                                  int(threads), C.byref(u), C.byref(e))
        self.useful, self.examined = u.value, e.value
        return out
