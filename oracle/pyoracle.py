"""ctypes wrapper around the C oracle (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  All vectors are float64 numpy arrays in natural order
i = ix + nx*(iy + ny*iz).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_libs = {}


def lib(omp=False):
    """The sequential oracle (the checker), or with omp=True the OpenMP
    timing build of the same source.  MGPCG_ORACLE_LIB names another build
    of the sequential oracle to load instead (the mutation tests use it)."""
    key = bool(omp)
    if key not in _libs:
        path = _build.LIB_OMP if omp else os.environ.get("MGPCG_ORACLE_LIB", _build.LIB)
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int, C.c_double
        L.ora_create.restype = vp
        L.ora_create.argtypes = [i32, i32, i32, i32, i32, vp]
        L.ora_destroy.argtypes = [vp]
        L.ora_set_sweeps.restype = i32
        L.ora_set_sweeps.argtypes = [vp, i32]
        L.ora_n.restype = i64
        L.ora_n.argtypes = [vp, i32]
        L.ora_nnz.restype = i64
        L.ora_nnz.argtypes = [vp, i32]
        L.ora_ncolours.restype = i32
        L.ora_ncolours.argtypes = [vp, i32]
        L.ora_get_crs.argtypes = [vp, i32, vp, vp, vp]
        L.ora_get_colours.argtypes = [vp, i32, vp]
        L.ora_get_f2c.argtypes = [vp, i32, vp]
        L.ora_spmv.argtypes = [vp, i32, vp, vp]
        L.ora_colour_pass.argtypes = [vp, i32, i32, vp, vp]
        L.ora_sgs.argtypes = [vp, i32, vp, vp]
        L.ora_restrict.argtypes = [vp, i32, vp, vp, vp]
        L.ora_prolong_add.argtypes = [vp, i32, vp, vp]
        L.ora_vcycle.argtypes = [vp, i32, vp, vp]
        L.ora_sgs_lex.argtypes = [vp, i32, vp, vp]
        L.ora_vcycle_lex.argtypes = [vp, i32, vp, vp]
        L.ora_vcycle32.argtypes = [vp, vp, vp]
        L.ora_sgs32.argtypes = [vp, i32, vp, vp]
        L.ora_pcg.restype = i32
        L.ora_pcg.argtypes = [vp, vp, vp, i32, dbl, i32, vp, vp]
        L.ora_theta_grad.argtypes = [i64, vp, vp, vp, vp]
        L.ora_dot.restype = dbl
        L.ora_dot.argtypes = [i64, vp, vp]
        L.ora_threads.restype = i32
        L.ora_threads.argtypes = []
        _libs[key] = L
    return _libs[key]


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


class Oracle:
    """One level hierarchy of the MG-PCG problem, built by the C oracle."""

    def __init__(self, nx, ny, nz, levels=4, colour_order=0, theta=None, sweeps=1, omp=False):
        self._L = lib(omp)
        self.dims = (nx, ny, nz)
        self.levels = levels
        self.colour_order = colour_order
        th = None
        if theta is not None:
            th = _f64(theta)
            assert th.size == nx * ny * nz
        self._h = self._L.ora_create(nx, ny, nz, levels, colour_order, None if th is None else _p(th))
        if not self._h:
            raise ValueError(f"oracle: invalid problem {nx}x{ny}x{nz} levels={levels}")
        if self._L.ora_set_sweeps(self._h, sweeps) != 0:
            self.close()
            raise ValueError(f"oracle: invalid sweep count {sweeps}")

    def close(self):
        if self._h:
            self._L.ora_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- introspection
    def n(self, level=0):
        return self._L.ora_n(self._h, level)

    def nnz(self, level=0):
        return self._L.ora_nnz(self._h, level)

    def ncolours(self, level=0):
        return self._L.ora_ncolours(self._h, level)

    def level_dims(self, level):
        return tuple(d >> level for d in self.dims)

    def crs(self, level=0):
        n, nnz = self.n(level), self.nnz(level)
        rp = np.zeros(n + 1, np.int64)
        col = np.zeros(nnz, np.int32)
        val = np.zeros(nnz, np.float64)
        self._L.ora_get_crs(self._h, level, _p(rp), _p(col), _p(val))
        return rp, col, val

    def dense(self, level=0):
        rp, col, val = self.crs(level)
        n = self.n(level)
        A = np.zeros((n, n))
        for i in range(n):
            A[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
        return A

    def colours(self, level=0):
        c = np.zeros(self.n(level), np.int32)
        self._L.ora_get_colours(self._h, level, _p(c))
        return c

    def f2c(self, level=0):
        m = np.zeros(self.n(level + 1), np.int64)
        self._L.ora_get_f2c(self._h, level, _p(m))
        return m

    # --- building blocks
    def spmv(self, x, level=0):
        x = _f64(x)
        y = np.zeros(self.n(level))
        self._L.ora_spmv(self._h, level, _p(x), _p(y))
        return y

    def colour_pass(self, k, r, z, level=0):
        r = _f64(r)
        z = _f64(z).copy()
        self._L.ora_colour_pass(self._h, level, k, _p(r), _p(z))
        return z

    def sgs(self, r, z, level=0):
        r = _f64(r)
        z = _f64(z).copy()
        self._L.ora_sgs(self._h, level, _p(r), _p(z))
        return z

    def sgs32(self, r, z, level=0):
        r = np.ascontiguousarray(r, dtype=np.float32)
        z = np.ascontiguousarray(z, dtype=np.float32).copy()
        self._L.ora_sgs32(self._h, level, _p(r), _p(z))
        return z

    def restrict(self, r, z, level=0):
        r, z = _f64(r), _f64(z)
        rc = np.zeros(self.n(level + 1))
        self._L.ora_restrict(self._h, level, _p(r), _p(z), _p(rc))
        return rc

    def prolong_add(self, zc, z, level=0):
        zc = _f64(zc)
        z = _f64(z).copy()
        self._L.ora_prolong_add(self._h, level, _p(zc), _p(z))
        return z

    def vcycle(self, r, level=0):
        r = _f64(r)
        z = np.zeros(self.n(level))
        self._L.ora_vcycle(self._h, level, _p(r), _p(z))
        return z

    def sgs_lex(self, r, z, level=0):
        """Sequential symmetric Gauss-Seidel (Eq. (1), natural row order)."""
        r = _f64(r)
        z = _f64(z).copy()
        self._L.ora_sgs_lex(self._h, level, _p(r), _p(z))
        return z

    def vcycle_lex(self, r, level=0):
        r = _f64(r)
        z = np.zeros(self.n(level))
        self._L.ora_vcycle_lex(self._h, level, _p(r), _p(z))
        return z

    def vcycle32(self, r):
        r = _f64(r)
        z = np.zeros(self.n(0))
        self._L.ora_vcycle32(self._h, _p(r), _p(z))
        return z

    def pcg(self, b, x0=None, max_iters=50, tol=0.0, precond=1):
        """Returns (x, history, iters, status)."""
        b = _f64(b)
        x = np.zeros(self.n(0)) if x0 is None else _f64(x0).copy()
        hist = np.zeros(max(max_iters, 1))
        it = C.c_int(0)
        st = self._L.ora_pcg(self._h, _p(b), _p(x), max_iters, float(tol), precond,
                           _p(hist), C.byref(it))
        return x, hist[: it.value].copy(), it.value, st

    def threads(self):
        """Threads this build's loops run on (1: the sequential checker)."""
        return self._L.ora_threads()

    @staticmethod
    def theta_grad(lam, x, theta):
        lam, x, theta = _f64(lam), _f64(x), _f64(theta)
        g = np.zeros(lam.size)
        lib().ora_theta_grad(lam.size, _p(lam), _p(x), _p(theta), _p(g))
        return g

    @staticmethod
    def dot(a, b):
        a, b = _f64(a), _f64(b)
        return lib().ora_dot(a.size, _p(a), _p(b))
