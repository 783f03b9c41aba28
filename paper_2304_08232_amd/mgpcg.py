"""Thin Python binding of libmgpcg.so (the C ABI in include/mgpcg.h).

Argument marshalling only: every step of the solver runs in the HIP library.
torch supplies device memory (tensor.data_ptr()) and streams
(torch.cuda.current_stream().cuda_stream).  The functions named mgpcg_* take
the same arguments as their C counterparts, with torch tensors for vectors;
`Problem` wraps a handle with allocation of outputs for convenience.
"""
import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgpcg.so")

FP64, FP32 = 0, 1
NATURAL, INTERNAL = 0, 1
SMOOTHER_COLOURED, SMOOTHER_SEQUENTIAL = 0, 1
STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "ERR_INVALID_ARG", -2: "ERR_DIMS", -3: "ERR_OOM",
          -4: "ERR_HIP", -5: "ERR_BREAKDOWN", -6: "ERR_NO_DEVICE"}
OK, NOT_CONVERGED, ERR_BREAKDOWN = 0, 1, -5

# every function declared in include/mgpcg.h
ABI_FUNCTIONS = [
    "mgpcg_create", "mgpcg_destroy", "mgpcg_info", "mgpcg_set_theta", "mgpcg_to_internal",
    "mgpcg_to_natural", "mgpcg_spmv", "mgpcg_make_rhs_ones", "mgpcg_gs_sweep", "mgpcg_colour_pass",
    "mgpcg_restrict",
    "mgpcg_prolong_add", "mgpcg_mg_vcycle", "mgpcg_mg_vcycle_noalloc", "mgpcg_pcg_solve", "mgpcg_solve_result",
    "mgpcg_theta_grad", "mgpcg_set_graph_mode", "mgpcg_set_coarse_mode", "mgpcg_get_schedule",
    "mgpcg_set_schedule", "mgpcg_autotune", "mgpcg_check", "mgpcg_last_error",
]


class MGPCGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Schedule(C.Structure):
    _fields_ = [("graph", C.c_int), ("coarse_mode", C.c_int), ("coarse_tail", C.c_int),
                ("wide_levels", C.c_uint), ("lex_run_rows", C.c_int)]


def _sched_dict(s):
    return {name: int(getattr(s, name)) for name, _ in _Schedule._fields_}


class _Config(C.Structure):
    _fields_ = [("ngrids", C.c_int), ("dims", C.POINTER(C.c_int)), ("levels", C.c_int),
                ("nrhs", C.c_int), ("mg_dtype", C.c_int), ("colour_order", C.c_int),
                ("theta", C.c_void_p), ("smoother", C.c_int), ("sweeps", C.c_int)]


_lib = None


def lib():
    """Load libmgpcg.so; fails loudly if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(there is no fallback implementation)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64p, dbl = C.c_void_p, C.c_int, C.POINTER(C.c_int64), C.c_double
        for name in ABI_FUNCTIONS:
            getattr(L, name).restype = C.c_int
        L.mgpcg_last_error.restype = C.c_char_p
        L.mgpcg_last_error.argtypes = []
        L.mgpcg_create.argtypes = [C.POINTER(_Config), vp, C.POINTER(vp)]
        L.mgpcg_destroy.argtypes = [vp]
        L.mgpcg_info.argtypes = [vp, i32, i64p, i64p, i64p]
        L.mgpcg_set_theta.argtypes = [vp, vp, vp]
        L.mgpcg_to_internal.argtypes = [vp, i32, vp, vp, vp]
        L.mgpcg_to_natural.argtypes = [vp, i32, vp, vp, vp]
        L.mgpcg_spmv.argtypes = [vp, i32, vp, vp, i32, vp]
        L.mgpcg_make_rhs_ones.argtypes = [vp, vp, i32, vp]
        L.mgpcg_gs_sweep.argtypes = [vp, i32, vp, vp, i32, vp]
        L.mgpcg_colour_pass.argtypes = [vp, i32, i32, vp, vp, i32, vp]
        L.mgpcg_restrict.argtypes = [vp, i32, vp, vp, vp, i32, vp]
        L.mgpcg_prolong_add.argtypes = [vp, i32, vp, vp, i32, vp]
        L.mgpcg_mg_vcycle.argtypes = [vp, vp, vp, i32, vp]
        L.mgpcg_mg_vcycle_noalloc.argtypes = [vp, vp, vp, i32, vp]
        L.mgpcg_pcg_solve.argtypes = [vp, vp, vp, i32, dbl, vp, vp, i32, vp]
        L.mgpcg_solve_result.argtypes = [vp, i32, vp, vp, vp]
        L.mgpcg_theta_grad.argtypes = [vp, vp, vp, vp, vp, vp]
        L.mgpcg_set_graph_mode.argtypes = [vp, i32]
        L.mgpcg_set_coarse_mode.argtypes = [vp, i32]
        L.mgpcg_get_schedule.argtypes = [vp, C.POINTER(_Schedule)]
        L.mgpcg_set_schedule.argtypes = [vp, C.POINTER(_Schedule), vp]
        L.mgpcg_autotune.argtypes = [vp, vp, i32, i32, C.c_char_p, C.POINTER(_Schedule), vp]
        L.mgpcg_check.argtypes = [vp, vp]
        _lib = L
    return _lib


def _check(st, allow=(OK,)):
    if st not in allow:
        raise MGPCGError(st, lib().mgpcg_last_error().decode(errors="replace"))
    return st


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), \
        "vectors must be contiguous float64 CUDA tensors"
    return C.c_void_p(t.data_ptr())


# ------------------------------------------------------- C-ABI-named calls

def mgpcg_create(dims, levels=4, nrhs=1, mg_dtype=FP64, colour_order=0, theta=None, stream=None,
                 smoother=SMOOTHER_COLOURED, sweeps=1):
    """dims: list of (nx, ny, nz).  Returns the opaque handle (int)."""
    flat = [int(d) for g in dims for d in g]
    arr = (C.c_int * len(flat))(*flat)
    cfg = _Config(len(dims), arr, levels, nrhs, mg_dtype, colour_order,
                  None if theta is None else _ptr(theta).value, smoother, sweeps)
    h = C.c_void_p()
    _check(lib().mgpcg_create(C.byref(cfg), _stream(stream), C.byref(h)))
    return h.value


def mgpcg_destroy(h):
    return _check(lib().mgpcg_destroy(C.c_void_p(h)))


def mgpcg_info(h, level):
    n, nnz, slots = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().mgpcg_info(C.c_void_p(h), level, C.byref(n), C.byref(nnz), C.byref(slots)))
    return n.value, nnz.value, slots.value


def mgpcg_set_theta(h, theta, stream=None):
    return _check(lib().mgpcg_set_theta(C.c_void_p(h), _ptr(theta), _stream(stream)))


def mgpcg_to_internal(h, level, src, dst, stream=None):
    return _check(lib().mgpcg_to_internal(C.c_void_p(h), level, _ptr(src), _ptr(dst), _stream(stream)))


def mgpcg_to_natural(h, level, src, dst, stream=None):
    return _check(lib().mgpcg_to_natural(C.c_void_p(h), level, _ptr(src), _ptr(dst), _stream(stream)))


def mgpcg_spmv(h, level, x, y, layout=NATURAL, stream=None):
    return _check(lib().mgpcg_spmv(C.c_void_p(h), level, _ptr(x), _ptr(y), layout, _stream(stream)))


def mgpcg_make_rhs_ones(h, b, layout=NATURAL, stream=None):
    return _check(lib().mgpcg_make_rhs_ones(C.c_void_p(h), _ptr(b), layout, _stream(stream)))


def mgpcg_gs_sweep(h, level, r, z, layout=NATURAL, stream=None):
    return _check(lib().mgpcg_gs_sweep(C.c_void_p(h), level, _ptr(r), _ptr(z), layout, _stream(stream)))


def mgpcg_colour_pass(h, level, colour, r, z, layout=NATURAL, stream=None):
    return _check(lib().mgpcg_colour_pass(C.c_void_p(h), level, colour, _ptr(r), _ptr(z), layout,
                                          _stream(stream)))


def mgpcg_restrict(h, level, r, z, rc, layout=NATURAL, stream=None):
    return _check(lib().mgpcg_restrict(C.c_void_p(h), level, _ptr(r), _ptr(z), _ptr(rc), layout,
                                       _stream(stream)))


def mgpcg_prolong_add(h, level, zc, z, layout=NATURAL, stream=None):
    return _check(lib().mgpcg_prolong_add(C.c_void_p(h), level, _ptr(zc), _ptr(z), layout, _stream(stream)))


def mgpcg_mg_vcycle(h, r, z, layout=NATURAL, stream=None):
    return _check(lib().mgpcg_mg_vcycle(C.c_void_p(h), _ptr(r), _ptr(z), layout, _stream(stream)))


def mgpcg_mg_vcycle_noalloc(h, r, z, layout=NATURAL, stream=None):
    return _check(lib().mgpcg_mg_vcycle_noalloc(C.c_void_p(h), _ptr(r), _ptr(z), layout, _stream(stream)))


def mgpcg_pcg_solve(h, b, x, max_iters, rel_tol=0.0, history=None, iters=None, layout=NATURAL,
                    stream=None):
    """history: host float64 numpy array (S*max_iters) or None; iters: host int32 array (S) or None."""
    hp = None if history is None else history.ctypes.data_as(C.c_void_p)
    ip = None if iters is None else iters.ctypes.data_as(C.c_void_p)
    return _check(lib().mgpcg_pcg_solve(C.c_void_p(h), _ptr(b), _ptr(x), int(max_iters), float(rel_tol), hp, ip,
                                        layout, _stream(stream)),
                  allow=(OK, NOT_CONVERGED, ERR_BREAKDOWN))


def mgpcg_solve_result(h, max_iters, history=None, iters=None, stream=None):
    hp = None if history is None else history.ctypes.data_as(C.c_void_p)
    ip = None if iters is None else iters.ctypes.data_as(C.c_void_p)
    return _check(lib().mgpcg_solve_result(C.c_void_p(h), int(max_iters), hp, ip, _stream(stream)),
                  allow=(OK, NOT_CONVERGED, ERR_BREAKDOWN))


def mgpcg_theta_grad(h, lam, x, theta, grad, stream=None):
    return _check(lib().mgpcg_theta_grad(C.c_void_p(h), _ptr(lam), _ptr(x), _ptr(theta), _ptr(grad),
                                         _stream(stream)))


def mgpcg_set_graph_mode(h, on):
    return _check(lib().mgpcg_set_graph_mode(C.c_void_p(h), int(on)))


def mgpcg_set_coarse_mode(h, mode):
    return _check(lib().mgpcg_set_coarse_mode(C.c_void_p(h), int(mode)))


def mgpcg_get_schedule(h):
    s = _Schedule()
    _check(lib().mgpcg_get_schedule(C.c_void_p(h), C.byref(s)))
    return _sched_dict(s)


def mgpcg_set_schedule(h, sched, stream=None):
    s = _Schedule(**{k: int(v) for k, v in sched.items()})
    return _check(lib().mgpcg_set_schedule(C.c_void_p(h), C.byref(s), _stream(stream)))


def mgpcg_autotune(h, b=None, iters=10, reps=3, cache_path=None, stream=None):
    s = _Schedule()
    _check(lib().mgpcg_autotune(C.c_void_p(h), None if b is None else _ptr(b), int(iters), int(reps),
                                None if cache_path is None else os.fsencode(cache_path), C.byref(s),
                                _stream(stream)))
    return _sched_dict(s)


def mgpcg_check(h, stream=None):
    return _check(lib().mgpcg_check(C.c_void_p(h), _stream(stream)))


# ------------------------------------------------------------- convenience

class Problem:
    """A level hierarchy of G grids x R right-hand sides on the current GPU."""

    def __init__(self, dims, levels=4, nrhs=1, mg_dtype="fp64", colour_order=0, theta=None, stream=None,
                 smoother="coloured", sweeps=1):
        if isinstance(dims[0], int):
            dims = [tuple(dims)]
        self.dims = [tuple(int(v) for v in d) for d in dims]
        self.levels = levels
        self.nrhs = nrhs
        self.mg_dtype = mg_dtype
        self.colour_order = colour_order
        dt = {"fp64": FP64, "fp32": FP32}[mg_dtype]
        self.smoother = smoother
        sm = {"coloured": SMOOTHER_COLOURED, "sequential": SMOOTHER_SEQUENTIAL}[smoother]
        self.sweeps = sweeps
        self.h = mgpcg_create(self.dims, levels, nrhs, dt, colour_order, theta, stream, sm, sweeps)
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if getattr(self, "h", None):
            mgpcg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nsys(self):
        return len(self.dims) * self.nrhs

    def n(self, level=0):
        return mgpcg_info(self.h, level)[0]

    def nnz(self, level=0):
        return mgpcg_info(self.h, level)[1]

    def size(self, level=0):
        return self.n(level) * self.nrhs

    def empty(self, level=0):
        return torch.empty(self.size(level), dtype=torch.float64, device=self.device)

    def zeros(self, level=0):
        return torch.zeros(self.size(level), dtype=torch.float64, device=self.device)

    def to_internal(self, v, level=0):
        out = self.empty(level)
        mgpcg_to_internal(self.h, level, v, out)
        return out

    def to_natural(self, v, level=0):
        out = self.empty(level)
        mgpcg_to_natural(self.h, level, v, out)
        return out

    def spmv(self, x, level=0, layout=NATURAL):
        y = self.empty(level)
        mgpcg_spmv(self.h, level, x, y, layout)
        return y

    def make_rhs_ones(self, layout=NATURAL):
        b = self.empty(0)
        mgpcg_make_rhs_ones(self.h, b, layout)
        return b

    def gs_sweep(self, r, z, level=0, layout=NATURAL):
        z = z.clone()
        mgpcg_gs_sweep(self.h, level, r, z, layout)
        return z

    def colour_pass(self, r, z, colour, level=0, layout=NATURAL):
        z = z.clone()
        mgpcg_colour_pass(self.h, level, colour, r, z, layout)
        return z

    def restrict(self, r, z, level=0, layout=NATURAL):
        rc = self.empty(level + 1)
        mgpcg_restrict(self.h, level, r, z, rc, layout)
        return rc

    def prolong_add(self, zc, z, level=0, layout=NATURAL):
        z = z.clone()
        mgpcg_prolong_add(self.h, level, zc, z, layout)
        return z

    def vcycle(self, r, layout=NATURAL):
        z = self.empty(0)
        mgpcg_mg_vcycle(self.h, r, z, layout)
        return z

    def solve(self, b, x0=None, max_iters=50, tol=0.0, layout=NATURAL):
        """Returns (x, history [S, iters_max], iters [S], status)."""
        import numpy as np
        x = self.zeros(0) if x0 is None else x0.clone()
        hist = np.zeros(self.nsys * max(max_iters, 1))
        its = np.zeros(self.nsys, np.int32)
        st = mgpcg_pcg_solve(self.h, b, x, max_iters, tol, hist, its, layout)
        hist = hist[: self.nsys * max_iters].reshape(self.nsys, max_iters)
        return x, hist, its, st

    def solve_async(self, b, x, max_iters=50, layout=NATURAL, stream=None):
        return mgpcg_pcg_solve(self.h, b, x, max_iters, 0.0, None, None, layout, stream)

    def set_theta(self, theta):
        mgpcg_set_theta(self.h, theta)

    def theta_grad(self, lam, x, theta):
        g = torch.empty_like(x)
        mgpcg_theta_grad(self.h, lam, x, theta, g)
        return g

    def set_graph_mode(self, on):
        mgpcg_set_graph_mode(self.h, on)

    def set_coarse_mode(self, mode):
        mgpcg_set_coarse_mode(self.h, mode)

    def check(self):
        return mgpcg_check(self.h)

    @property
    def schedule(self):
        """The execution schedule (mgpcg_schedule) as a dict."""
        return mgpcg_get_schedule(self.h)

    def set_schedule(self, **fields):
        """Change some fields of the schedule; the rest keep their values."""
        s = self.schedule
        s.update(fields)
        mgpcg_set_schedule(self.h, s)

    def autotune(self, b=None, iters=10, reps=3, cache_path=None):
        """Time candidate schedules, apply the fastest; returns it."""
        return mgpcg_autotune(self.h, b, iters, reps, cache_path)


class MGPCGSolve(torch.autograd.Function):
    """x = A(theta)^{-1} b with a_ii = 26 + softplus(theta_i) on one grid.

    Forward: MG-PCG to `tol`.  Backward: the adjoint solve lambda = A^{-1} dL/dx
    with the same MG-PCG (A is symmetric), then dL/dtheta = -lambda * x *
    logistic(theta) in one fused kernel, and dL/db = lambda.
    """

    @staticmethod
    def forward(ctx, theta, b, dims, levels=4, tol=1e-10, max_iters=500):
        theta = theta.detach().contiguous()
        prob = Problem(tuple(dims), levels=levels, theta=theta)
        x, hist, its, st = prob.solve(b.detach().contiguous(), max_iters=max_iters, tol=tol)
        if st != OK:
            raise MGPCGError(st, "forward solve did not converge")
        ctx.prob, ctx.tol, ctx.max_iters = prob, tol, max_iters
        ctx.save_for_backward(theta, x)
        ctx.forward_iters = int(its[0])
        return x

    @staticmethod
    def backward(ctx, gx):
        theta, x = ctx.saved_tensors
        prob = ctx.prob
        lam, hist, its, st = prob.solve(gx.contiguous(), max_iters=ctx.max_iters, tol=ctx.tol)
        if st != OK:
            raise MGPCGError(st, "adjoint solve did not converge")
        gtheta = prob.theta_grad(lam, x, theta)
        return gtheta, lam, None, None, None, None
