"""Seeded synthetic inputs shared by tests and benchmarks.

Random draws only (numpy PCG64 via default_rng); none of the solver's
arithmetic lives here.  Every array is float64 in natural grid order.
"""
import numpy as np

BATCH_DIM_CHOICES = (24, 32, 48, 64, 96)


def uniform(seed, n, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, n)


def perturbation(seed, n, amp=1e-3):
    """U[-amp, amp] added to b = A*1 for the mixed-precision workload."""
    return np.random.default_rng(seed).uniform(-amp, amp, n)


def batch_dims(seed, count=64, choices=BATCH_DIM_CHOICES):
    """count grids with nx, ny, nz each drawn from `choices`."""
    rng = np.random.default_rng(seed)
    return [tuple(int(v) for v in row) for row in rng.choice(np.array(choices), size=(count, 3))]


def batch_rhs(seed, sizes):
    """One U[-1,1] right-hand side per grid, drawn in grid order, packed."""
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.uniform(-1.0, 1.0, int(n)) for n in sizes])


def multi_rhs(seed, nrhs, n):
    """nrhs right-hand sides of length n, U[-1,1], packed rhs after rhs."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, (nrhs, n)).ravel()


def differentiable_inputs(seed, n):
    """theta ~ N(0, 0.5^2), then b ~ U[-1,1], then x_target ~ U[-1,1]."""
    rng = np.random.default_rng(seed)
    theta = rng.normal(0.0, 0.5, n)
    b = rng.uniform(-1.0, 1.0, n)
    xt = rng.uniform(-1.0, 1.0, n)
    return theta, b, xt
