"""Seeded synthetic inputs for tests and benchmarks.

This module only draws numbers; it holds none of the product's arithmetic,
so both the FP64 oracle and the HIP path may take their inputs from it.

Every generator uses numpy's PCG64 (``numpy.random.default_rng``) with an
explicit integer seed, draws in float64 and returns float64; callers round to
the storage dtype and hand the *same* rounded values to both sides.

Workload recipes (the paper measures square matrices of unstated size,
Sec. 7; these stand in for them):
* ``uniform``       -- i.i.d. U[lo, hi)
* ``normal``        -- i.i.d. N(0, 1)
* ``small_int``     -- i.i.d. integers in [lo, hi] (exact in every dtype used)
* ``row_scaled``    -- N(0, 1) times a per-row scale 10**U[-3, 3), i.e. scales
                       log-uniform in [1e-3, 1e3]
"""
import numpy as np

BASE_SEED = 9809105


def rng(seed):
    return np.random.default_rng(np.random.PCG64(int(seed)))


def uniform(shape, seed, lo=-1.0, hi=1.0):
    return rng(seed).uniform(lo, hi, size=shape)


def normal(shape, seed):
    return rng(seed).standard_normal(size=shape)


def small_int(shape, seed, lo=-8, hi=8):
    return rng(seed).integers(lo, hi + 1, size=shape).astype(np.float64)


def row_scaled(shape, seed, lo_exp=-3.0, hi_exp=3.0):
    g = rng(seed)
    x = g.standard_normal(size=shape)
    scale = 10.0 ** g.uniform(lo_exp, hi_exp, size=(shape[0], 1))
    return x * scale


def sample_rows(n_rows, count, seed):
    """``count`` distinct sorted row indices in [0, n_rows)."""
    count = min(count, n_rows)
    return np.sort(rng(seed).choice(n_rows, size=count, replace=False)).astype(np.int64)
