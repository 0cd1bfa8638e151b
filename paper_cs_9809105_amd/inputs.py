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
* ``plummer``       -- n bodies (x, y, z, m) drawn from a Plummer sphere, the
                       standard model of a globular cluster (the application
                       the paper names for the gravitational n^2-problem)
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


def plummer(n, seed, scale=1.0, total_mass=1.0, unequal=False, u_max=0.999):
    """n x 4 array of bodies (x, y, z, m) from a Plummer sphere of scale
    length ``scale``: the enclosed mass fraction u = r^3 / (r^2 + a^2)^(3/2)
    is drawn uniformly in [0, u_max) (u_max < 1 cuts the far tail) and
    inverted, r = a / sqrt(u^(-2/3) - 1); directions are isotropic.  Masses
    are equal (total_mass / n) or, with ``unequal``, proportional to
    U[0.5, 1.5) and normalised to total_mass."""
    g = rng(seed)
    u = g.uniform(0.0, u_max, size=n)
    with np.errstate(divide="ignore"):
        r = scale / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    cos_t = g.uniform(-1.0, 1.0, size=n)
    phi = g.uniform(0.0, 2.0 * np.pi, size=n)
    sin_t = np.sqrt(1.0 - cos_t * cos_t)
    out = np.empty((n, 4), np.float64)
    out[:, 0] = r * sin_t * np.cos(phi)
    out[:, 1] = r * sin_t * np.sin(phi)
    out[:, 2] = r * cos_t
    if unequal:
        w = g.uniform(0.5, 1.5, size=n)
        out[:, 3] = w * (total_mass / w.sum()) if n else w
    else:
        out[:, 3] = total_mass / max(n, 1)
    return out
