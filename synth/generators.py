"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no step of the MDS method: it only draws data, so both the
oracle and the HIP path may take their inputs from it.  Every generator uses
``numpy.random.Generator(PCG64(seed))`` and draws rows in fixed chunks, so
the same (shape, seed) always yields the same array on any machine.

Workload shapes (the paper's simulation design is Section 4.1; its real data
set in Section 5 is 814,255 grey-scale 28x28 images, which is not available
here and is stood in for by ``image_mixture``):

* ``gaussian_columns``: independent zero-mean Gaussian columns with given
  standard deviations; the paper's design uses variance 15 on the first h
  columns and 1 on the rest (``paper_design``).
* ``image_mixture``: a 10-component Gaussian mixture in 784 dimensions with
  integer values 0..255, like flattened 8-bit images.
* ``low_rank``: points lying exactly in an r-dimensional affine subspace.
* ``request_sizes`` / ``poisson_arrivals``: serving traffic.
"""

import numpy as np

CHUNK_ROWS = 1 << 16

SIGMAS_SMALL = np.array([15.0, 10.0] + [1.0] * 8)
SIGMAS_WIDE = np.concatenate([np.linspace(20.0, 2.0, 10), np.ones(90)])
SIGMAS_P50 = np.concatenate([np.linspace(20.0, 2.0, 10), np.ones(40)])


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def gaussian_columns(n, sigmas, seed, dtype=np.float32):
    """Rows iid N(0, diag(sigmas^2)), drawn in FP64 and cast once."""
    sigmas = np.asarray(sigmas, dtype=np.float64)
    p = sigmas.shape[0]
    rng = _rng(seed)
    out = np.empty((int(n), p), dtype=dtype)
    for s in range(0, int(n), CHUNK_ROWS):
        e = min(int(n), s + CHUNK_ROWS)
        out[s:e] = (rng.standard_normal((e - s, p)) * sigmas).astype(dtype)
    return out


def paper_design(n, k, h, seed, dtype=np.float64):
    """The simulation design of Section 4.1: variance 15 on the first h of
    k columns, variance 1 on the others."""
    sig = np.ones(k)
    sig[:h] = np.sqrt(15.0)
    return gaussian_columns(n, sig, seed, dtype=dtype)


def small_gaussian(n=5000, seed=11, dtype=np.float64):
    """n x 10 rows, column std devs (15, 10, 1, ..., 1)."""
    return gaussian_columns(n, SIGMAS_SMALL, seed, dtype=dtype)


def wide_gaussian(n=1_000_000, seed=12, dtype=np.float32):
    """n x 100 rows, first 10 std devs linearly spaced 20 -> 2, rest 1."""
    return gaussian_columns(n, SIGMAS_WIDE, seed, dtype=dtype)


def image_mixture(n=1_000_000, p=784, components=10, std=40.0, seed=13,
                  dtype=np.float32):
    """Equal-weight Gaussian mixture with means uniform in [0, 255]^p and
    isotropic std ``std``; values rounded half-to-even and clipped to
    0..255, stored as ``dtype``."""
    rng = _rng(seed)
    mu = rng.uniform(0.0, 255.0, size=(components, p))
    out = np.empty((int(n), p), dtype=dtype)
    for s in range(0, int(n), CHUNK_ROWS):
        e = min(int(n), s + CHUNK_ROWS)
        comp = rng.integers(0, components, size=e - s)
        x = mu[comp] + std * rng.standard_normal((e - s, p))
        np.rint(x, out=x)
        np.clip(x, 0.0, 255.0, out=x)
        out[s:e] = x.astype(dtype)
    return out


def low_rank(n, p, r, seed, scale=5.0, dtype=np.float64):
    """n points in an r-dimensional affine subspace of R^p: Z B + b with
    Z ~ N(0, scale^2), B an r x p matrix with orthonormal rows.  Returns
    (X, Z) where Z holds the intrinsic coordinates (X is an isometric image
    of Z)."""
    rng = _rng(seed)
    Z = scale * rng.standard_normal((n, r)) * np.linspace(2.0, 1.0, r)
    B, _ = np.linalg.qr(rng.standard_normal((p, r)))
    b = rng.uniform(-10.0, 10.0, size=p)
    return (Z @ B.T + b).astype(dtype), Z


def request_sizes(count, max_points, seed):
    """Request point counts floor(exp(U[0, ln(max_points + 1)))), i.e.
    log-uniform in [1, max_points]."""
    rng = _rng(seed)
    u = rng.uniform(0.0, np.log(max_points + 1.0), size=count)
    return np.maximum(1, np.floor(np.exp(u))).astype(np.int64)


def poisson_arrivals(count, rate, seed):
    """Arrival times (seconds) of a Poisson process with the given rate."""
    rng = _rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
