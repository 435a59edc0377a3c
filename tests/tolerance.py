"""Tolerances of the GPU results against the FP64 oracle.

Two readings of "relative error" are checked for every result (per output
column k, R the oracle's coordinates, D = Y - R; dead columns must be
exactly zero):

* rms_rel     |D_k|_2 / |R_k|_2             (the binding reading)
* maxabs_rms  max_i |D_ik| / rms(R_k)

FP64: 1e-9 on both.  FP32 and the split forms: 1e-4 on both, for results
whose r columns are all strong directions of the data (the workloads the
paper simulates with r = h: the first columns of the Gaussian laws, integer
data, data of rank r).

Weak directions.  When the output also holds directions from a Gaussian
law's isotropic unit-variance bulk (r = 16, 20 on the 10-strong-column
laws), the error of column k grows as (per-value scale of the data) /
(spread of column k) times the rounding unit of the distance products, and
FP32 arithmetic itself no longer keeps the max-abs reading under 1e-4.
An emulation of the kernels' arithmetic on the CPU (BF16/FP16 parts by
bit operations, FP32 products) on those cases gives, worst over the cases
(rms_rel / maxabs_rms):

    FP32         1.3e-5 / 1.6e-4
    split FP16   1.3e-5 / 1.6e-4   (11-bit parts: as accurate as FP32)
    split BF16   1.0e-4 / 3.7e-4   (8-bit parts, four products)

so the weak-direction bounds are, about twice those values: FP32 and split
FP16 rms_rel 1e-4 and maxabs_rms 3e-4; split BF16 rms_rel 2e-4 and
maxabs_rms 8e-4.
"""

import numpy as np

from synth import errors

STRONG = {
    "fp64": (1e-9, 1e-9),
    "fp32": (1e-4, 1e-4),
    "split_fp16": (1e-4, 1e-4),
    "split_bf16": (1e-4, 1e-4),
}
WEAK = {
    "fp64": (1e-9, 1e-9),
    "fp32": (1e-4, 3e-4),
    "split_fp16": (1e-4, 3e-4),
    "split_bf16": (2e-4, 8e-4),
}


def bounds(prec, weak=False):
    return (WEAK if weak else STRONG)[prec]


def check_embed(Y, Yo, prec, weak=False):
    """Both readings against the oracle over the rows given."""
    e = errors.column_errors(Y, Yo)
    rms_tol, max_tol = bounds(prec, weak)
    assert e["rms_rel"] <= rms_tol, (prec, weak, e)
    assert e["maxabs_rms"] <= max_tol, (prec, weak, e)
    return e


def check_rows(Y, Yo, scale, prec, weak=False):
    """A subset of rows (a serving request, possibly a single row) against
    the oracle, normalised by the column RMS `scale` of the whole data set
    the rows come from: RMS and max of |D_k| / scale_k."""
    Y = np.asarray(Y, dtype=np.float64)
    Yo = np.asarray(Yo, dtype=np.float64)
    assert Y.shape == Yo.shape, (Y.shape, Yo.shape)
    if Y.shape[0] == 0:
        return
    rms_tol, max_tol = bounds(prec, weak)
    for k in range(Yo.shape[1]):
        if scale[k] == 0.0:
            assert np.all(Y[:, k] == 0.0), (prec, k)
            continue
        d = np.abs(Y[:, k] - Yo[:, k]) / scale[k]
        assert np.sqrt(np.mean(d * d)) <= rms_tol, (prec, k, float(np.sqrt(np.mean(d * d))))
        assert np.max(d) <= max_tol, (prec, k, float(np.max(d)))


def column_rms(Yo):
    Yo = np.asarray(Yo, dtype=np.float64)
    return np.sqrt(np.mean(Yo * Yo, axis=0))
