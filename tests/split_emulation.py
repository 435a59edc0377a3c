"""CPU model of the embed kernels' arithmetic (test infrastructure).

It reproduces, with NumPy, what the FP32 and split-precision kernels do to
the numbers, so that the error bounds stated in tests/tolerance.py can be
re-derived without a GPU:

* the model is cast to FP32 as the library stores it: landmarks M, the
  weights W = 1/2 V Lambda^{-1/2} and the bias c = q - |m|^2;
* row norms |x|^2 in FP32;
* x.m either in FP32 or from split operands: a value is cut into parts,
  each the round-to-nearest-even BF16 (or FP16) value of what the earlier
  parts leave, the chosen products of parts are formed exactly and summed
  in FP32 (FP16 operands are first scaled by a power of two that puts the
  largest landmark value near 2^12, as the fit does);
* e = (c - |x|^2) + 2 x.m and y = E W in FP32.

The summation order of an FP32 matrix product here is NumPy's, not the
matrix cores', so figures agree with the GPU's to their leading digit, not
bit for bit.  Nothing here is used by the library or by the oracle.
"""

import numpy as np

# products (part of x, part of m) summed by each precision form
PRODUCTS = {
    "split_bf16": ((0, 0), (0, 1), (1, 0), (1, 1)),  # four products, as the kernel
    "split_bf16_three": ((0, 0), (0, 1), (1, 0)),    # without lo.lo, for comparison
    "split_fp16": ((0, 0), (0, 1), (1, 0)),
}


def round_bf16(x):
    """Round-to-nearest-even of FP32 values to BF16, returned as FP32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32)


def round_fp16(x):
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float32)


def split(x, rnd, parts=2):
    out, rest = [], np.asarray(x, dtype=np.float32)
    for _ in range(parts):
        h = rnd(rest)
        out.append(h)
        rest = (rest - h).astype(np.float32)
    return out


def embed(fit, X, prec):
    """Coordinates of the rows X for the oracle's fit, in the kernels'
    arithmetic for prec in {"fp32"} | PRODUCTS."""
    M = fit.M.astype(np.float32)
    scale_w = np.where(fit.live, 0.5 / np.sqrt(np.where(fit.live, fit.lam, 1.0)), 0.0)
    W = (fit.V * scale_w[None, :]).astype(np.float32)
    c = (fit.q - np.sum(fit.M ** 2, axis=1)).astype(np.float32)
    X32 = np.asarray(X, dtype=np.float32)
    xn = np.sum(X32 * X32, axis=1, dtype=np.float32)
    if prec == "fp32":
        S = X32 @ M.T
    else:
        fp16 = prec == "split_fp16"
        rnd = round_fp16 if fp16 else round_bf16
        s = 1.0
        if fp16:
            s = float(2.0 ** (12 - np.ceil(np.log2(np.max(np.abs(M))))))
        xs = split(X32 * np.float32(s), rnd)
        ms = split(M * np.float32(s), rnd)
        S = np.zeros((X32.shape[0], M.shape[0]), dtype=np.float32)
        for a, b in PRODUCTS[prec]:
            S = (S + xs[a] @ ms[b].T).astype(np.float32)
        S = (S / np.float32(s * s)).astype(np.float32)
    E = ((c[None, :] - xn[:, None]) + np.float32(2.0) * S).astype(np.float32)
    return (E @ W).astype(np.float64)
