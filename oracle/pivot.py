"""FP64 CPU oracle of MaxMin landmark selection and pivot MDS (test
infrastructure only; nothing on the product path may import it).

* MaxMin (the landmark choice of LMDS, Section 3.1): start from a given
  point; repeatedly add the point whose smallest squared distance to the
  points chosen so far is largest.  Readings: squared Euclidean distances
  (the same ordering as distances); each squared distance is summed over
  the columns in order, one rounded product and one rounded sum per column,
  so any implementation that follows this order obtains the same values
  and takes the same decisions; ties go to the smallest index; fewer than
  l distinct points is an error.
* Pivot MDS (Section 3.1): with l pivot points, C is the n x l block of
  inner products between all points and the pivots, and the singular value
  decomposition of C stands in for the eigendecomposition of Q.  Readings:
  C is the double centring of the n x l block of squared distances
  (c_ij = -1/2 (d_ij - row mean_i - column mean_j + grand mean), the only
  centring available without all n^2 distances); the eigenvalues of Q are
  estimated from the singular values as lambda = sigma sqrt(n / l), which is
  exact when the pivots are all the points (C = Q); the configuration is
  X = U_r Lambda_r^{1/2}; the sign of each column follows the right
  singular vector in pivot space (largest-magnitude entry positive, first
  on ties).
* Live directions.  Classical MDS (Section 2, step 3) keeps the r greatest
  non-negative eigenvalues of the matrix it decomposes; the reading used for
  every method here is "eigenvalue > TAU times the largest".  Pivot MDS
  decomposes C through its singular value decomposition, i.e. the
  eigendecomposition of C'C (right singular vectors = its eigenvectors,
  squared singular values = its eigenvalues), so the rule applies to
  sigma_k^2: direction k is live when sigma_k^2 > TAU sigma_1^2.  The
  estimate lambda = sigma sqrt(n / l) only rescales what was decomposed.
  In terms of lambda this is lambda_k > sqrt(TAU) lambda_1; dead columns
  are zero and report lambda = 0.
"""

import numpy as np

from .mds import TAU, DegenerateError


def sqdist_to(X, m):
    """Squared distance from every row of X to the point m, summed over the
    columns in order with separately rounded products and sums."""
    X = np.asarray(X, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    acc = np.zeros(X.shape[0])
    for k in range(X.shape[1]):
        d = X[:, k] - m[k]
        acc = acc + d * d
    return acc


def maxmin_landmarks(X, l, first):
    """l indices in selection order: first, then greedy MaxMin."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    if not (1 <= l <= n) or not (0 <= first < n):
        raise ValueError("need 1 <= l <= n and 0 <= first < n")
    idx = [int(first)]
    dmin = sqdist_to(X, X[first])
    for _ in range(1, l):
        j = int(np.argmax(dmin))  # first maximum: smallest index on ties
        if not dmin[j] > 0.0:
            raise DegenerateError("fewer than l distinct points")
        idx.append(j)
        dmin = np.minimum(dmin, sqdist_to(X, X[j]))
    return np.array(idx, dtype=np.int64)


def pivot_block(X, idx):
    """C: double-centred n x l block of squared distances to the pivots."""
    X = np.asarray(X, dtype=np.float64)
    M = X[idx]
    D = np.empty((X.shape[0], M.shape[0]))
    for j in range(M.shape[0]):
        D[:, j] = sqdist_to(X, M[j])
    return -0.5 * (D - D.mean(axis=1)[:, None] - D.mean(axis=0)[None, :] + D.mean())


def pivot_mds(X, idx, r):
    """Pivot MDS configuration (n x r), eigenvalue estimates (r) and the
    pivot-space singular vectors W (l x r, sign-fixed)."""
    X = np.asarray(X, dtype=np.float64)
    n, l = X.shape[0], len(idx)
    C = pivot_block(X, idx)
    U, s, Wt = np.linalg.svd(C, full_matrices=False)
    U = U[:, :r].copy()
    W = Wt[:r].T.copy()
    s = s[:r]
    for k in range(W.shape[1]):
        i = int(np.argmax(np.abs(W[:, k])))
        if W[i, k] < 0:
            W[:, k] = -W[:, k]
            U[:, k] = -U[:, k]
    lam = s * np.sqrt(n / l)
    if not lam[0] > 0:
        raise DegenerateError("largest eigenvalue is not positive")
    live = s * s > TAU * s[0] * s[0]  # eigenvalues of C'C (module docstring)
    lam = np.where(live, lam, 0.0)
    Y = np.zeros((n, len(lam)))
    Y[:, live] = U[:, live] * np.sqrt(lam[live])
    return Y, lam, W


def pivot_mds_large(X, idx, r, rows=None, chunk=65536):
    """Pivot MDS for large n without holding the n x l block: squared
    distances by the oracle's centred FP64 expansion (sqdist_rows_expanded),
    C'C accumulated over row chunks, its eigenpairs (sigma^2, W), then
    Y = C W Sigma^{-1} Lambda^{1/2} for the requested rows only (all when
    rows is None).  Same readings as pivot_mds; returns (Y_rows, lam, W)."""
    from .mds import sqdist_rows_expanded
    X = np.asarray(X)
    n, l = X.shape[0], len(idx)
    M = np.asarray(X[idx], dtype=np.float64)
    colsum = np.zeros(l)
    tot = 0.0
    for s in range(0, n, chunk):
        D = sqdist_rows_expanded(X[s:s + chunk].astype(np.float64), M)
        colsum += D.sum(axis=0)
        tot += D.sum()
    colmean = colsum / n
    grand = tot / (n * l)

    def block(s, e):
        D = sqdist_rows_expanded(X[s:e].astype(np.float64), M)
        return -0.5 * (D - D.mean(axis=1)[:, None] - colmean[None, :] + grand)

    CtC = np.zeros((l, l))
    for s in range(0, n, chunk):
        C = block(s, min(n, s + chunk))
        CtC += C.T @ C
    th, V = np.linalg.eigh(0.5 * (CtC + CtC.T))
    order = np.argsort(-th, kind="stable")[:r]
    th = th[order]
    W = V[:, order].copy()
    for k in range(r):
        i = int(np.argmax(np.abs(W[:, k])))
        if W[i, k] < 0:
            W[:, k] = -W[:, k]
    sigma = np.sqrt(np.maximum(th, 0.0))
    lam = sigma * np.sqrt(n / l)
    if not lam[0] > 0:
        raise DegenerateError("largest eigenvalue is not positive")
    live = th > TAU * th[0]
    lam = np.where(live, lam, 0.0)
    fac = np.zeros(r)
    fac[live] = np.sqrt(lam[live]) / sigma[live]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    Y = np.empty((len(rows), r))
    for s in range(0, len(rows), chunk):
        sel = rows[s:s + chunk]
        D = sqdist_rows_expanded(X[sel].astype(np.float64), M)
        C = -0.5 * (D - D.mean(axis=1)[:, None] - colmean[None, :] + grand)
        Y[s:s + chunk] = (C @ W) * fac[None, :]
    return Y, lam, W
