"""FP64 CPU oracle of interpolation MDS (test infrastructure only).

Nothing on the product path may import this module: only the tests, the
smoke check and the CPU-baseline leg of the benchmark use it.  It shares no
code with the HIP library.

What it computes, following Delicado and Pachon-Garcia, "Multidimensional
scaling for big data":

* Classical MDS (Section 2, the four-step algorithm and eq. (1)):
  Q = -1/2 P Delta P with the centring matrix P = I - 11'/n, eigenpairs of Q
  sorted by decreasing eigenvalue, keep the r largest non-negative ones,
  X = V_r Lambda_r^{1/2}; the columns of X have variance Lambda_r / n.
* Interpolation MDS (Section 3.1): classical MDS on a random subset of l
  points (the landmarks), then Gower's interpolation formula, eq. (2),
      X2 = 1/(2l) (1 q1' - A21^2) X1 S1^{-1},   S1 = Lambda_{1,r} / l,
  where q1 = diag(Q1) and A21^2 holds squared distances from new points to
  the landmarks.  New points are processed in blocks of m = l rows, as the
  paper proposes.
* Landmark MDS triangulation, eq. (3), used only to check Proposition 1:
      X2_LMDS = 1/2 (1 d1' - A21^2) V_{1,r} Lambda_{1,r}^{-1/2},
  with d1 = Delta1 1 / l.

Readings where the paper is silent (the same ones the library takes):
* squared Euclidean distances between data rows are the dissimilarities
  (Section 4.1 uses Euclidean distances between rows);
* an eigenvalue counts as "non-negative" (live) only when it exceeds
  TAU * lambda_1; dead columns get exactly zero coordinates;
* the sign of each eigenvector is fixed by making its largest-magnitude
  component positive (smallest index on exact ties);
* every row handed to the interpolation step is interpolated, landmarks
  included, and rows come back in input order.
"""

from dataclasses import dataclass

import numpy as np

from .sampler import sample_landmarks

TAU = 1e-9


@dataclass
class Fit:
    idx: np.ndarray      # (l,) int64 ascending landmark indices
    M: np.ndarray        # (l, p) FP64 landmark rows
    D1: np.ndarray       # (l, l) squared distances Delta1
    Q1: np.ndarray       # (l, l) -1/2 P Delta1 P
    q: np.ndarray        # (l,) diag(Q1)
    d1: np.ndarray       # (l,) row means of Delta1
    dbar: float          # grand mean of Delta1
    lam: np.ndarray      # (r,) top eigenvalues, descending (dead ones kept)
    V: np.ndarray        # (l, r) eigenvectors after the sign convention
    live: np.ndarray     # (r,) bool, lam > TAU * lam[0]
    X1: np.ndarray       # (l, r) V Lambda^{1/2}, dead columns zero
    r_eff: int


class DegenerateError(ValueError):
    """All landmarks coincide: lambda_1 <= 0, no configuration exists."""


def sqdist_rows(A, B):
    """Squared Euclidean distances between the rows of A and of B, by direct
    differences (the definition d_ij^2 = sum_k (a_ik - b_jk)^2, Section 2)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    out = np.empty((A.shape[0], B.shape[0]))
    for i in range(A.shape[0]):
        diff = B - A[i]
        out[i] = np.einsum("jk,jk->j", diff, diff)
    return out


def sqdist_rows_expanded(A, B):
    """Same quantity through the expansion |a-c|^2 + |b-c|^2 - 2 (a-c).(b-c)
    about the centre c of B, with one FP64 matrix product.  Used for the
    large cross blocks of the CPU baseline; checked against sqdist_rows."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    c = B.mean(axis=0)
    Ac = A - c
    Bc = B - c
    na = np.einsum("ik,ik->i", Ac, Ac)
    nb = np.einsum("jk,jk->j", Bc, Bc)
    return na[:, None] + nb[None, :] - 2.0 * (Ac @ Bc.T)


def centring_matrix(n):
    """P = I_n - (1/n) 1 1' (Section 2)."""
    return np.eye(n) - np.full((n, n), 1.0 / n)


def inner_products(D):
    """Step 1 of classical MDS: Q = -1/2 P Delta P (Section 2)."""
    n = D.shape[0]
    P = centring_matrix(n)
    return -0.5 * (P @ D @ P)


def top_eigenpairs(Q, r):
    """Step 2-3 of classical MDS: eigenpairs sorted by decreasing eigenvalue,
    the r largest kept.  LAPACK's symmetric solver stands in for the paper's
    Lanczos routine; any accurate FP64 eigensolver gives the same pairs."""
    lam_all, vec_all = np.linalg.eigh(Q)
    order = np.argsort(-lam_all, kind="stable")[:r]
    return lam_all[order].copy(), vec_all[:, order].copy()


def sign_convention(V):
    """Make the largest-magnitude entry of every column positive (the first
    such entry when several tie)."""
    V = V.copy()
    for k in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, k])))
        if V[i, k] < 0:
            V[:, k] = -V[:, k]
    return V


def live_columns(lam):
    """Columns kept as "non-negative eigenvalues": lam_k > TAU * lam_1."""
    if not lam[0] > 0:
        raise DegenerateError("largest eigenvalue is not positive")
    return lam > TAU * lam[0]


def classical_mds(D, r):
    """Classical MDS of a full squared-distance matrix (Section 2).

    Returns (X, lam, V, live, Q) with X = V_r Lambda_r^{1/2} and dead columns
    zeroed."""
    Q = inner_products(D)
    lam, V = top_eigenpairs(Q, r)
    live = live_columns(lam)
    V = sign_convention(V)
    X = np.zeros_like(V)
    X[:, live] = V[:, live] * np.sqrt(lam[live])
    return X, lam, V, live, Q


def fit_landmarks(X, l, r, seed=0, idx=None):
    """Classical MDS on l landmarks of the data X (Section 3.1)."""
    X = np.asarray(X)
    n = X.shape[0]
    if idx is None:
        idx = np.asarray(sample_landmarks(n, l, seed), dtype=np.int64)
    else:
        idx = np.sort(np.asarray(idx, dtype=np.int64))
    M = X[idx].astype(np.float64)
    D1 = sqdist_rows(M, M)
    X1, lam, V, live, Q1 = classical_mds(D1, r)
    q = np.diag(Q1).copy()
    d1 = D1.mean(axis=1)
    dbar = float(D1.mean())
    return Fit(idx=idx, M=M, D1=D1, Q1=Q1, q=q, d1=d1, dbar=dbar, lam=lam,
               V=V, live=live, X1=X1, r_eff=int(live.sum()))


def gower_block(fit, A2):
    """Eq. (2) for one block: 1/(2l) (1 q1' - A21^2) X1 S1^{-1},
    S1 = Lambda/l (dead columns give zero)."""
    l = fit.M.shape[0]
    s1_inv = np.zeros_like(fit.lam)
    s1_inv[fit.live] = l / fit.lam[fit.live]
    return (1.0 / (2.0 * l)) * ((fit.q[None, :] - A2) @ fit.X1) * s1_inv[None, :]


def lmds_block(fit, A2):
    """Eq. (3): 1/2 (1 d1' - A21^2) V Lambda^{-1/2} (dead columns zero)."""
    scale = np.zeros_like(fit.lam)
    scale[fit.live] = 1.0 / np.sqrt(fit.lam[fit.live])
    return 0.5 * ((fit.d1[None, :] - A2) @ fit.V) * scale[None, :]


def interpolate(fit, Xnew, block=None, formula=gower_block, expanded=None):
    """Gower interpolation of every row of Xnew, in blocks of m = l rows.

    Distances are direct differences unless the block is large
    (n*l*p > 1e9), where the expanded FP64 form is used; ``expanded`` forces
    either choice."""
    Xnew = np.asarray(Xnew)
    n_new = Xnew.shape[0]
    l, p = fit.M.shape
    m = l if block is None else int(block)
    if expanded is None:
        expanded = n_new * l * p > 1e9
    dist = sqdist_rows_expanded if expanded else sqdist_rows
    Y = np.empty((n_new, fit.lam.shape[0]))
    for s in range(0, n_new, m):
        rows = Xnew[s:s + m].astype(np.float64)
        Y[s:s + m] = formula(fit, dist(rows, fit.M))
    return Y


def fit_from_sqdist(D1, r):
    """Classical MDS of l points given only their l x l squared
    dissimilarities (Section 2 starts from such a matrix; it need not come
    from Euclidean vectors, so Q1 may have negative eigenvalues)."""
    D1 = np.asarray(D1, dtype=np.float64)
    l = D1.shape[0]
    X1, lam, V, live, Q1 = classical_mds(D1, r)
    return Fit(idx=np.arange(l, dtype=np.int64), M=np.zeros((l, 0)), D1=D1, Q1=Q1,
               q=np.diag(Q1).copy(), d1=D1.mean(axis=1), dbar=float(D1.mean()), lam=lam, V=V,
               live=live, X1=X1, r_eff=int(live.sum()))


def interpolate_sqdist(fit, A2, formula=None):
    """Eq. (2) for new points given their squared dissimilarities A2 (m x l)
    to the landmarks."""
    formula = gower_block if formula is None else formula
    return formula(fit, np.asarray(A2, dtype=np.float64))


def affine_map(fit):
    """For squared Euclidean distances eq. (2) is an affine map of x.  With
    the centred landmarks Mc = M - 1 mbar' (mbar their mean) classical MDS of
    the landmarks is their principal-component analysis (Section 2), and
    Gower's formula is the projection y = Lambda^{-1/2} V' Mc (x - mbar)
    (derived from eq. (2) with V'1 = 0).  Returns (A, b) with y = A x + b:
    A = Lambda^{-1/2} V' Mc (r x p), b = -A mbar; dead columns give zero
    rows."""
    M = fit.M
    mbar = M.mean(axis=0)
    scale = np.where(fit.live, 1.0 / np.sqrt(np.where(fit.live, fit.lam, 1.0)), 0.0)
    A = scale[:, None] * (fit.V.T @ (M - mbar))
    return A, -A @ mbar


def interpolate_affine(fit, Xnew):
    """Rows of Xnew through the affine form of eq. (2) (Euclidean input
    only); every row, in input order."""
    A, b = affine_map(fit)
    return np.asarray(Xnew, dtype=np.float64) @ A.T + b


def interpolation_mds(X, l, r, seed=0, idx=None):
    """Interpolation MDS of the data X: fit on l landmarks, then interpolate
    all n rows (landmarks included) in input order."""
    fit = fit_landmarks(X, l, r, seed=seed, idx=idx)
    return interpolate(fit, X), fit


def interpolation_mds_paper_layout(X, l, r, seed=0):
    """The paper's assembly (Section 3.1): X1 for the landmark subset and
    eq. (2) for every other row, each row returned at its input position."""
    fit = fit_landmarks(X, l, r, seed=seed)
    n = X.shape[0]
    rest = np.setdiff1d(np.arange(n), fit.idx)
    Y = np.empty((n, fit.lam.shape[0]))
    Y[fit.idx] = fit.X1
    if rest.size:
        Y[rest] = interpolate(fit, X[rest])
    return Y, fit
