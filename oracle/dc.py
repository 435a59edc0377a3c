"""FP64 CPU oracle of divide-and-conquer MDS (test infrastructure only).

Nothing on the product path may import this module.

What it computes (Delicado and Pachon-Garcia, Section 3.2):

1. c connecting points are drawn at random; the other n - c points are
   split at random, without replacement, into parts of l - c points.  There
   are P = ceil(1 + (n - l) / (l - c)) parts (P = 1 when n <= l); every
   part holds the c connecting points plus its own points, so all parts
   have l points except perhaps the last.
2. Classical MDS (Section 2) runs on every part, giving an n_j x r
   configuration X_j and eigenvalues lambda^j.
3. Each X_j with j >= 2 is aligned to X_1 by the Procrustes transformation
   (rotation T_j, shift t_j) fitted on the c connecting rows; its own rows
   become X_j^a T_j + 1 t_j'.
4. The global configuration stacks X_1 and the aligned parts; the
   eigenvalue estimates are lambda_bar_i = (1/P) sum_j lambda_i^j / n_j.

Readings where the paper leaves a choice open (the library takes the same):
* the random split is one permutation of 0..n-1: row i gets the key
  k_i = the (i+1)-th output of SplitMix64 seeded with `seed` (Steele, Lea
  and Flood 2014), rows are ordered by (key, index), the first c rows of
  that order are the connecting points and the rest are cut, in order, into
  consecutive pieces of l - c;
* inside a part the rows come in that order, connecting points first;
* the Procrustes fit is orthogonal with a shift and no dilation (the paper
  names only T_j and t_j), over the live columns of X_1; the other columns
  of the output are zero;
* a part whose connecting rows do not fix the rotation (smallest singular
  value of the cross-product matrix <= 1e-9 of the largest) is an error;
* the output rows come back in input order instead of stacked by part;
* the eigenvalue estimates use the r eigenvalues as computed (dead ones
  included), as the fit reports them.
"""

from dataclasses import dataclass

import numpy as np

from .mds import DegenerateError, classical_mds, sqdist_rows
from .sampler import GAMMA, MASK64, MIX1, MIX2, SplitMix64

ALIGN_TOL = 1e-9


def partition_keys(n, seed):
    """k_i for i = 0..n-1: SplitMix64 advances its state by a constant, so
    its (i+1)-th output is the finaliser applied to seed + (i+1) gamma
    (mod 2^64).  Vectorised form of SplitMix64(seed).next() called n times."""
    i = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(int(seed) & MASK64) + i * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
    return z ^ (z >> np.uint64(31))


def partition_keys_sequential(n, seed):
    """The same keys drawn one by one from the generator (slow; small n)."""
    g = SplitMix64(seed)
    return [g.next() for _ in range(n)]


def num_parts(n, l, c):
    """P = ceil(1 + (n - l) / (l - c)), and 1 when n <= l (Section 3.2)."""
    if n <= l:
        return 1
    return 1 + -(-(n - l) // (l - c))


def partition(n, l, c, seed):
    """Row order (position -> row index) and the number of parts."""
    keys = partition_keys(n, seed)
    order = np.argsort(keys, kind="stable").astype(np.int64)
    return order, num_parts(n, l, c)


def part_rows(order, n, l, c, j):
    """Rows of part j (0-based): the connecting rows, then its own rows."""
    lo = c + j * (l - c)
    hi = min(c + (j + 1) * (l - c), n)
    if num_parts(n, l, c) == 1:
        hi = n
    return np.concatenate([order[:c], order[lo:hi]])


def procrustes_fit(A, B):
    """Orthogonal T and shift t minimising |A - (B T + 1 t')| (Procrustes
    rotation with translation, Borg and Groenen, Chapter 20): with
    C = (B - 1 b')' (A - 1 a') = U S W', T = U W' and t = a - T' b."""
    a = A.mean(axis=0)
    b = B.mean(axis=0)
    C = (B - b).T @ (A - a)
    U, s, Wt = np.linalg.svd(C)
    if not s[-1] > ALIGN_TOL * s[0]:
        raise DegenerateError("connecting points do not fix the Procrustes rotation")
    T = U @ Wt
    return T, a - T.T @ b


@dataclass
class DCResult:
    Y: np.ndarray          # (n, r) configuration, input row order
    lam_bar: np.ndarray    # (r,) eigenvalue estimates
    r_eff: int             # live columns of the first part
    order: np.ndarray      # (n,) position -> row
    P: int                 # number of parts
    lam_parts: dict        # part j -> (r,) eigenvalues
    sizes: dict            # part j -> n_j


def check_args(n, l, c, r):
    if r < 1:
        raise ValueError("need r >= 1")
    if c < r + 1:
        raise ValueError("need c >= r + 1 (Section 3.2)")
    if l <= c:
        raise ValueError("need l > c")
    if n <= c:
        raise ValueError("need n > c")


def part_mds(X, rows, r):
    """Classical MDS of one part (Section 2): squared distances by direct
    differences, Q = -1/2 P Delta P, top r eigenpairs, X_j = V Lambda^{1/2}."""
    M = X[rows]
    Xj, lam, _, live, _ = classical_mds(sqdist_rows(M, M), r)
    return Xj, lam, live


def dc_mds(X, l, c, r, seed, parts=None):
    """Divide-and-conquer MDS of the rows of X.

    With ``parts`` given (a set of part indices), only those parts and the
    first one are computed and only their rows of Y are filled (the others
    stay NaN); lam_bar is then None.  This keeps full-size checks cheap."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    check_args(n, l, c, r)
    order, P = partition(n, l, c, seed)
    todo = range(P) if parts is None else sorted(set(parts) | {0})
    Y = np.full((n, r), np.nan)
    lam_parts, sizes = {}, {}
    X0 = None
    r0 = 0
    for j in todo:
        if j >= P:
            raise ValueError("part index out of range")
        rows = part_rows(order, n, l, c, j)
        Xj, lam, live = part_mds(X, rows, r)
        lam_parts[j] = lam
        sizes[j] = len(rows)
        if j == 0:
            r0 = int(live.sum())
            X0 = Xj
            Y[rows] = Xj
            continue
        T, t = procrustes_fit(X0[:c, :r0], Xj[:c, :r0])
        own = np.zeros((len(rows) - c, r))
        own[:, :r0] = Xj[c:, :r0] @ T + t
        Y[rows[c:]] = own
    lam_bar = None
    if parts is None:
        lam_bar = sum(lam_parts[j] / sizes[j] for j in range(P)) / P
    return DCResult(Y, lam_bar, r0, order, P, lam_parts, sizes)
