"""Checks that pin the FP64 oracle to facts outside its own code.

Each ``check_*`` raises AssertionError when the oracle (as currently bound
in ``oracle.mds``) violates a fact fixed by the paper or by mathematics.
The normal tests call them on the real oracle; the mutation tests plant a
mistake in the oracle and require at least one check to fail.
"""

import itertools

import numpy as np

import oracle
from oracle import mds as om
from synth import generators as gen


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def check_self_reproduction(X, l, r, seed, tol=1e-10):
    """Interpolating a landmark returns its own classical-MDS coordinate:
    q - Delta_i. = 2 Q1[i, :] + const and Q1 V = V Lambda, V'1 = 0, so eq. (2)
    applied to landmark i gives X1[i, :] (Section 3.1)."""
    fit = om.fit_landmarks(X, l, r, seed=seed)
    Y = om.interpolate(fit, X[fit.idx])
    assert _rel(Y, fit.X1) < tol, f"landmark rows differ from X1: {_rel(Y, fit.X1)}"


def check_proposition_1(X, l, r, seed, tol=1e-10):
    """Proposition 1: the LMDS triangulation, eq. (3), equals eq. (2)."""
    fit = om.fit_landmarks(X, l, r, seed=seed)
    Yg = om.interpolate(fit, X, formula=om.gower_block)
    Yl = om.interpolate(fit, X, formula=om.lmds_block)
    assert _rel(Yg, Yl) < tol, f"eq.(2) vs eq.(3): {_rel(Yg, Yl)}"


def check_pca_closed_form(X, l, r, seed, tol=1e-9):
    """For squared Euclidean distances, classical MDS of the landmarks is the
    PCA of the centred landmark rows: Lambda = singular values squared, V =
    left singular vectors, and Gower's formula is the projection of x - mean
    onto the right singular vectors.  Computed by an SVD, with no distance
    matrix, centring matrix or eigensolver involved."""
    fit = om.fit_landmarks(X, l, r, seed=seed)
    M = X[fit.idx].astype(np.float64)
    mbar = M.mean(axis=0)
    U, S, Rt = np.linalg.svd(M - mbar, full_matrices=False)
    U = U[:, :r].copy()
    R = Rt[:r].T.copy()
    for k in range(r):
        i = int(np.argmax(np.abs(U[:, k])))
        if U[i, k] < 0:
            U[:, k] = -U[:, k]
            R[:, k] = -R[:, k]
    lam = S[:r] ** 2
    assert _rel(fit.lam, lam) < tol, f"eigenvalues vs SVD: {_rel(fit.lam, lam)}"
    assert _rel(fit.V, U) < 1e-7, f"eigenvectors vs SVD: {_rel(fit.V, U)}"
    Y = om.interpolate(fit, X)
    Ypca = (np.asarray(X, dtype=np.float64) - mbar) @ R
    assert _rel(Y, Ypca) < tol, f"embedding vs PCA projection: {_rel(Y, Ypca)}"


def check_exact_recovery(n=300, p=12, r=3, l=40, seed=5, tol=1e-9):
    """Points lying in an r-dimensional affine subspace are an exact
    Euclidean configuration (Section 2); interpolation MDS with r columns
    must reproduce all their pairwise distances."""
    X, Z = gen.low_rank(n, p, r, seed)
    Y, _ = om.interpolation_mds(X, l, r, seed=seed)
    sub = np.arange(0, n, 7)
    dx = om.sqdist_rows(X[sub], X[sub])
    dy = om.sqdist_rows(Y[sub], Y[sub])
    assert _rel(dy, dx) < tol, f"distances not preserved: {_rel(dy, dx)}"
    aligned, _, _ = oracle.procrustes(Z, Y)
    assert _rel(aligned, Z) < 1e-8, "Procrustes residual not ~0"


def brute_classical_mds(X, r):
    """Classical MDS written out with Python loops and the Jacobi method."""
    n = X.shape[0]
    D = [[float(sum((X[i, k] - X[j, k]) ** 2 for k in range(X.shape[1])))
          for j in range(n)] for i in range(n)]
    row = [sum(D[i]) / n for i in range(n)]
    col = [sum(D[i][j] for i in range(n)) / n for j in range(n)]
    tot = sum(row) / n
    Q = np.array([[-(D[i][j] - row[i] - col[j] + tot) / 2.0 for j in range(n)]
                  for i in range(n)])
    lam, V = oracle.jacobi_eigh(Q)
    order = sorted(range(n), key=lambda i: -lam[i])[:r]
    lam = lam[order]
    V = V[:, order]
    for k in range(r):
        i = max(range(n), key=lambda t: (abs(V[t, k]), -t))
        if V[i, k] < 0:
            V[:, k] = -V[:, k]
    return V * np.sqrt(lam), lam


def check_l_equals_n(n=24, p=5, r=3, seed=3, tol=1e-9):
    """With l = n interpolation MDS is classical MDS (Section 3.1, p = 1)."""
    X = gen.gaussian_columns(n, np.array([4.0, 3.0, 2.0, 1.0, 0.5]), seed,
                             dtype=np.float64)
    Y, fit = om.interpolation_mds(X, n, r, seed=seed)
    Xb, lamb = brute_classical_mds(X, r)
    assert _rel(fit.lam, lamb) < tol, f"eigenvalues vs Jacobi: {_rel(fit.lam, lamb)}"
    perm_Y = np.empty_like(Y)
    perm_Y[:] = Y
    assert _rel(perm_Y, Xb) < tol, f"l = n vs brute force: {_rel(perm_Y, Xb)}"


def check_centring(X, l, seed, tol=1e-10):
    """Double centring (Section 2, Section 3.1): Q1 has zero row and column
    sums, equals the element-wise formula -(d_ij - d_i. - d_.j + d_..)/2,
    equals the Gram matrix of the centred landmark rows, and q1 = d1 - dbar/2
    (the identity proved before Proposition 1)."""
    fit = om.fit_landmarks(X, l, 2, seed=seed)
    D, Q = fit.D1, fit.Q1
    scale = np.max(np.abs(Q))
    assert np.max(np.abs(Q.sum(axis=0))) < tol * scale * l
    assert np.max(np.abs(Q.sum(axis=1))) < tol * scale * l
    di = D.mean(axis=1)
    dj = D.mean(axis=0)
    dd = D.mean()
    Qe = -(D - di[:, None] - dj[None, :] + dd) / 2.0
    assert _rel(Q, Qe) < tol
    Mc = fit.M - fit.M.mean(axis=0)
    assert _rel(Q, Mc @ Mc.T) < tol
    assert _rel(fit.q, di - dd / 2.0) < tol


def check_eigen(X, l, r, seed, tol=1e-10):
    """Eigen-decomposition facts of Section 2 and eq. (1)."""
    fit = om.fit_landmarks(X, l, r, seed=seed)
    Q, V, lam = fit.Q1, fit.V, fit.lam
    nQ = np.linalg.norm(Q, 2)
    assert np.linalg.norm(Q @ V - V * lam) < tol * nQ
    assert np.max(np.abs(V.T @ V - np.eye(r))) < 1e-12
    assert np.max(np.abs(V.T @ np.ones(l))) < 1e-9
    assert np.all(np.diff(lam) <= 0), "eigenvalues not descending"
    # eq. (1): Var(X1) = X1'X1/l = Lambda/l, centred columns
    X1 = fit.X1
    assert _rel(X1.T @ X1 / l, np.diag(lam) / l) < 1e-9
    assert np.max(np.abs(X1.mean(axis=0))) < 1e-9 * np.sqrt(lam[0])
    lam_all, _ = om.top_eigenpairs(Q, l)
    assert abs(lam_all.sum() - np.trace(Q)) < 1e-9 * abs(np.trace(Q))


def check_integer_distances(seed=4, tol=0):
    """Integer data 0..255: Delta1 in FP64 is exact (sums below 2^53)."""
    X = gen.image_mixture(n=50, p=64, seed=seed, dtype=np.float32)
    M = X[:30].astype(np.int64)
    D = om.sqdist_rows(X[:30], X[:30])
    exact = np.array([[int(((M[i] - M[j]) ** 2).sum()) for j in range(30)]
                      for i in range(30)], dtype=np.float64)
    assert np.array_equal(D, exact)


def check_rigid_invariance(X, l, r, seed, tol=1e-8):
    """Distances, hence the whole method, are invariant under rotation and
    translation of the data; permuting rows permutes the output."""
    X = np.asarray(X, dtype=np.float64)
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    Rm, _ = np.linalg.qr(rng.standard_normal((X.shape[1], X.shape[1])))
    b = rng.uniform(-50, 50, size=X.shape[1])
    Y0, fit = om.interpolation_mds(X, l, r, seed=seed)
    Y1, _ = om.interpolation_mds(X @ Rm + b, l, r, idx=fit.idx)
    assert _rel(Y1, Y0) < tol, f"not rotation invariant: {_rel(Y1, Y0)}"
    perm = rng.permutation(X.shape[0])
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    Y2, _ = om.interpolation_mds(X[perm], l, r, idx=inv[fit.idx])
    assert _rel(Y2, Y0[perm]) < tol


class _NeedDraw(Exception):
    pass


def _enumerate_shuffles(n, l):
    """Run the partial Fisher-Yates once for every possible sequence of
    draws, branching over exactly the range each draw requests."""
    outcomes = []

    def run(path):
        pos = [0]
        asked = [None]

        def draw(k):
            if pos[0] < len(path):
                v = path[pos[0]]
                pos[0] += 1
                if not 0 <= v < k:
                    raise AssertionError("replayed draw out of range")
                return v
            asked[0] = k
            raise _NeedDraw

        try:
            out = oracle.fisher_yates_prefix(n, l, draw)
        except _NeedDraw:
            for v in range(asked[0]):
                run(path + [v])
            return
        outcomes.append(tuple(out))

    run([])
    return outcomes


def check_sampler_enumeration(n=5, l=3):
    """Partial Fisher-Yates: over all equally likely draw sequences every
    ordered l-tuple of distinct indices appears exactly once, so every
    l-subset is equally likely."""
    outcomes = _enumerate_shuffles(n, l)
    expected = set(itertools.permutations(range(n), l))
    assert len(outcomes) == len(expected), "wrong number of draw sequences"
    assert set(outcomes) == expected, "some ordered tuples missing or invalid"


def check_lemire_power_of_two(seed=99):
    """For k = 2^m Lemire's draw is the top m bits of the raw output (the
    rejection threshold (2^64 - k) mod k is 0)."""
    for m in (1, 5, 17, 40, 63):
        g1 = oracle.SplitMix64(seed)
        g2 = oracle.SplitMix64(seed)
        for _ in range(50):
            assert oracle.bounded(g1, 1 << m) == g2.next() >> (64 - m)
