"""Small dense helpers of the oracle (test infrastructure only).

* ``jacobi_eigh``: the cyclic Jacobi eigenvalue method for symmetric
  matrices (Jacobi 1846; textbook form in Golub and Van Loan, "Matrix
  Computations", Section 8.5), in plain Python loops.  It uses no LAPACK, so
  it gives an independent brute-force classical MDS for tiny n.
* ``procrustes``: orthogonal Procrustes alignment (Borg and Groenen, "Modern
  Multidimensional Scaling", Chapter 20), which the paper uses to compare
  configurations up to rotation and shift (Section 4.1).
"""

import math

import numpy as np


def jacobi_eigh(A, tol=1e-15, max_sweeps=60):
    """Eigenvalues and eigenvectors of a small symmetric matrix by cyclic
    Jacobi rotations.  Returns (lam, V) with A V = V diag(lam), unsorted."""
    a = [list(map(float, row)) for row in np.asarray(A, dtype=np.float64)]
    n = len(a)
    v = [[1.0 if i == j else 0.0 for j in range(n)] for i in range(n)]
    scale = math.sqrt(sum(x * x for row in a for x in row)) or 1.0
    for _ in range(max_sweeps):
        off = math.sqrt(sum(a[i][j] ** 2 for i in range(n) for j in range(n) if i != j))
        if off <= tol * scale:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = a[p][q]
                if abs(apq) <= 1e-300:
                    continue
                # rotation angle that annihilates a[p][q]
                theta = (a[q][q] - a[p][p]) / (2.0 * apq)
                t = math.copysign(1.0, theta) / (abs(theta) + math.sqrt(theta * theta + 1.0))
                c = 1.0 / math.sqrt(t * t + 1.0)
                s = t * c
                for k in range(n):
                    akp = a[k][p]
                    akq = a[k][q]
                    a[k][p] = c * akp - s * akq
                    a[k][q] = s * akp + c * akq
                for k in range(n):
                    apk = a[p][k]
                    aqk = a[q][k]
                    a[p][k] = c * apk - s * aqk
                    a[q][k] = s * apk + c * aqk
                for k in range(n):
                    vkp = v[k][p]
                    vkq = v[k][q]
                    v[k][p] = c * vkp - s * vkq
                    v[k][q] = s * vkp + c * vkq
    lam = np.array([a[i][i] for i in range(n)])
    return lam, np.array(v)


def procrustes(ref, X):
    """Rotation T (orthogonal) and shift t minimising |ref - (X T + 1 t')|.

    Returns (aligned, T, t)."""
    ref = np.asarray(ref, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    mr = ref.mean(axis=0)
    mx = X.mean(axis=0)
    U, _, Vt = np.linalg.svd((X - mx).T @ (ref - mr))
    T = U @ Vt
    t = mr - mx @ T
    return X @ T + t, T, t
