"""Oracle pins for dissimilarity input (the problem as Section 2 states it:
an n x n matrix of squared dissimilarities, not necessarily Euclidean)."""

import numpy as np

import oracle
from oracle import mds as om
from synth import generators as gen

from .pins import _rel


def l1_sqdist(A, B):
    """Squared city-block distances: a dissimilarity that is not squared
    Euclidean, so Q1 has negative eigenvalues."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    return np.array([np.abs(B - a).sum(axis=1) ** 2 for a in A])


def test_euclidean_input_matches_vector_path():
    X = gen.small_gaussian(600, seed=3)
    fit_v = om.fit_landmarks(X, 80, 3, seed=2)
    fit_d = oracle.fit_from_sqdist(fit_v.D1, 3)
    assert _rel(fit_d.lam, fit_v.lam) < 1e-12
    assert _rel(fit_d.X1, fit_v.X1) < 1e-10
    A2 = om.sqdist_rows(X, fit_v.M)
    assert _rel(oracle.interpolate_sqdist(fit_d, A2), om.interpolate(fit_v, X)) < 1e-10


def test_non_euclidean_brute_force():
    """Classical MDS of a non-Euclidean matrix against cyclic Jacobi."""
    X = gen.small_gaussian(30, seed=4)
    D = l1_sqdist(X, X)
    fit = oracle.fit_from_sqdist(D, 3)
    n = D.shape[0]
    J = np.eye(n) - 1.0 / n
    lam_all, V = oracle.jacobi_eigh(-0.5 * J @ D @ J)
    order = np.argsort(-lam_all)
    assert lam_all[order][-1] < -1e-6 * lam_all[order][0]  # genuinely non-Euclidean
    assert _rel(fit.lam, lam_all[order][:3]) < 1e-10


def test_non_euclidean_self_reproduction_and_proposition_1():
    X = gen.small_gaussian(200, seed=5)
    D = l1_sqdist(X[:50], X[:50])
    fit = oracle.fit_from_sqdist(D, 4)
    # landmark rows reproduce X1 (only Q1 V = V Lambda is used)
    assert _rel(oracle.interpolate_sqdist(fit, D), fit.X1) < 1e-10
    A2 = l1_sqdist(X, X[:50])
    g = oracle.interpolate_sqdist(fit, A2)
    lm = oracle.interpolate_sqdist(fit, A2, formula=om.lmds_block)
    assert _rel(g, lm) < 1e-10
