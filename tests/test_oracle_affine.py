"""Pins of the affine form of Gower's formula (Euclidean input): it must
agree with eq. (2) computed from distances by direct differences, with the
principal-component projection obtained from an SVD, and reproduce data
that lie in R^r exactly."""

import numpy as np
import pytest

import oracle
from oracle import mds as om
from synth import generators as gen

from . import pins


def check_affine_vs_eq2(X, l, r, seed, tol=1e-10):
    fit = om.fit_landmarks(X, l, r, seed=seed)
    Yd = om.interpolate(fit, X)
    Ya = om.interpolate_affine(fit, X)
    assert pins._rel(Ya, Yd) < tol, pins._rel(Ya, Yd)


def check_affine_vs_svd(X, l, r, seed, tol=1e-10):
    fit = om.fit_landmarks(X, l, r, seed=seed)
    M = X[fit.idx].astype(np.float64)
    mbar = M.mean(axis=0)
    U, S, Rt = np.linalg.svd(M - mbar, full_matrices=False)
    R = Rt[:r].T.copy()
    for k in range(r):
        i = int(np.argmax(np.abs(U[:, k])))
        if U[i, k] < 0:
            R[:, k] = -R[:, k]
    Ysvd = (np.asarray(X, dtype=np.float64) - mbar) @ R
    Ya = om.interpolate_affine(fit, X)
    assert pins._rel(Ya, Ysvd) < tol, pins._rel(Ya, Ysvd)


def test_affine_equals_eq2():
    check_affine_vs_eq2(gen.small_gaussian(800, seed=3), 100, 3, seed=1)


def test_affine_equals_svd_projection():
    check_affine_vs_svd(gen.small_gaussian(600, seed=4), 90, 2, seed=2)


def test_affine_exact_on_low_rank_data():
    X, Z = gen.low_rank(400, 9, 3, seed=6)
    fit = om.fit_landmarks(X, 50, 3, seed=1)
    Y = om.interpolate_affine(fit, X)
    aligned, _, _ = oracle.procrustes(Z, Y)
    assert pins._rel(aligned, Z) < 1e-9


def test_dead_columns_are_zero():
    X = gen.small_gaussian(300, seed=5)[:, :2]
    fit = om.fit_landmarks(X, 40, 4, seed=3)
    A, b = om.affine_map(fit)
    assert fit.r_eff == 2
    assert np.all(A[2:] == 0) and np.all(b[2:] == 0)


@pytest.mark.parametrize("name", ["shift dropped", "no scaling", "sign of shift"])
def test_planted_mistakes(monkeypatch, name):
    def wrong(fit):
        M = fit.M
        mbar = M.mean(axis=0)
        scale = np.where(fit.live, 1.0 / np.sqrt(np.where(fit.live, fit.lam, 1.0)), 0.0)
        if name == "no scaling":
            scale = np.where(fit.live, 1.0, 0.0)
        A = scale[:, None] * (fit.V.T @ (M - mbar))
        if name == "shift dropped":
            return A, np.zeros(A.shape[0])
        return A, (A @ mbar if name == "sign of shift" else -A @ mbar)
    monkeypatch.setattr(om, "affine_map", wrong)
    X = gen.small_gaussian(500, seed=8)
    with pytest.raises(AssertionError):
        check_affine_vs_eq2(X, 80, 3, seed=1)
        check_affine_vs_svd(X, 80, 3, seed=1)
