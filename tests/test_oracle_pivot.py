"""Pins of the MaxMin and pivot MDS oracle to facts outside its own code:
MaxMin checked step by step by brute force and on points of a line whose
sequence is known; pivot MDS with every point as a pivot is classical MDS
(brute-force Jacobi); the double-centred block equals the inner products
of the centred points with the centred pivots; the configuration spans the
centred data for data in R^r; the eigenvalue estimates and correlations of
the Section 4.1 design."""


import numpy as np
import pytest

import oracle
from oracle import pivot as opv
from synth import generators as gen

from . import pins


def check_maxmin_brute(X, l, first):
    idx = opv.maxmin_landmarks(X, l, first)
    assert idx[0] == first and len(set(idx.tolist())) == l
    for s in range(1, l):
        chosen = idx[:s]
        best, arg = -1.0, -1
        for i in range(X.shape[0]):  # brute force over every candidate
            dm = min(float(np.sum((X[i] - X[j]) ** 2)) for j in chosen)
            if dm > best:
                best, arg = dm, i
        assert idx[s] == arg, (s, idx[s], arg)
    return idx


def test_maxmin_brute_force():
    check_maxmin_brute(gen.small_gaussian(60, seed=1), 12, 5)


def test_maxmin_integer_line():
    # ten points 0..9 on a line from 0: 9, then 4 (min(4, 5) = 4 ties with 5:
    # smaller index), then 2 or 6 ... the full greedy sequence by hand:
    # chosen {0, 9, 4}: best min distance 2 at 2, 6, 7 -> 2;
    # {0, 9, 4, 2}: min distances 1 at 1, 3, 5, 8, and 2 at 6, 7 -> 6;
    # {.., 6}: 1 at 1, 3, 5, 7, 8 -> 1; then 3, 5, 7, 8.
    X = np.arange(10, dtype=np.float64)[:, None]
    assert opv.maxmin_landmarks(X, 10, 0).tolist() == [0, 9, 4, 2, 6, 1, 3, 5, 7, 8]


def test_maxmin_duplicates_error():
    X = np.zeros((6, 2))
    X[3] = 1.0
    with pytest.raises(oracle.DegenerateError):
        opv.maxmin_landmarks(X, 3, 0)


def check_all_pivots_is_classical(n=18, r=3, seed=7, tol=1e-9):
    X = gen.gaussian_columns(n, np.array([4.0, 3.0, 2.0, 1.0]), seed, dtype=np.float64)
    Xb, lamb = pins.brute_classical_mds(X, r)
    for idx in (np.arange(n), np.random.default_rng(seed).permutation(n)):
        Y, lam, _ = opv.pivot_mds(X, idx, r)
        assert pins._rel(lam, lamb) < 1e-12, (lam, lamb)
        # column signs follow the pivot-space vectors: compare up to sign
        for k in range(r):
            sgn = np.sign(np.dot(Y[:, k], Xb[:, k]))
            assert pins._rel(sgn * Y[:, k], Xb[:, k]) < tol


def test_all_pivots_is_classical_mds():
    check_all_pivots_is_classical()


def check_block_is_centred_inner_products(seed=3):
    X = gen.small_gaussian(300, seed=seed)[:, :5]
    idx = np.array([3, 17, 40, 41, 77, 150, 299])
    C = opv.pivot_block(X, idx)
    Xc = X - X.mean(axis=0)
    Mc = X[idx] - X[idx].mean(axis=0)
    assert pins._rel(C, Xc @ Mc.T) < 1e-12


def test_block_is_centred_inner_products():
    check_block_is_centred_inner_products()


def check_span(seed=4):
    X, _ = gen.low_rank(500, 7, 3, seed)
    idx = opv.maxmin_landmarks(X, 40, 0)
    Y, _, _ = opv.pivot_mds(X, idx, 3)
    Xc = X - X.mean(axis=0)
    G, *_ = np.linalg.lstsq(Xc, Y, rcond=None)
    assert pins._rel(Xc @ G, Y) < 1e-10


def test_configuration_spans_centred_data():
    check_span()


def test_paper_design_statistics():
    """Random pivots, as the scale estimate lambda = sigma sqrt(n / l)
    assumes pivots representative of the data (MaxMin pivots are not: they
    favour extreme points and inflate the estimates)."""
    X = gen.paper_design(20000, 10, 2, seed=11)
    idx = np.array(oracle.sample_landmarks(20000, 200, 5))
    Y, lam, _ = opv.pivot_mds(X, idx, 2)
    assert np.all(np.abs(lam / X.shape[0] - 15.0) < 1.5), lam / X.shape[0]
    aligned, _, _ = oracle.procrustes(X[:, :2], Y)
    for k in range(2):
        assert np.corrcoef(aligned[:, k], X[:, k])[0, 1] > 0.99


def _all_checks():
    return [
        lambda: check_maxmin_brute(gen.small_gaussian(40, seed=2), 8, 0),
        check_all_pivots_is_classical,
        check_block_is_centred_inner_products,
        check_span,
    ]


def _caught():
    for c in _all_checks():
        try:
            c()
        except (AssertionError, ValueError, IndexError, np.linalg.LinAlgError):
            return True
    return False


_ORIG_BLOCK = opv.pivot_block
_ORIG_SQ = opv.sqdist_to


def _block_wrong_sign(X, idx):
    return -_ORIG_BLOCK(X, idx)


def _block_no_grand_mean(X, idx):
    X = np.asarray(X, dtype=np.float64)
    D = np.stack([_ORIG_SQ(X, X[j]) for j in idx], axis=1)
    return -0.5 * (D - D.mean(axis=1)[:, None] - D.mean(axis=0)[None, :])


def _sq_abs(X, m):
    return np.sum(np.abs(np.asarray(X, dtype=np.float64) - m), axis=1)


@pytest.mark.parametrize("name,target,fn", [
    ("block sign", "pivot_block", _block_wrong_sign),
    ("grand mean dropped", "pivot_block", _block_no_grand_mean),
    ("L1 instead of squared distances", "sqdist_to", _sq_abs),
])
def test_planted_mistakes_are_caught(monkeypatch, name, target, fn):
    assert not _caught()
    monkeypatch.setattr(opv, target, fn)
    assert _caught(), name


def test_planted_mistake_in_scale(monkeypatch):
    orig = opv.pivot_mds

    def no_scale(X, idx, r):
        Y, lam, W = orig(X, idx, r)
        l, n = len(idx), np.asarray(X).shape[0]
        return Y * (l / n) ** 0.25, lam * np.sqrt(l / n), W

    monkeypatch.setattr(opv, "pivot_mds", no_scale)
    with pytest.raises(AssertionError):
        test_paper_design_statistics()


def _two_scale_points(ratio, n=20, seed=9):
    """n points in R^2 whose centred coordinates are orthogonal columns of
    norms 1 and ratio (so with every point as a pivot C = Q has singular
    values 1 and ratio^2), shifted away from the origin."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, 2))
    Z -= Z.mean(axis=0)
    H, _ = np.linalg.qr(Z)
    return H * np.array([1.0, ratio]) + np.array([3.0, -2.0]), H


@pytest.mark.parametrize("ratio,live", [
    (1e-3, False),    # sigma_2 / sigma_1 = 1e-6: between TAU and sqrt(TAU)
    (10 ** -2.75, False),  # sigma ratio 10^-5.5, eigenvalue ratio of C'C 1e-11
    (10 ** -2.125, True),  # sigma ratio 10^-4.25, eigenvalue ratio 10^-8.5
    (1e-1, True),
])
def test_live_threshold_on_eigenvalues_of_ctc(ratio, live):
    """The eigenvalue test of Section 2 applied to C'C: sigma_k^2 > TAU
    sigma_1^2.  The two dead cases have sigma_2 / sigma_1 above TAU, so a
    test on sigma (or on lambda = sigma sqrt(n / l)) would keep them."""
    X, H = _two_scale_points(ratio)
    n = X.shape[0]
    for Y, lam in [opv.pivot_mds(X, np.arange(n), 2)[:2],
                   opv.pivot_mds_large(X, np.arange(n), 2, chunk=7)[:2]]:
        # all points as pivots: lambda are the eigenvalues of Q, 1 and ratio^2
        assert abs(lam[0] - 1.0) < 1e-12
        if live:
            # the chunked route takes sigma from the eigenvalues of C'C, good
            # to about eps sigma_1^2 / (2 sigma_2^2) relative
            assert abs(lam[1] / ratio ** 2 - 1.0) < 1e-6
            sgn = np.sign(np.dot(Y[:, 1], H[:, 1]))
            assert pins._rel(sgn * Y[:, 1], ratio * H[:, 1]) < 1e-6
        else:
            assert lam[1] == 0.0 and np.all(Y[:, 1] == 0.0)


def test_large_route_matches_direct():
    X = gen.small_gaussian(3000, seed=21)[:, :6]
    idx = np.array(oracle.sample_landmarks(3000, 60, 2))
    Y, lam, W = opv.pivot_mds(X, idx, 3)
    rows = np.array([0, 5, 1000, 2999])
    Yl, laml, Wl = opv.pivot_mds_large(X, idx, 3, rows=rows, chunk=700)
    assert pins._rel(laml, lam) < 1e-12
    assert pins._rel(Wl, W) < 1e-9
    assert pins._rel(Yl, Y[rows]) < 1e-9
