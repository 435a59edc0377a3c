"""Pins of the divide-and-conquer oracle (Section 3.2) to facts outside its
own code: the published SplitMix64 outputs, brute-force partitions, the
single-part case against a Jacobi classical MDS, exact recovery of data
lying in R^r, invariance under rigid motions, a Procrustes fit of a known
motion, and the trace identity behind the eigenvalue estimates.  Planted
mistakes must break at least one of them."""

import json
import os
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle
from oracle import dc
from synth import generators as gen

from . import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_keys_are_splitmix64_outputs():
    with open(os.path.join(GOLDEN, "splitmix64_seed1234567.json")) as f:
        g = json.load(f)
    keys = dc.partition_keys(5, g["seed"])
    assert [int(k) for k in keys] == [int(s) for s in g["outputs"]]
    for seed in (0, 7, (1 << 64) - 3):  # last one wraps the state
        assert [int(k) for k in dc.partition_keys(40, seed)] == dc.partition_keys_sequential(40, seed)


def check_partition(n, l, c, seed):
    order, P = dc.partition(n, l, c, seed)
    keys = dc.partition_keys_sequential(n, seed)
    brute = sorted(range(n), key=lambda i: (keys[i], i))
    assert list(order) == brute, "order is not the key order"
    want = 1 if n <= l else math.ceil(1 + Fraction(n - l, l - c))
    assert P == want, (P, want)
    seen = []
    for j in range(P):
        rows = dc.part_rows(order, n, l, c, j)
        assert list(rows[:c]) == brute[:c], "connecting points must lead every part"
        if j < P - 1:
            assert len(rows) == l, "only the last part may be short"
        assert len(rows) > c
        seen.extend(rows[c:])
    assert sorted(seen + brute[:c]) == list(range(n)), "every row exactly once"


@pytest.mark.parametrize("n,l,c", [(1000, 120, 20), (50, 50, 5), (37, 60, 4), (401, 40, 11), (10, 9, 8)])
def test_partition_structure(n, l, c):
    check_partition(n, l, c, seed=3)


def test_single_part_is_classical_mds():
    """n <= l gives P = 1: the result is classical MDS of all rows
    (Section 3.2), here computed by brute force with the Jacobi method."""
    X = gen.gaussian_columns(22, np.array([4.0, 3.0, 2.0, 1.0, 0.5]), 9, dtype=np.float64)
    res = dc.dc_mds(X, 30, 5, 3, seed=4)
    assert res.P == 1
    Xb, lamb = pins.brute_classical_mds(X, 3)
    assert pins._rel(res.Y, Xb) < 1e-9
    assert pins._rel(res.lam_bar, lamb / 22) < 1e-12


def check_exact_recovery(n=900, p=6, r=3, l=100, c=10, seed=5, tol=1e-9):
    """Rows lying in an r-dimensional affine subspace: every part's classical
    MDS is an isometric copy, so after alignment all pairwise distances of
    the whole configuration equal those of the data."""
    X, Z = gen.low_rank(n, p, r, seed)
    res = dc.dc_mds(X, l, c, r, seed=seed)
    assert res.P > 3
    sub = np.arange(0, n, 5)
    dx = oracle.sqdist_rows(X[sub], X[sub])
    dy = oracle.sqdist_rows(res.Y[sub], res.Y[sub])
    assert pins._rel(dy, dx) < tol, f"distances not preserved: {pins._rel(dy, dx)}"
    aligned, _, _ = oracle.procrustes(Z, res.Y)
    assert pins._rel(aligned, Z) < 1e-8


def test_exact_recovery():
    check_exact_recovery()


def check_rigid_invariance(tol=1e-9):
    X = gen.small_gaussian(700, seed=21)[:, :6]
    rng = np.random.default_rng(2)
    R, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    shift = rng.standard_normal(6) * 50
    a = dc.dc_mds(X, 90, 12, 2, seed=8)
    b = dc.dc_mds(X @ R + shift, 90, 12, 2, seed=8)
    assert pins._rel(b.Y, a.Y) < tol, pins._rel(b.Y, a.Y)
    assert pins._rel(b.lam_bar, a.lam_bar) < 1e-12


def test_rigid_invariance():
    check_rigid_invariance()


def check_known_motion():
    """A = B T0 + 1 t0' with T0 orthogonal (a reflection included): the fit
    must return T0 and t0."""
    rng = np.random.default_rng(5)
    B = rng.standard_normal((15, 4))
    T0, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    if np.linalg.det(T0) > 0:
        T0[:, 0] = -T0[:, 0]
    t0 = rng.standard_normal(4)
    T, t = dc.procrustes_fit(B @ T0 + t0, B)
    assert np.max(np.abs(T - T0)) < 1e-12
    assert np.max(np.abs(t - t0)) < 1e-12


def test_procrustes_known_motion():
    check_known_motion()


def test_procrustes_degenerate():
    B = np.zeros((6, 2))
    B[:, 0] = np.arange(6.0)  # collinear in two dimensions
    with pytest.raises(oracle.DegenerateError):
        dc.procrustes_fit(B + 1.0, B)


def check_trace_identity(n=800, p=5, r=5, l=90, c=12, seed=6):
    """With r equal to the data rank the r eigenvalues of a part sum to
    trace(Q_j) = sum of squared distances of its rows to their mean; so
    sum_i lambda_bar_i = (1/P) sum_j (1/n_j) sum_{x in part j} |x - mean_j|^2,
    computed here from the raw rows alone."""
    X = gen.gaussian_columns(n, np.array([3.0, 2.5, 2.0, 1.5, 1.0]), seed, dtype=np.float64)
    res = dc.dc_mds(X, l, c, r, seed=seed)
    tot = 0.0
    for j in range(res.P):
        rows = dc.part_rows(res.order, n, l, c, j)
        M = X[rows]
        tot += np.sum((M - M.mean(axis=0)) ** 2) / len(rows)
    assert abs(res.lam_bar.sum() - tot / res.P) < 1e-10 * tot


def test_trace_identity():
    check_trace_identity()


def test_paper_design_statistics():
    """Section 4.1 design (h dominant columns of variance 15, the rest 1):
    the estimates lambda_bar are close to 15 and the configuration is
    highly correlated with the dominant columns after Procrustes."""
    X = gen.paper_design(20000, 10, 2, seed=31)
    res = dc.dc_mds(X, 400, 10, 2, seed=2)
    assert np.all(np.abs(res.lam_bar - 15.0) < 1.5), res.lam_bar
    aligned, _, _ = oracle.procrustes(X[:, :2], res.Y)
    for k in range(2):
        assert np.corrcoef(aligned[:, k], X[:, k])[0, 1] > 0.995


def test_sampled_parts_match_full_run():
    X = gen.small_gaussian(1500, seed=7)[:, :5]
    full = dc.dc_mds(X, 150, 15, 2, seed=1)
    part = dc.dc_mds(X, 150, 15, 2, seed=1, parts={3, 7})
    for j in (0, 3, 7):
        rows = dc.part_rows(full.order, 1500, 150, 15, j)
        own = rows if j == 0 else rows[15:]
        assert np.array_equal(part.Y[own], full.Y[own])


def test_argument_checks():
    X = np.zeros((30, 3))
    for l, c, r in [(10, 2, 2), (10, 10, 2), (40, 30, 2), (10, 3, 0)]:
        with pytest.raises(ValueError):
            dc.dc_mds(X, l, c, r, seed=0)


def _all_checks():
    return [
        lambda: check_partition(300, 40, 7, 2),
        lambda: check_exact_recovery(n=400, l=60, c=8),
        check_rigid_invariance,
        check_known_motion,
        lambda: check_trace_identity(n=300, l=60, c=8),
    ]


def _caught():
    for check in _all_checks():
        try:
            check()
        except (AssertionError, ValueError, IndexError, np.linalg.LinAlgError):
            return True
    return False


def _transposed_fit(A, B):
    a, b = A.mean(axis=0), B.mean(axis=0)
    U, _, Wt = np.linalg.svd((B - b).T @ (A - a))
    T = (U @ Wt).T
    return T, a - T.T @ b


def _no_shift_fit(A, B):
    a, b = A.mean(axis=0), B.mean(axis=0)
    U, _, Wt = np.linalg.svd((B - b).T @ (A - a))
    return U @ Wt, np.zeros_like(a)


def _wrong_shift_fit(A, B):
    a, b = A.mean(axis=0), B.mean(axis=0)
    U, _, Wt = np.linalg.svd((B - b).T @ (A - a))
    T = U @ Wt
    return T, a - T @ b


def _uncentred_fit(A, B):
    a, b = A.mean(axis=0), B.mean(axis=0)
    U, _, Wt = np.linalg.svd(B.T @ A)
    T = U @ Wt
    return T, a - T.T @ b


def _parts_plus_one(n, l, c):
    return _ORIG_NUM_PARTS(n, l, c) + 1


def _rows_without_connecting(order, n, l, c, j):
    rows = _ORIG_PART_ROWS(order, n, l, c, j)
    return np.concatenate([order[c:2 * c], rows[c:]])


def _reversed_keys(n, seed):
    return _ORIG_KEYS(n, seed)[::-1].copy()


_ORIG_PART_ROWS = dc.part_rows
_ORIG_KEYS = dc.partition_keys
_ORIG_NUM_PARTS = dc.num_parts


@pytest.mark.parametrize("name,target,fn", [
    ("rotation transposed", "procrustes_fit", _transposed_fit),
    ("shift dropped", "procrustes_fit", _no_shift_fit),
    ("shift with T instead of T'", "procrustes_fit", _wrong_shift_fit),
    ("cross-product not centred", "procrustes_fit", _uncentred_fit),
    ("connecting rows differ per part", "part_rows", _rows_without_connecting),
    ("keys assigned to the wrong rows", "partition_keys", _reversed_keys),
    ("one part too many", "num_parts", _parts_plus_one),
])
def test_planted_mistakes_are_caught(monkeypatch, name, target, fn):
    assert not _caught()
    monkeypatch.setattr(dc, target, fn)
    assert _caught(), f"mistake not caught: {name}"


def test_planted_mistake_in_estimator(monkeypatch):
    orig = dc.part_mds

    def halve_last(X, rows, r):
        Xj, lam, live = orig(X, rows, r)
        return Xj, lam * (0.5 if len(rows) < 60 else 1.0), live

    monkeypatch.setattr(dc, "part_mds", halve_last)
    with pytest.raises(AssertionError):
        check_trace_identity(n=300, l=60, c=8)
