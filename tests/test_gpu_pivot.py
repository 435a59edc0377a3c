"""MaxMin landmarks and pivot MDS through the C ABI against the FP64 oracle
(needs a GPU): MaxMin indices must match exactly, pivot MDS to FP64
tolerances."""

import numpy as np
import pytest

import oracle
from oracle import pivot as opv
from synth import errors
from synth import generators as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_Y = 1e-9
TOL_LAM = 1e-12


def mds():
    import paper_2007_11919_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("name,make,l,first", [
    ("gaussian", lambda: gen.small_gaussian(5000, seed=1), 50, 0),
    ("ragged n, fp32", lambda: gen.wide_gaussian(3001, seed=2), 40, 17),
    ("integer image rows", lambda: gen.image_mixture(2000, p=784, seed=3).astype(np.float64), 30, 5),
    ("one landmark", lambda: gen.small_gaussian(100, seed=4), 1, 9),
], ids=lambda v: v if isinstance(v, str) else "")
def test_maxmin_matches_oracle(name, make, l, first):
    X = make()
    idx = mds().maxmin_landmarks(dev(X), l, first)
    ref = opv.maxmin_landmarks(X.astype(np.float64), l, first)
    assert np.array_equal(idx, ref), (idx[:10], ref[:10])


@pytest.mark.parametrize("p,extra,n", [
    (12, 0, 1000),    # 16-byte row loads, ragged chunk and ragged last block
    (128, 0, 777),    # whole chunks only
    (64, 4, 900),     # 16-byte aligned strided rows
    (10, 0, 1000),    # p % 4 != 0: single-column loads
    (132, 0, 700),    # a ragged fifth chunk
], ids=["p12", "p128", "p64-strided", "p10", "p132"])
def test_maxmin_fp32_layouts(p, extra, n):
    """FP32 rows through both load paths of the MaxMin step (bit-exact indices)."""
    rng = np.random.Generator(np.random.PCG64(p + n))
    Xw = rng.standard_normal((n, p + extra)).astype(np.float32)
    X = np.ascontiguousarray(Xw[:, :p])
    idx = mds().maxmin_landmarks(dev(Xw)[:, :p], 30, 4)
    assert np.array_equal(idx, opv.maxmin_landmarks(X.astype(np.float64), 30, 4))


def test_maxmin_strided_and_duplicates():
    X = gen.small_gaussian(700, seed=5)
    wide = np.zeros((700, 13))
    wide[:, :10] = X
    idx = mds().maxmin_landmarks(dev(wide)[:, :10], 25, 3)
    assert np.array_equal(idx, opv.maxmin_landmarks(X, 25, 3))
    D = np.zeros((50, 3))
    D[7] = 1.0
    with pytest.raises(mds().MDSError) as ei:
        mds().maxmin_landmarks(dev(D), 3, 0)
    assert ei.value.status == 4


def constant_column(n, seed):
    """Wide rows with one zero-variance column: the covariance is singular,
    so its Cholesky factor does not exist and the l x l route is taken."""
    X = gen.wide_gaussian(n, seed=seed).astype(np.float64)
    X[:, 5] = 3.0
    return X


def compare_pivot(X, l, r, seed=0, idx=None, dtype=np.float64):
    Xs = X.astype(dtype)
    Y, lam, r_eff = mds().pivot_mds(dev(Xs), l, r, seed=seed, idx=idx)
    pidx = np.asarray(idx) if idx is not None else np.array(oracle.sample_landmarks(X.shape[0], l, seed))
    Yo, lamo, _ = opv.pivot_mds(Xs.astype(np.float64), pidx, r)
    assert np.max(np.abs(lam - lamo)) <= TOL_LAM * lamo[0], (lam, lamo)
    e = errors.column_errors(Y.cpu().numpy(), Yo)
    assert e["maxabs_rms"] <= TOL_Y, e
    assert r_eff == int(np.sum(lamo > oracle.TAU * lamo[0]))
    return Y.cpu().numpy(), lam


@pytest.mark.parametrize("name,make,l,r", [
    ("paper design, l=200", lambda: gen.paper_design(20000, 10, 2, seed=6), 200, 2),
    ("wide, l x l route, eigen in registers", lambda: gen.wide_gaussian(8000, seed=7).astype(np.float64), 80, 10),
    ("wide, l x l route, l = 30", lambda: gen.wide_gaussian(6000, seed=17).astype(np.float64), 30, 8),
    ("wide, p x p route", lambda: gen.wide_gaussian(8000, seed=8).astype(np.float64), 300, 10),
    ("constant column: l x l route, eigen in global memory", lambda: constant_column(8000, 13), 300, 10),
    ("rank below r", lambda: gen.small_gaussian(2000, seed=9)[:, :3], 50, 5),
    ("all rows are pivots", lambda: gen.small_gaussian(150, seed=10), 150, 3),
], ids=lambda v: v if isinstance(v, str) else "")
def test_pivot_matches_oracle(name, make, l, r):
    X = make()
    Y, _ = compare_pivot(X, l, r, seed=3)
    if name == "rank below r":
        assert np.all(Y[:, 3:] == 0.0)


@pytest.mark.parametrize("p,n,l,dtype", [
    (17, 3001, 40, np.float64),    # one whole and one ragged 16-column tile; ragged row steps
    (128, 5000, 60, np.float32),   # the largest p of the matrix-core covariance: 8 x 8 tiles
    (129, 4000, 60, np.float64),   # the smallest p of the vector covariance kernel
    (300, 4000, 350, np.float32),  # vector covariance over several 64 x 64 tiles
], ids=["p17", "p128-fp32", "p129", "p300-fp32"])
def test_pivot_covariance_shapes(p, n, l, dtype):
    """Column counts on both sides of the covariance kernel choice."""
    k = min(p, 10)
    sig = np.concatenate([np.linspace(10.0, 2.0, k), np.ones(p - k)])
    X = gen.gaussian_columns(n, sig, seed=p, dtype=dtype)
    compare_pivot(X, l, 10, seed=1, dtype=dtype)


def test_pivot_with_maxmin_pivots_and_fp32():
    X = gen.wide_gaussian(6000, seed=11)
    idx = mds().maxmin_landmarks(dev(X), 120, 0)
    compare_pivot(X, 120, 10, idx=idx, dtype=np.float32)


def test_pivot_full_size_sampled_rows():
    """n = 10^6 rows of the 100-column workload, l = 200 random pivots (the
    pivot MDS setting of Section 4.1), r = 10; rows sampled for the check."""
    X = gen.wide_gaussian(1_000_000, seed=12)
    Y, lam, _ = mds().pivot_mds(dev(X), 200, 10, seed=4)
    pidx = np.array(oracle.sample_landmarks(1_000_000, 200, 4))
    rows = np.sort(np.random.default_rng(0).choice(1_000_000, 3000, replace=False))
    Yo, lamo, _ = opv.pivot_mds_large(X, pidx, 10, rows=rows)
    assert np.max(np.abs(lam - lamo)) <= 1e-10 * lamo[0], (lam, lamo)
    e = errors.column_errors(Y.cpu().numpy()[rows], Yo)
    assert e["maxabs_rms"] <= 1e-8, e


@pytest.mark.parametrize("ratio,live", [(1e-3, False), (10 ** -2.75, False),
                                        (10 ** -2.125, True), (1e-1, True)])
def test_pivot_live_threshold(ratio, live):
    """Liveness on the eigenvalues of C'C (sigma_k^2 > TAU sigma_1^2), as in
    the oracle: points in R^2 with every point a pivot, so C = Q has
    singular values 1 and ratio^2.  The dead cases have sigma_2 / sigma_1
    between TAU and sqrt(TAU).  A direction this close to the threshold is
    only resolved to about eps sigma_1^2 / sigma_2^2 through C'C, so live
    columns are compared to 1e-6."""
    rng = np.random.default_rng(9)
    Z = rng.standard_normal((20, 2))
    Z -= Z.mean(axis=0)
    H, _ = np.linalg.qr(Z)
    X = H * np.array([1.0, ratio]) + np.array([3.0, -2.0])
    idx = np.arange(20)
    Y, lam, r_eff = mds().pivot_mds(dev(X), 20, 2, idx=idx)
    Yo, lamo, _ = opv.pivot_mds(X, idx, 2)
    Y = Y.cpu().numpy()
    assert r_eff == (2 if live else 1)
    assert abs(lam[0] - lamo[0]) <= 1e-12
    if live:
        assert abs(lam[1] / lamo[1] - 1.0) <= 1e-6, (lam, lamo)
        e = errors.column_errors(Y, Yo)
        assert e["maxabs_rms"] <= 1e-6, e
    else:
        assert lam[1] == 0.0 and np.all(Y[:, 1] == 0.0)


def test_pivot_error_codes():
    m = mds()
    X = dev(gen.small_gaussian(300, seed=13))
    for l, r in [(1, 1), (50, 50), (301, 2), (3000, 2)]:
        with pytest.raises(m.MDSError) as ei:
            m.pivot_mds(X, l, r)
        assert ei.value.status == 1, (l, r)
    with pytest.raises(m.MDSError) as ei:
        m.pivot_mds(X, 10, 2, idx=np.array([1, 2, 3, 4, 5, 6, 7, 8, 9, 9]))
    assert ei.value.status == 1
    bad = gen.small_gaussian(300, seed=13)
    bad[5, 1] = np.inf
    with pytest.raises(m.MDSError) as ei:
        m.pivot_mds(dev(bad), 20, 2)
    assert ei.value.status == 1
