"""HIP library against the FP64 oracle, through the C ABI (needs a GPU).

Tolerances (tests/tolerance.py; per output column, dead columns exactly
zero): FP64 1e-9, FP32 and split 1e-4, on both the RMS-relative and the
max-abs / RMS reading; every case here has r columns among the data's
strong directions.  Landmark indices are compared bit for bit, eigenvalues
to 1e-12 relative, landmark coordinates X1 to 1e-10 of their largest entry.
"""

import numpy as np
import pytest

import oracle
from synth import generators as gen

from . import tolerance

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def mds():
    import paper_2007_11919_amd as m
    return m


def dev(X):
    return torch.from_numpy(np.ascontiguousarray(X)).cuda()


def embed_np(model, Xd, prec):
    if prec != "fp64" and Xd.dtype != torch.float32:
        Xd = Xd.float()
    Y = mds().embed(model, Xd, prec=prec)
    torch.cuda.synchronize()
    return Y.cpu().numpy().astype(np.float64)


def check_fit(model, fit):
    assert np.array_equal(model.landmarks(), fit.idx)
    lam = model.eigenvalues()
    assert np.max(np.abs(lam - fit.lam)) <= 1e-12 * fit.lam[0]
    X1 = model.landmark_coords()
    assert np.max(np.abs(X1 - fit.X1)) <= 1e-10 * np.max(np.abs(fit.X1))
    q = model.q()
    assert np.max(np.abs(q - fit.q)) <= 1e-12 * np.max(np.abs(fit.q))
    assert model.r_eff == fit.r_eff


def check_embed(Y, Yo, prec):
    return tolerance.check_embed(Y, Yo, prec)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_small_fp64(seed):
    """5,000 x 10 FP64 Gaussian rows, std (15, 10, 1, ...), l = 200, r = 2."""
    X = gen.small_gaussian(5000, seed=11)
    model = mds().fit_landmarks(dev(X), 200, 2, seed=seed)
    fit = oracle.fit_landmarks(X, 200, 2, seed=seed)
    check_fit(model, fit)
    Yo = oracle.interpolate(fit, X)
    check_embed(embed_np(model, dev(X), "fp64"), Yo, "fp64")
    for prec in ("fp32", "split_bf16", "split_fp16"):
        check_embed(embed_np(model, dev(X), prec), Yo, prec)


def test_wide_all_precisions():
    """100 columns (std 20..2 then 1), l = 1000, r = 10, ragged row count."""
    X = gen.wide_gaussian(20037, seed=12)
    model = mds().fit_landmarks(dev(X), 1000, 10, seed=1)
    fit = oracle.fit_landmarks(X, 1000, 10, seed=1)
    check_fit(model, fit)
    Yo = oracle.interpolate(fit, X)
    Xd = dev(X)
    check_embed(embed_np(model, Xd, "fp64"), Yo, "fp64")
    for prec in ("fp32", "split_bf16", "split_fp16"):
        check_embed(embed_np(model, Xd, prec), Yo, prec)


def test_image_mixture_all_precisions():
    """784 integer-valued columns, l = 2000, r = 10 (image-like mixture)."""
    X = gen.image_mixture(3000, seed=13)
    model = mds().fit_landmarks(dev(X), 2000, 10, seed=2)
    fit = oracle.fit_landmarks(X, 2000, 10, seed=2)
    check_fit(model, fit)
    Yo = oracle.interpolate(fit, X)
    Xd = dev(X)
    check_embed(embed_np(model, Xd, "fp64"), Yo, "fp64")
    for prec in ("fp32", "split_bf16", "split_fp16"):
        check_embed(embed_np(model, Xd, prec), Yo, prec)


def _sampled_rows(n, rng, k=3000):
    rows = np.unique(np.concatenate([
        rng.choice(n, size=k, replace=False), np.arange(128), np.arange(n - 200, n)]))
    return rows


@pytest.mark.parametrize("which", ["wide", "image"])
def test_full_size_sampled(which):
    """10^6 rows at the benchmark's shapes; every row is embedded on the GPU
    in the benchmark's launch configuration and the oracle checks a sample
    of rows one by one (plus the first and last tiles)."""
    if which == "wide":
        X = gen.wide_gaussian(1_000_000, seed=12)
        l, r, seed = 1000, 10, 0
    else:
        X = gen.image_mixture(1_000_000, seed=13)
        l, r, seed = 2000, 10, 0
    Xd = dev(X)
    model = mds().fit_landmarks(Xd, l, r, seed=seed)
    fit = oracle.fit_landmarks(X, l, r, seed=seed)
    check_fit(model, fit)
    rows = _sampled_rows(X.shape[0], np.random.Generator(np.random.PCG64(3)))
    Yo = oracle.interpolate(fit, X[rows])
    for prec in ("fp32", "split_bf16"):
        Y = mds().embed(model, Xd, prec=prec)
        torch.cuda.synchronize()
        Ys = Y[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(Y.cpu().numpy()))
        check_embed(Ys, Yo, prec)
        del Y
    Yd = mds().embed(model, Xd[torch.from_numpy(rows).cuda()].contiguous(), prec="fp64")
    check_embed(Yd.cpu().numpy(), Yo, "fp64")


def test_landmark_self_reproduction():
    """Interpolating a landmark gives its classical-MDS coordinate X1."""
    X = gen.wide_gaussian(5000, seed=21).astype(np.float64)
    model = mds().fit_landmarks(dev(X), 400, 6, seed=5)
    idx = model.landmarks()
    Y = embed_np(model, dev(X[idx]), "fp64")
    X1 = model.landmark_coords()
    assert np.max(np.abs(Y - X1)) <= 1e-9 * np.max(np.abs(X1))


def test_l_equals_n_is_classical_mds():
    """l = n: the GPU result is classical MDS of all points, checked against
    the brute-force Jacobi solution."""
    from tests.pins import brute_classical_mds
    X = gen.gaussian_columns(40, np.array([5.0, 3.0, 2.0, 1.0, 0.5]), 3, dtype=np.float64)
    model = mds().fit_landmarks(dev(X), 40, 3, seed=0)
    Y = embed_np(model, dev(X), "fp64")
    Xb, lamb = brute_classical_mds(X, 3)
    assert np.max(np.abs(model.eigenvalues() - lamb)) <= 1e-10 * lamb[0]
    assert np.max(np.abs(Y - Xb)) <= 1e-9 * np.max(np.abs(Xb))


def test_exact_recovery_of_low_dimensional_data():
    """Points in a 3-dimensional affine subspace of R^12 are reproduced up to
    an isometry: all pairwise distances survive."""
    X, _ = gen.low_rank(3000, 12, 3, seed=5)
    model = mds().fit_landmarks(dev(X), 100, 3, seed=1)
    Y = embed_np(model, dev(X), "fp64")
    sub = np.arange(0, 3000, 13)
    dx = oracle.sqdist_rows(X[sub], X[sub])
    dy = oracle.sqdist_rows(Y[sub], Y[sub])
    assert np.max(np.abs(dx - dy)) <= 1e-9 * np.max(dx)


def test_repeated_eigenvalues():
    """A 3-D grid is isotropic: lambda_1 = lambda_2 = lambda_3 exactly.  A
    single Krylov run sees one copy of a repeated eigenvalue, so the solver
    must restart; distances are preserved whatever basis it picks."""
    g = np.arange(3.0)
    X = np.array([[a, b, c] for a in g for b in g for c in g])
    model = mds().fit_landmarks(dev(X), 27, 3, seed=0)
    lam = model.eigenvalues()
    fit = oracle.fit_landmarks(X, 27, 3, seed=0)
    assert np.max(np.abs(lam - fit.lam)) <= 1e-10 * fit.lam[0]
    Y = embed_np(model, dev(X), "fp64")
    dx = oracle.sqdist_rows(X, X)
    dy = oracle.sqdist_rows(Y, Y)
    assert np.max(np.abs(dx - dy)) <= 1e-9 * np.max(dx)


def test_rank_deficient_columns_exactly_zero():
    X, _ = gen.low_rank(2000, 8, 3, seed=7)
    model = mds().fit_landmarks(dev(X), 300, 5, seed=4)
    fit = oracle.fit_landmarks(X, 300, 5, seed=4)
    assert model.r_eff == 3 == fit.r_eff
    Yo = oracle.interpolate(fit, X)
    Xd = dev(X)
    for prec in ("fp64", "fp32", "split_bf16", "split_fp16"):
        Y = embed_np(model, Xd, prec)
        assert np.all(Y[:, 3:] == 0.0)
        check_embed(Y, Yo, prec)


@pytest.mark.parametrize("p", [1, 3, 10, 33, 130])
@pytest.mark.parametrize("r", [1, 16, 17, 35])
def test_shapes(p, r):
    """Odd p (scalar loads, ragged chunks), l not a multiple of the tile,
    r across one, two and four 16-column blocks, ragged n, strided rows."""
    n, l = 1000, 130
    if r >= l or r > p + 5:
        r = min(r, p)
    sig = np.linspace(6.0, 1.0, p)
    Xw = gen.gaussian_columns(n, np.concatenate([sig, np.ones(7)]), 40 + p, dtype=np.float32)
    X = np.ascontiguousarray(Xw[:, :p])
    Xd_wide = dev(Xw)
    Xd = Xd_wide[:, :p]  # ldx = p + 7
    model = mds().fit_landmarks(Xd, l, r, seed=p)
    fit = oracle.fit_landmarks(X, l, r, seed=p)
    check_fit(model, fit)
    for m in (1, 127, 128, 129, n):
        Yo = oracle.interpolate(fit, X[:m])
        for prec in ("fp64", "fp32"):
            check_embed(embed_np(model, Xd[:m], prec), Yo, prec)


def test_zero_rows_is_noop():
    X = gen.wide_gaussian(500, seed=3)
    model = mds().fit_landmarks(dev(X), 100, 4, seed=0)
    Y = torch.full((0, 4), 7.0, device="cuda")
    out = mds().embed(model, dev(X)[:0], prec="fp32", Y=Y)
    assert out.shape == (0, 4)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "split_bf16", "split_fp16"])
def test_batch_invariance(prec):
    """A row's result is bit-identical alone, at any offset, in any batch."""
    X = gen.wide_gaussian(4000, seed=31)
    model = mds().fit_landmarks(dev(X), 500, 10, seed=3)
    Xd = dev(X)
    full = embed_np(model, Xd, prec)
    for s, k in [(0, 1), (5, 1), (77, 300), (128, 128), (1000, 2500), (3999, 1)]:
        part = embed_np(model, Xd[s:s + k], prec)
        assert np.array_equal(part, full[s:s + k]), (s, k)
    perm = np.random.Generator(np.random.PCG64(1)).permutation(4000)
    permuted = embed_np(model, Xd[torch.from_numpy(perm).cuda()].contiguous(), prec)
    assert np.array_equal(permuted, full[perm])


def test_deterministic_fit_and_embed():
    X = gen.image_mixture(2500, seed=17)
    a = mds().fit_landmarks(dev(X), 700, 10, seed=9)
    b = mds().fit_landmarks(dev(X), 700, 10, seed=9)
    assert np.array_equal(a.eigenvalues(), b.eigenvalues())
    assert np.array_equal(a.landmark_coords(), b.landmark_coords())
    Xd = dev(X)
    assert np.array_equal(embed_np(a, Xd, "fp32"), embed_np(b, Xd, "fp32"))


def test_duplicate_points():
    X = gen.wide_gaussian(300, seed=8)
    X = np.concatenate([X, X[:150]])  # duplicated rows, some become landmarks
    model = mds().fit_landmarks(dev(X), 200, 5, seed=2)
    fit = oracle.fit_landmarks(X, 200, 5, seed=2)
    check_fit(model, fit)
    Yo = oracle.interpolate(fit, X)
    check_embed(embed_np(model, dev(X), "fp64"), Yo, "fp64")


def test_given_landmarks():
    X = gen.wide_gaussian(2000, seed=9)
    idx = np.arange(1999, 0, -10)  # unsorted on purpose
    model = mds().fit_landmarks(dev(X), idx.size, 4, idx=idx)
    fit = oracle.fit_landmarks(X, idx.size, 4, idx=idx)
    check_fit(model, fit)


def test_error_codes_on_device():
    m = mds()
    X = gen.wide_gaussian(300, seed=4)
    with pytest.raises(m.MDSError) as ei:
        m.fit_landmarks(dev(np.ones((50, 3))), 10, 2)
    assert ei.value.status == 4  # degenerate
    Xbad = X.copy()
    idx = m.sample_landmarks(300, 50, 0)
    Xbad[idx[3], 2] = np.nan
    with pytest.raises(m.MDSError) as ei:
        m.fit_landmarks(dev(Xbad), 50, 2, seed=0)
    assert ei.value.status == 1
    model = m.fit_landmarks(dev(X), 50, 2, seed=0)
    with pytest.raises(m.MDSError) as ei:
        m.embed(model, dev(X).double(), prec="fp32")
    assert ei.value.status == 1
