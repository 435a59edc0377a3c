"""Affine form of eq. (2) through the C ABI (needs a GPU): against the
oracle's principal-component form and against the distance path."""

import numpy as np
import pytest

from oracle import mds as om
from synth import errors
from synth import generators as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "fp32": 1e-4}


def mds():
    import paper_2007_11919_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("maker,l,r", [
    (lambda: gen.small_gaussian(5000, seed=11), 200, 2),
    (lambda: gen.wide_gaussian(20000, seed=12), 1000, 10),
    (lambda: gen.image_mixture(6000, p=784, seed=13), 500, 17),
    (lambda: gen.small_gaussian(3000, seed=14)[:, :3], 100, 5),  # dead columns
])
def test_matches_oracle(maker, l, r):
    X = maker()
    Xf = X.astype(np.float32)
    model = mds().fit_landmarks(dev(Xf), l, r, seed=2)
    fit = om.fit_landmarks(Xf, l, r, seed=2)
    Yo = om.interpolate_affine(fit, Xf)
    for prec, Xin in (("fp64", Xf), ("fp64", Xf.astype(np.float64)), ("fp32", Xf)):
        Y = mds().embed_affine(model, dev(Xin), prec=prec).cpu().numpy()
        e = errors.column_errors(Y, Yo)
        assert e["rms_rel"] <= TOL[prec], (prec, e)
        assert e["maxabs_rms"] <= TOL[prec], (prec, e)
    Yd = mds().embed(model, dev(Xf), prec="fp64").cpu().numpy()
    Ya = mds().embed_affine(model, dev(Xf), prec="fp64").cpu().numpy()
    assert errors.column_errors(Ya, Yd)["maxabs_rms"] < 1e-9


@pytest.mark.parametrize("n", [0, 1, 63, 65, 129])
def test_ragged_and_strided(n):
    X = gen.small_gaussian(300, seed=15)
    model = mds().fit_landmarks(dev(X), 100, 3, seed=1)
    fit = om.fit_landmarks(X, 100, 3, seed=1)
    wide = np.zeros((max(n, 1), X.shape[1] + 3))
    wide[:n, :X.shape[1]] = X[:n]
    Xd = dev(wide)[:n, :X.shape[1]]
    Y = torch.full((max(n, 1), 5), 9.0, dtype=torch.float64, device="cuda")[:n, :3]
    mds().embed_affine(model, Xd, prec="fp64", Y=Y)
    if n:
        Yo = om.interpolate_affine(fit, X[:n])
        assert np.max(np.abs(Y.cpu().numpy() - Yo)) <= 1e-9 * np.max(np.abs(Yo))
        full = Y.as_strided((n, 2), (5, 1), 3).cpu().numpy()
        assert np.all(full == 9.0)


def test_batch_invariance_bitwise():
    X = dev(gen.wide_gaussian(5000, seed=16))
    model = mds().fit_landmarks(X, 500, 10, seed=3)
    full = mds().embed_affine(model, X).cpu().numpy()
    for s, k in [(0, 1), (7, 64), (100, 1000)]:
        part = mds().embed_affine(model, X[s:s + k]).cpu().numpy()
        assert np.array_equal(part, full[s:s + k])



@pytest.mark.parametrize("p,r", [(132, 33), (8, 7), (124, 64)])
def test_fp32_row_stream(p, r):
    """FP32 shapes around the kernel's 32-column steps (p = 132 ends in a
    step of 4 columns, p = 124 in one of 28, p = 8 is a single partial
    step) and up to four 16-column output tiles (r = 64).  Rows that
    start on 16-byte boundaries take the unmasked 16-byte loads; the same
    rows at an odd row stride take the masked loads.  Both match the
    oracle, and each other to FP32 rounding."""
    n, l = 3000, 300
    X = gen.gaussian_columns(n, np.linspace(6.0, 1.0, p), seed=p, dtype=np.float32)
    model = mds().fit_landmarks(dev(X), l, r, seed=4)
    fit = om.fit_landmarks(X, l, r, seed=4)
    Yo = om.interpolate_affine(fit, X)
    Y = mds().embed_affine(model, dev(X), prec="fp32").cpu().numpy()
    e = errors.column_errors(Y, Yo)
    assert e["rms_rel"] <= TOL["fp32"] and e["maxabs_rms"] <= TOL["fp32"], e
    wide = np.zeros((n, p + 1), np.float32)
    wide[:, :p] = X
    Ys = mds().embed_affine(model, dev(wide)[:, :p], prec="fp32").cpu().numpy()
    es = errors.column_errors(Ys, Yo)
    assert es["rms_rel"] <= TOL["fp32"] and es["maxabs_rms"] <= TOL["fp32"], es
    assert errors.column_errors(Ys, Y)["maxabs_rms"] <= 1e-5
    model.free()


def test_error_codes():
    m = mds()
    X = gen.small_gaussian(300, seed=17)
    model = m.fit_landmarks(dev(X.astype(np.float32)), 50, 2, seed=1)
    with pytest.raises(m.MDSError) as ei:
        m.embed_affine(model, dev(X), prec="fp32")  # FP32 needs float input
    assert ei.value.status == 1
    with pytest.raises(m.MDSError) as ei:
        m.embed_affine(model, dev(X.astype(np.float32)), prec="split_bf16")
    assert ei.value.status == 1
    D = ((X[:40, None, :] - X[None, :40, :]) ** 2).sum(-1)
    sq = m.fit_from_sqdist(dev(D), 2)
    with pytest.raises(m.MDSError) as ei:
        m.embed_affine(sq, dev(X[:5].astype(np.float32)))
    assert ei.value.status == 1
