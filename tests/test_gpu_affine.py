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
