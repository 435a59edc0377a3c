"""Dissimilarity input through the C ABI against the FP64 oracle (needs a
GPU): mds_fit_from_sqdist and mds_embed_from_sqdist."""

import numpy as np
import pytest

import oracle
from synth import errors
from synth import generators as gen

from .test_oracle_sqdist import l1_sqdist

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "fp32": 1e-4}


def mds():
    import paper_2007_11919_amd as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check(Y, Yo, prec):
    e = errors.column_errors(Y, Yo)
    assert e["rms_rel"] <= TOL[prec], (prec, e)
    assert e["maxabs_rms"] <= TOL[prec], (prec, e)


def test_euclidean_distances_match_vector_path():
    X = gen.wide_gaussian(6000, seed=12)
    model = mds().fit_landmarks(dev(X), 500, 10, seed=1)
    fit = oracle.fit_landmarks(X, 500, 10, seed=1)
    A2 = oracle.sqdist_rows(X[:3000], fit.M)
    Yo = oracle.interpolate(fit, X[:3000])
    for prec, A in (("fp64", A2), ("fp32", A2.astype(np.float32))):
        Y = mds().embed_from_sqdist(model, dev(A), prec=prec).cpu().numpy()
        check(Y, Yo, prec)
    Yv = mds().embed(model, dev(X[:3000]), prec="fp64").cpu().numpy()
    Ys = mds().embed_from_sqdist(model, dev(A2), prec="fp64").cpu().numpy()
    assert errors.column_errors(Ys, Yv)["maxabs_rms"] < 1e-9


@pytest.mark.parametrize("l,r", [(300, 4), (130, 17)])
def test_non_euclidean_fit_and_embed(l, r):
    X = gen.small_gaussian(2000, seed=5)
    D = l1_sqdist(X[:l], X[:l])
    model = mds().fit_from_sqdist(dev(D), r)
    fit = oracle.fit_from_sqdist(D, r)
    lam = model.eigenvalues()
    assert np.max(np.abs(lam - fit.lam)) <= 1e-12 * fit.lam[0]
    assert np.max(np.abs(model.landmark_coords() - fit.X1)) <= 1e-10 * np.max(np.abs(fit.X1))
    assert model.r_eff == fit.r_eff
    A2 = l1_sqdist(X[l:], X[:l])
    Yo = oracle.interpolate_sqdist(fit, A2)
    for prec, A in (("fp64", A2), ("fp32", A2.astype(np.float32))):
        Y = mds().embed_from_sqdist(model, dev(A), prec=prec).cpu().numpy()
        check(Y, Yo, prec)
    # landmark rows reproduce X1
    Y1 = mds().embed_from_sqdist(model, dev(D), prec="fp64").cpu().numpy()
    assert np.max(np.abs(Y1 - fit.X1)) <= 1e-9 * np.max(np.abs(fit.X1))


@pytest.mark.parametrize("n", [1, 63, 65, 700])
def test_ragged_and_strided(n):
    X = gen.small_gaussian(900, seed=6)
    l = 130
    D = l1_sqdist(X[:l], X[:l])
    model = mds().fit_from_sqdist(dev(D), 3)
    fit = oracle.fit_from_sqdist(D, 3)
    A2 = l1_sqdist(X[l:l + n], X[:l])
    wide = np.zeros((n, l + 5))
    wide[:, :l] = A2
    Ad = dev(wide)[:, :l]  # lda = l + 5
    Yo = oracle.interpolate_sqdist(fit, A2)
    check(mds().embed_from_sqdist(model, Ad, prec="fp64").cpu().numpy(), Yo, "fp64")
    check(mds().embed_from_sqdist(model, Ad.float(), prec="fp32").cpu().numpy(), Yo, "fp32")



@pytest.mark.parametrize("l,r", [(132, 12), (124, 5), (400, 3)])
def test_fp32_row_stream(l, r):
    """FP32 shapes around the kernel's 64-landmark chunks (l = 132 ends
    in a chunk of 4, l = 124 in one of 60, l = 400 in one of
    16).  Rows of A2 that start on 16-byte boundaries take the 16-byte
    loads; the same rows at an odd row stride take the element loads.
    Both match the oracle, and each other to FP32 rounding."""
    X = gen.small_gaussian(2000, seed=9)
    D = l1_sqdist(X[:l], X[:l])
    model = mds().fit_from_sqdist(dev(D), r)
    fit = oracle.fit_from_sqdist(D, r)
    A2 = l1_sqdist(X[l:], X[:l])
    Yo = oracle.interpolate_sqdist(fit, A2)
    A = A2.astype(np.float32)
    Y = mds().embed_from_sqdist(model, dev(A), prec="fp32").cpu().numpy()
    check(Y, Yo, "fp32")
    wide = np.zeros((A.shape[0], l + 1), np.float32)
    wide[:, :l] = A
    Ys = mds().embed_from_sqdist(model, dev(wide)[:, :l], prec="fp32").cpu().numpy()
    check(Ys, Yo, "fp32")
    assert errors.column_errors(Ys, Y)["maxabs_rms"] <= 1e-5
    model.free()


def test_batch_invariance_bitwise():
    X = gen.small_gaussian(3000, seed=7)
    D = l1_sqdist(X[:200], X[:200])
    model = mds().fit_from_sqdist(dev(D), 5)
    A = dev(l1_sqdist(X[200:], X[:200]).astype(np.float32))
    full = mds().embed_from_sqdist(model, A, prec="fp32").cpu().numpy()
    for s, k in [(0, 1), (3, 64), (100, 777)]:
        part = mds().embed_from_sqdist(model, A[s:s + k], prec="fp32").cpu().numpy()
        assert np.array_equal(part, full[s:s + k])


def test_error_codes():
    m = mds()
    X = gen.small_gaussian(300, seed=8)
    D = l1_sqdist(X[:50], X[:50])
    bad = D.copy()
    bad[3, 7] += 1.0
    with pytest.raises(m.MDSError) as ei:
        m.fit_from_sqdist(dev(bad), 2)
    assert ei.value.status == 1
    bad = D.copy()
    bad[2, 2] = np.nan
    with pytest.raises(m.MDSError) as ei:
        m.fit_from_sqdist(dev(bad), 2)
    assert ei.value.status == 1
    model = m.fit_from_sqdist(dev(D), 2)
    with pytest.raises(m.MDSError) as ei:
        m.embed(model, dev(X[:10].astype(np.float32)), prec="fp32")
    assert ei.value.status == 1
    with pytest.raises(m.MDSError) as ei:
        m.embed_from_sqdist(model, dev(D.astype(np.float32)), prec="split_bf16")
    assert ei.value.status == 1
