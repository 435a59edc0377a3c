"""Split-precision embed in the variant that walks the landmarks 512 at a
time (at large p, and at any p with enough landmarks to fill the passes)
against the FP64 oracle, through the C ABI (needs a GPU).

Covers: general FP32 data (nonzero lo parts), integer data (lo parts
skipped), p not a multiple of 4 and strided rows (scalar loads), a landmark
count whose padded size is not a multiple of 512 (dead quarters in the last
pass), ragged row counts, batch invariance, output columns from the
data's unit-variance bulk (r = 16, 20: the weak-direction bounds of
tests/tolerance.py) and the serving path against the oracle."""

import numpy as np
import pytest

import oracle
from synth import generators as gen

from .tolerance import check_embed, check_rows, column_rms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def mds():
    import paper_2007_11919_amd as m
    return m


def embed_np(model, Xd, prec):
    Y = mds().embed(model, Xd, prec=prec)
    torch.cuda.synchronize()
    return Y.cpu().numpy().astype(np.float64)


def gaussian(n, p, seed, extra=0):
    sig = np.concatenate([np.linspace(20.0, 2.0, 10), np.ones(p - 10 + extra)])
    return gen.gaussian_columns(n, sig, seed, dtype=np.float32)


@pytest.mark.parametrize("p,extra,l,r,weak", [
    (300, 0, 700, 10, False),    # contiguous rows, 768 padded landmarks: 1.5 passes
    (301, 7, 1000, 16, True),    # odd p, strided rows, r at one full column block
    (256, 0, 512, 3, False),     # smallest p of the variant, one exact pass
    (784, 0, 2000, 10, False),   # the image shape with Gaussian values
    (300, 0, 100, 4, False),     # 128 padded landmarks: three quarters idle in the only pass
    (512, 0, 260, 10, False),    # 384 padded landmarks: one idle quarter
], ids=["p300", "p301-strided", "p256", "p784", "l100", "l260"])
@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
def test_wide_split_matches_oracle(p, extra, l, r, weak, prec):
    n = 2500
    Xw = gaussian(n, p, seed=p, extra=extra)
    X = np.ascontiguousarray(Xw[:, :p])
    Xd = torch.from_numpy(Xw).cuda()[:, :p]
    model = mds().fit_landmarks(Xd, l, r, seed=1)
    fit = oracle.fit_landmarks(X.astype(np.float64), l, r, seed=1)
    Yo = oracle.interpolate(fit, X.astype(np.float64))
    full = embed_np(model, Xd, prec)
    check_embed(full, Yo, prec, weak=weak)
    # ragged row counts (partial tiles): the same bits as inside the full run
    for m in (1, 127, 128, 129):
        assert np.array_equal(embed_np(model, Xd[:m], prec), full[:m]), m


@pytest.mark.parametrize("p,extra,l,r,weak", [
    (100, 0, 1000, 10, False),   # the 10^6 x 100 shape: two whole passes
    # odd p, strided rows; 896 padded landmarks: one idle quarter.  r = 16
    # reaches 6 columns into the unit-variance bulk (weak directions)
    (33, 3, 800, 16, True),
    (10, 0, 512, 2, False),      # one chunk of 32 values, one exact pass
], ids=["p100", "p33-strided-r16", "p10"])
@pytest.mark.parametrize("integer", [False, True], ids=["float", "integer"])
@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16", "fp32"])
def test_wide_split_small_p(p, extra, l, r, weak, integer, prec):
    """Small p with enough landmarks to fill 512-landmark passes; integer-valued
    data has all lo parts zero (the three-buffer landmark-hi form)."""
    n = 2500
    Xw = gaussian(n, max(p, 10), seed=40 + p, extra=extra)[:, :p + extra]
    if integer:
        Xw = np.rint(Xw).astype(np.float32)
    X = np.ascontiguousarray(Xw[:, :p])
    Xd = torch.from_numpy(np.ascontiguousarray(Xw)).cuda()[:, :p]
    model = mds().fit_landmarks(Xd, l, r, seed=5)
    fit = oracle.fit_landmarks(X.astype(np.float64), l, r, seed=5)
    Yo = oracle.interpolate(fit, X.astype(np.float64))
    full = embed_np(model, Xd, prec)
    check_embed(full, Yo, prec, weak=weak)
    for s, m in [(0, 1), (0, 129), (700, 300), (2499, 1)]:
        assert np.array_equal(embed_np(model, Xd[s:s + m], prec), full[s:s + m]), (s, m)


@pytest.mark.parametrize("l", [900, 200])
def test_wide_split_integer_data_and_batch_invariance(l):
    """Integer data (hi-only landmark form); l = 200 leaves idle quarters."""
    X = gen.image_mixture(3000, seed=21)
    Xd = torch.from_numpy(X).cuda()
    model = mds().fit_landmarks(Xd, l, 10, seed=4)
    fit = oracle.fit_landmarks(X.astype(np.float64), l, 10, seed=4)
    Yo = oracle.interpolate(fit, X.astype(np.float64))
    for prec in ("split_bf16", "split_fp16"):
        full = embed_np(model, Xd, prec)
        check_embed(full, Yo, prec)
        for s, k in [(0, 1), (77, 300), (128, 128), (2999, 1)]:
            assert np.array_equal(embed_np(model, Xd[s:s + k], prec), full[s:s + k]), (prec, s, k)


@pytest.mark.parametrize("p,l", [(100, 1000), (50, 800), (10, 600)], ids=["p100", "p50", "p10"])
@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16", "fp32"])
def test_r20_weak_directions(p, l, prec):
    """r = 20 (two output column blocks: the 128-landmark kernel), as in the
    multi-model serving mix.  The Gaussian laws have 10 strong columns, so
    columns 11..20 lie in the unit-variance bulk (p = 10 uses the small law
    std (15, 10, 1, ...): rank 10, columns 11..20 dead and exactly zero)."""
    if p == 10:
        X = gen.small_gaussian(3000, seed=70).astype(np.float32)
    else:
        X = gaussian(3000, p, seed=60 + p)
    Xd = torch.from_numpy(X).cuda()
    model = mds().fit_landmarks(Xd, l, 20, seed=6)
    fit = oracle.fit_landmarks(X.astype(np.float64), l, 20, seed=6)
    assert model.r_eff == fit.r_eff == min(p, 20)
    Yo = oracle.interpolate(fit, X.astype(np.float64))
    full = embed_np(model, Xd, prec)
    check_embed(full, Yo, prec, weak=True)
    assert np.all(full[:, fit.r_eff:] == 0.0)
    for s, k in [(0, 1), (129, 300), (2999, 1)]:
        assert np.array_equal(embed_np(model, Xd[s:s + k], prec), full[s:s + k]), (s, k)


def test_wide_split_serving_matches_plain():
    """Served results: bit for bit the plain call's, and within the
    tolerances of the FP64 oracle for every request."""
    from paper_2007_11919_amd import serve
    m = mds()
    Xa_h = gen.image_mixture(6000, seed=22)
    Xb_h = gaussian(5000, 300, seed=23)
    Xa = torch.from_numpy(Xa_h).cuda()
    Xb = torch.from_numpy(Xb_h).cuda()
    ma = m.fit_landmarks(Xa, 700, 10, seed=0)
    mb = m.fit_landmarks(Xb, 600, 5, seed=1)
    refs = []
    for X in (Xa_h, Xb_h):
        fit = oracle.fit_landmarks(X.astype(np.float64), *((700, 10, 0) if X is Xa_h else (600, 5, 1)))
        Yo = oracle.interpolate(fit, X.astype(np.float64))
        refs.append((Yo, column_rms(Yo)))
    srv = serve.Server(budget_bytes=4 << 30, max_slots=8, tiles_per_step=64)
    ids = [srv.add_model(ma), srv.add_model(mb)]
    rng = np.random.Generator(np.random.PCG64(5))
    jobs = []
    for k in range(16):
        model, X, mid = [(ma, Xa, ids[0]), (mb, Xb, ids[1])][k % 2]
        n = int(rng.integers(1, 2000))
        off = int(rng.integers(0, X.shape[0] - n))
        prec = ["split_bf16", "split_fp16", "fp32"][k % 3]
        Xs = X[off:off + n]
        Y = torch.full((n, model.r), float("nan"), device="cuda")
        jobs.append((k % 2, off, model, Xs, prec, Y, srv.submit(mid, Xs, prec, Y)))
    for *_, t in jobs:
        srv.wait(t, timeout=120.0)
    for which, off, model, Xs, prec, Y, _ in jobs:
        ref = m.embed(model, Xs, prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(Y, ref), (prec, Xs.shape)
        Yo, scale = refs[which]
        check_rows(Y.cpu().numpy(), Yo[off:off + Xs.shape[0]], scale, prec)
    srv.close()
