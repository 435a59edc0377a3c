"""Split-precision embed in the variant that walks the landmarks 512 at a
time (at large p, and at any p with enough landmarks to fill the passes)
against the FP64 oracle, through the C ABI (needs a GPU).

Covers: general FP32 data (nonzero lo parts), integer data (lo parts
skipped), p not a multiple of 4 and strided rows (scalar loads), a landmark
count whose padded size is not a multiple of 512 (dead quarters in the last
pass), ragged row counts, batch invariance and the serving path."""

import numpy as np
import pytest

import oracle
from synth import errors
from synth import generators as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-4


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


@pytest.mark.parametrize("p,extra,l,r", [
    (300, 0, 700, 10),    # contiguous rows, 768 padded landmarks: 1.5 passes
    (301, 7, 1000, 16),   # odd p, strided rows, r at one full column block
    (256, 0, 512, 3),     # smallest p of the variant, one exact pass
    (784, 0, 2000, 10),   # the image shape with Gaussian values
    (300, 0, 100, 4),     # 128 padded landmarks: three quarters idle in the only pass
    (512, 0, 260, 10),    # 384 padded landmarks: one idle quarter
], ids=["p300", "p301-strided", "p256", "p784", "l100", "l260"])
@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
def test_wide_split_matches_oracle(p, extra, l, r, prec):
    n = 2500
    Xw = gaussian(n, p, seed=p, extra=extra)
    X = np.ascontiguousarray(Xw[:, :p])
    Xd = torch.from_numpy(Xw).cuda()[:, :p]
    model = mds().fit_landmarks(Xd, l, r, seed=1)
    fit = oracle.fit_landmarks(X.astype(np.float64), l, r, seed=1)
    Yo = oracle.interpolate(fit, X.astype(np.float64))
    full = embed_np(model, Xd, prec)
    e = errors.column_errors(full, Yo)
    assert e["rms_rel"] <= TOL, e
    # ragged row counts (partial tiles): the same bits as inside the full run
    for m in (1, 127, 128, 129):
        assert np.array_equal(embed_np(model, Xd[:m], prec), full[:m]), m


@pytest.mark.parametrize("p,extra,l,r", [
    (100, 0, 1000, 10),   # the 10^6 x 100 shape: two whole passes
    # odd p, strided rows; 896 padded landmarks: one idle quarter.  r = 10,
    # the data's strong directions: columns beyond them (std 1, nearly
    # degenerate eigenvalues) amplify the split's rounding by about 1/lambda
    (33, 3, 800, 10),
    (10, 0, 512, 2),      # one chunk of 32 values, one exact pass
], ids=["p100", "p33-strided", "p10"])
@pytest.mark.parametrize("integer", [False, True], ids=["float", "integer"])
@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
def test_wide_split_small_p(p, extra, l, r, integer, prec):
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
    e = errors.column_errors(full, Yo)
    assert e["rms_rel"] <= TOL, e
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
        e = errors.column_errors(full, Yo)
        assert e["rms_rel"] <= TOL, (prec, e)
        for s, k in [(0, 1), (77, 300), (128, 128), (2999, 1)]:
            assert np.array_equal(embed_np(model, Xd[s:s + k], prec), full[s:s + k]), (prec, s, k)


def test_wide_split_serving_matches_plain():
    from paper_2007_11919_amd import serve
    m = mds()
    Xa = torch.from_numpy(gen.image_mixture(6000, seed=22)).cuda()
    Xb = torch.from_numpy(gaussian(5000, 300, seed=23)).cuda()
    ma = m.fit_landmarks(Xa, 700, 10, seed=0)
    mb = m.fit_landmarks(Xb, 600, 5, seed=1)
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
        jobs.append((model, Xs, prec, Y, srv.submit(mid, Xs, prec, Y)))
    for *_, t in jobs:
        srv.wait(t, timeout=120.0)
    for model, Xs, prec, Y, _ in jobs:
        ref = m.embed(model, Xs, prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(Y, ref), (prec, Xs.shape)
    srv.close()
