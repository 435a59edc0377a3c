"""FP32 embed in the variant that walks the landmarks 512 at a time, against
the FP64 oracle, through the C ABI (needs a GPU).

The variant runs for models with one output column block and at least 512
padded landmarks, when under a quarter of the last 512-landmark pass would
be idle.  Covers: p with a ragged tail k-block (products past p skipped), p
below one k-block, p not a multiple of 4 with strided rows (scalar loads),
aligned strided rows (data chunks copied straight to LDS),
idle landmark quarters in the last pass, ragged row counts, batch
invariance, and serving requests of every precision against plain calls
and the oracle."""

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


def embed_np(model, Xd, prec="fp32"):
    Y = mds().embed(model, Xd, prec=prec)
    torch.cuda.synchronize()
    return Y.cpu().numpy().astype(np.float64)


def gaussian(n, p, seed, extra=0):
    k = min(p, 10)
    sig = np.concatenate([np.linspace(20.0, 2.0, k), np.ones(p - k + extra)])
    return gen.gaussian_columns(n, sig, seed, dtype=np.float32)


@pytest.mark.parametrize("p,extra,l,r,weak", [
    (100, 0, 1000, 10, False),   # two whole passes; tail k-block of 4 values
    (101, 5, 800, 16, True),     # odd p, strided rows; 896 padded landmarks: one idle quarter
    (3, 0, 512, 2, False),       # p below one k-block; one exact pass
    (16, 0, 1300, 10, False),    # one whole k-block; three passes, the last with an idle quarter
    (47, 0, 1024, 5, False),     # p % 4 = 3: tail k-block of 15 values, scalar loads
    (784, 0, 2000, 10, False),   # the image shape with Gaussian values
    (64, 4, 1024, 10, False),    # 16-byte aligned strided rows: data chunks copied straight to LDS
    (48, 3, 1024, 10, False),    # whole k-blocks (no ragged-block branches) from unaligned rows
], ids=["p100", "p101-strided", "p3", "p16-l1300", "p47", "p784", "p64-strided", "p48-oddstride"])
def test_wide_fp32_matches_oracle(p, extra, l, r, weak):
    n = 2500
    Xw = gaussian(n, p, seed=p, extra=extra)
    X = np.ascontiguousarray(Xw[:, :p])
    Xd = torch.from_numpy(Xw).cuda()[:, :p]
    model = mds().fit_landmarks(Xd, l, r, seed=2)
    fit = oracle.fit_landmarks(X.astype(np.float64), l, r, seed=2)
    Yo = oracle.interpolate(fit, X.astype(np.float64))
    full = embed_np(model, Xd)
    check_embed(full, Yo, "fp32", weak=weak)
    # ragged row counts (partial tiles) and offsets: the same bits as in the full run
    for s, m in [(0, 1), (0, 127), (0, 128), (0, 129), (1000, 300), (2499, 1)]:
        assert np.array_equal(embed_np(model, Xd[s:s + m]), full[s:s + m]), (s, m)


def test_variant_boundary_landmark_counts_agree_with_oracle():
    """Landmark counts on both sides of the variant choice (640 padded rows
    stay on the 128-landmark kernel, 896 take the 512-landmark one)."""
    X = gaussian(3000, 60, seed=8)
    Xd = torch.from_numpy(X).cuda()
    for l in (600, 800):
        model = mds().fit_landmarks(Xd, l, 10, seed=3)
        fit = oracle.fit_landmarks(X.astype(np.float64), l, 10, seed=3)
        check_embed(embed_np(model, Xd), oracle.interpolate(fit, X.astype(np.float64)), "fp32")


def test_wide_fp32_serving_matches_plain():
    """Served results: bit for bit the plain call's, and within the
    tolerances of the FP64 oracle for every request."""
    from paper_2007_11919_amd import serve
    m = mds()
    Xa_h = gaussian(6000, 100, seed=31)
    Xb_h = gaussian(5000, 47, seed=32)
    Xa = torch.from_numpy(Xa_h).cuda()
    Xb = torch.from_numpy(Xb_h).cuda()
    ma = m.fit_landmarks(Xa, 1000, 10, seed=0)  # 512-landmark variant in FP32
    mb = m.fit_landmarks(Xb, 600, 5, seed=1)    # 128-landmark kernel in FP32
    refs = []
    for X, (l, r, seed) in ((Xa_h, (1000, 10, 0)), (Xb_h, (600, 5, 1))):
        Yo = oracle.interpolate(oracle.fit_landmarks(X.astype(np.float64), l, r, seed=seed),
                                X.astype(np.float64))
        refs.append((Yo, column_rms(Yo)))
    srv = serve.Server(budget_bytes=4 << 30, max_slots=8, tiles_per_step=64)
    ids = [srv.add_model(ma), srv.add_model(mb)]
    rng = np.random.Generator(np.random.PCG64(6))
    jobs = []
    for k in range(18):
        model, X, mid = [(ma, Xa, ids[0]), (mb, Xb, ids[1])][k % 2]
        n = int(rng.integers(1, 2000))
        off = int(rng.integers(0, X.shape[0] - n))
        prec = ["fp32", "split_bf16", "fp32", "split_fp16"][k % 4]
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


def test_whole_kblocks_serving_matches_plain():
    """p a multiple of 16: the plain launch takes the form without the
    ragged-k-block branches and the serving launch the general form; the
    branches are always taken there, so the two give the same bits."""
    from paper_2007_11919_amd import serve
    m = mds()
    X = torch.from_numpy(gaussian(4000, 64, seed=33)).cuda()
    model = m.fit_landmarks(X, 1000, 10, seed=4)  # 512-landmark variant in FP32
    srv = serve.Server(budget_bytes=2 << 30, max_slots=4, tiles_per_step=64)
    mid = srv.add_model(model)
    jobs = []
    for off, n in [(0, 4000), (5, 700), (1234, 129)]:
        Y = torch.full((n, model.r), float("nan"), device="cuda")
        jobs.append((off, n, Y, srv.submit(mid, X[off:off + n], "fp32", Y)))
    for *_, t in jobs:
        srv.wait(t, timeout=120.0)
    for off, n, Y, _ in jobs:
        ref = m.embed(model, X[off:off + n], prec="fp32")
        torch.cuda.synchronize()
        assert torch.equal(Y, ref), (off, n)
    srv.close()
