"""Continuous-batching server: every request's result must equal the plain
mds_embed result for the same rows bit for bit, alone and in any mix of
requests, models and precisions, and match the FP64 oracle within the
stated tolerances (needs a GPU)."""

import numpy as np
import pytest

import oracle
from synth import generators as gen

from .tolerance import check_rows, column_rms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def mds():
    import paper_2007_11919_amd as m
    return m


def serving():
    from paper_2007_11919_amd import serve
    return serve


def oracle_pool(X, l, r, seed):
    """The oracle's coordinates of every row of a pool, and their column RMS."""
    X64 = X.astype(np.float64)
    Yo = oracle.interpolate(oracle.fit_landmarks(X64, l, r, seed=seed), X64)
    return Yo, column_rms(Yo)


def test_mixed_stream_matches_plain_embed():
    m, sv = mds(), serving()
    hosts = [gen.wide_gaussian(60000, seed=12),
             gen.gaussian_columns(30000, gen.SIGMAS_SMALL, 5, dtype=np.float32),
             gen.image_mixture(8000, seed=13)]
    shapes = [(1000, 10, 0), (300, 2, 1), (700, 20, 2)]  # (l, r, seed) per pool
    Xa, Xb, Xc = (torch.from_numpy(h).cuda() for h in hosts)
    ma, mb, mc = (m.fit_landmarks(X, l, r, seed=sd) for X, (l, r, sd) in zip((Xa, Xb, Xc), shapes))
    refs = [oracle_pool(h, *sh) for h, sh in zip(hosts, shapes)]
    srv = sv.Server(budget_bytes=8 << 30, max_slots=16, tiles_per_step=512)
    ids = [srv.add_model(x) for x in (ma, mb, mc)]
    pools = [(ma, Xa, ids[0]), (mb, Xb, ids[1]), (mc, Xc, ids[2])]
    rng = np.random.Generator(np.random.PCG64(7))
    jobs = []
    for k in range(60):
        model, X, mid = pools[k % 3]
        n = int(np.floor(np.exp(rng.uniform(0, np.log(X.shape[0] // 2)))))
        off = int(rng.integers(0, X.shape[0] - n))
        prec = ["fp32", "split_bf16", "split_fp16"][int(rng.integers(0, 3))]
        Xs = X[off:off + n]
        Y = torch.full((n, model.r), float("nan"), device="cuda")
        t = srv.submit(mid, Xs, prec, Y)
        jobs.append((k % 3, off, model, Xs, prec, Y, t))
    for *_, t in jobs:
        srv.wait(t, timeout=120.0)
    for which, off, model, Xs, prec, Y, t in jobs:
        ref = m.embed(model, Xs, prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(Y, ref), (prec, Xs.shape)
        Yo, scale = refs[which]
        check_rows(Y.cpu().numpy(), Yo[off:off + Xs.shape[0]], scale, prec)
        st = srv.poll(t)
        assert st["state"] == 2 and st["t_done"] >= st["t_admit"] >= st["t_submit"]
    stats = srv.stats()
    assert stats["completed"] == len(jobs) and stats["queued"] == 0 and stats["in_flight"] == 0
    srv.close()


def test_admission_by_bytes_and_slots():
    m, sv = mds(), serving()
    Xh = gen.wide_gaussian(20000, seed=3)
    X = torch.from_numpy(Xh).cuda()
    model = m.fit_landmarks(X, 500, 10, seed=0)
    Yo, scale = oracle_pool(Xh, 500, 10, 0)
    # budget: the model plus room for ~5000 points of requests at a time
    budget = model.nbytes + 4 * 5000 * (100 + 10)
    srv = sv.Server(budget_bytes=budget, max_slots=2, tiles_per_step=64)
    mid = srv.add_model(model)
    with pytest.raises(m.MDSError) as ei:
        srv.submit(mid, X[:6000], "fp32", torch.empty((6000, 10), device="cuda"))
    assert ei.value.status == 3
    outs = []
    for k in range(12):
        Xs = X[k * 1500:(k + 1) * 1500]
        Y = torch.empty((1500, 10), device="cuda")
        outs.append((k, Xs, Y, srv.submit(mid, Xs, "fp32", Y)))
    for k, Xs, Y, t in outs:
        srv.wait(t, timeout=60.0)
        assert torch.equal(Y, m.embed(model, Xs, prec="fp32"))
        check_rows(Y.cpu().numpy(), Yo[k * 1500:(k + 1) * 1500], scale, "fp32")
    st = srv.stats()
    assert st["bytes_in_use"] == model.nbytes
    srv.close()
    big = m.fit_landmarks(X, 500, 10, seed=1)
    srv2 = sv.Server(budget_bytes=big.nbytes - 1, max_slots=4)
    with pytest.raises(m.MDSError) as ei:
        srv2.add_model(big)
    assert ei.value.status == 3
    srv2.close()


def test_submit_rejects_wrong_dtype_and_shapes():
    """Rows the serving kernels cannot read or write as float are refused
    before anything runs."""
    m, sv = mds(), serving()
    X = torch.from_numpy(gen.wide_gaussian(3000, seed=3)).cuda()
    model = m.fit_landmarks(X, 200, 4, seed=0)
    srv = sv.Server(budget_bytes=1 << 30, max_slots=4)
    mid = srv.add_model(model)
    Y = torch.empty((100, 4), device="cuda")
    for Xs, Ys in [(X[:100].double(), Y), (X[:100], Y.double()), (X[:100, :50], Y),
                   (X[:100], torch.empty((99, 4), device="cuda")),
                   (X[:100], torch.empty((100, 3), device="cuda"))]:
        with pytest.raises(ValueError):
            srv.submit(mid, Xs, "fp32", Ys)
    # the C entry point itself refuses anything but float rows
    import ctypes
    from paper_2007_11919_amd import _lib
    t = ctypes.c_int64()
    st = _lib.lib().mds_serve_submit(srv._h, mid, ctypes.c_void_p(X.data_ptr()), 1, 100, 100, 1,
                                     ctypes.c_void_p(Y.data_ptr()), 4, ctypes.byref(t))
    assert st == 1  # MDS_ERR_INVALID_ARG
    srv.close()


def test_zero_point_request_completes():
    m, sv = mds(), serving()
    X = torch.from_numpy(gen.wide_gaussian(2000, seed=3)).cuda()
    model = m.fit_landmarks(X, 200, 3, seed=0)
    srv = sv.Server(budget_bytes=1 << 30, max_slots=4)
    mid = srv.add_model(model)
    t = srv.submit(mid, X[:0], "fp32", torch.empty((0, 3), device="cuda"))
    srv.wait(t, timeout=10.0)
    assert srv.poll(t)["state"] == 2
    srv.close()
