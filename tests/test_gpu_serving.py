"""Continuous-batching server: every request's result must equal the plain
mds_embed result for the same rows bit for bit, alone and in any mix of
requests, models and precisions (needs a GPU)."""

import numpy as np
import pytest

from synth import generators as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def mds():
    import paper_2007_11919_amd as m
    return m


def serving():
    from paper_2007_11919_amd import serve
    return serve


def test_mixed_stream_matches_plain_embed():
    m, sv = mds(), serving()
    Xa = torch.from_numpy(gen.wide_gaussian(60000, seed=12)).cuda()
    Xb = torch.from_numpy(gen.gaussian_columns(30000, gen.SIGMAS_SMALL, 5, dtype=np.float32)).cuda()
    Xc = torch.from_numpy(gen.image_mixture(8000, seed=13)).cuda()
    ma = m.fit_landmarks(Xa, 1000, 10, seed=0)
    mb = m.fit_landmarks(Xb, 300, 2, seed=1)
    mc = m.fit_landmarks(Xc, 700, 20, seed=2)
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
        jobs.append((model, Xs, prec, Y, t))
    for *_, t in jobs:
        srv.wait(t, timeout=120.0)
    for model, Xs, prec, Y, t in jobs:
        ref = m.embed(model, Xs, prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(Y, ref), (prec, Xs.shape)
        st = srv.poll(t)
        assert st["state"] == 2 and st["t_done"] >= st["t_admit"] >= st["t_submit"]
    stats = srv.stats()
    assert stats["completed"] == len(jobs) and stats["queued"] == 0 and stats["in_flight"] == 0
    srv.close()


def test_admission_by_bytes_and_slots():
    m, sv = mds(), serving()
    X = torch.from_numpy(gen.wide_gaussian(20000, seed=3)).cuda()
    model = m.fit_landmarks(X, 500, 10, seed=0)
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
        outs.append((Xs, Y, srv.submit(mid, Xs, "fp32", Y)))
    for Xs, Y, t in outs:
        srv.wait(t, timeout=60.0)
        assert torch.equal(Y, m.embed(model, Xs, prec="fp32"))
    st = srv.stats()
    assert st["bytes_in_use"] == model.nbytes
    srv.close()
    big = m.fit_landmarks(X, 500, 10, seed=1)
    srv2 = sv.Server(budget_bytes=big.nbytes - 1, max_slots=4)
    with pytest.raises(m.MDSError) as ei:
        srv2.add_model(big)
    assert ei.value.status == 3
    srv2.close()


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
