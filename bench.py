"""Benchmark of interpolation MDS on one MI355X.

A step is one pass of the whole method over one batch: landmark sampling
and the FP64 fit (gather, squared distances, double centring, Lanczos
eigenpairs, finalisation) followed by the fused FP32 embed of every row.
`value` is rows per second over the timed steps, inputs resident in HBM.

Headline workload: 1,000,000 x 784 integer rows 0..255 from a 10-component
Gaussian mixture (std 40; image-like data standing in for the grey-scale
image set of Section 5), l = 2000 landmarks, r = 10.  On the same data: the
split-BF16 and split-FP16 embeds (speed-up and error; which products ran),
the FP64 embed, the embed kernel's roofline fraction, and the FP64 oracle
on the host cores (bounded sample).

Further legs, each with its own error check:
* 1,000,000 x 100 Gaussian rows (std 20 -> 2 on 10 columns, 1 on 90),
  l = 1000, r = 10: the same step and embed figures, serving (20,000
  requests of 1..200,000 rows at three loads, FP32 and split BF16), the
  embed from squared dissimilarities (Section 2 input), the affine form of
  eq. (2), MaxMin landmark selection and pivot MDS (Section 3.1), and
  divide-and-conquer MDS (Section 3.2) on the simulation design of
  Section 4.1;
* 5,000 x 10 FP64 rows (std 15, 10, 1, ...), l = 200, r = 2: latency of the
  fit and the embed, beside the oracle;
* 48 fitted models served together under a 24 GiB budget (p in {10, 50,
  100, 784} x r in {2, 5, 10, 20} x 3, l log-uniform in [500, 4000]),
  FP32 and split BF16, with the error against the oracle per (p, r).

    python bench.py [--steps K] [--warmup W] [--workload image|wide]
    python bench.py --only-embed fp32 --workload image --iters 20   (rocprofv3 runs)
    python bench.py --only-fit --iters 5                             (rocprofv3 runs)
    python bench.py --only-dc | --only-affine | --only-sqdist | --only-pivot --iters K
    python bench.py --copy-calib 1073741824                          (counter calibration)
"""

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3e12   # MI355X dense FP32 matrix, FLOP/s
PEAK_FP64_MFMA = 78.6e12    # MI355X dense FP64 matrix, FLOP/s
PEAK_BF16_MFMA = 2.5e15     # MI355X dense BF16 matrix, FLOP/s
PEAK_HBM = 8.0e12           # bytes/s

WORKLOADS = {
    "wide": dict(n=1_000_000, p=100, l=1000, r=10,
                 desc="interpolation MDS, 1,000,000 x 100 Gaussian rows (std 20..2 on 10 "
                      "columns, 1 on 90), l=1000 landmarks, r=10; FP64 fit, FP32 embed"),
    "image": dict(n=1_000_000, p=784, l=2000, r=10,
                  desc="interpolation MDS, 1,000,000 x 784 integer rows 0..255 from a "
                       "10-component Gaussian mixture (std 40), l=2000 landmarks, r=10; "
                       "FP64 fit, FP32 embed"),
}
SMALL = dict(n=5000, p=10, l=200, r=2, seeds=(0, 1, 2),
             desc="interpolation MDS, 5,000 x 10 FP64 Gaussian rows (std 15, 10, 1 x 8), "
                  "l=200 landmarks, r=2; FP64 fit and embed")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_data(name, n=None):
    from synth import generators as gen
    w = WORKLOADS[name]
    n = w["n"] if n is None else n
    if name == "wide":
        return gen.wide_gaussian(n, seed=12)
    return gen.image_mixture(n, p=w["p"], seed=13)


def flops_per_point(p, l, r):
    # distances 2lp, epilogue 3l, projection 2lr, row norm 2p
    return 2.0 * l * p + 3.0 * l + 2.0 * l * r + 2.0 * p


def time_embed(mds, torch, model, Xd, prec, iters):
    """Average duration of one mds_embed launch, from HIP events recorded on
    the stream the kernel is launched on (torch's current stream)."""
    st = torch.cuda.current_stream()
    Y = mds.embed(model, Xd, prec=prec)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(iters):
        mds.embed(model, Xd, prec=prec, Y=Y)
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / iters, Y


def embed_kernel(prec, p, l, r):
    """Name of the embed kernel the library runs for a model of this shape
    (same rule as the library's variant choice)."""
    l_pad = -(-l // 128) * 128
    span = -(-l_pad // 512) * 512
    fills = l_pad >= 512 and 4 * (span - l_pad) < span
    if r <= 16 and (fills or (prec != "fp32" and p >= 256)):
        if prec == "fp32":
            return "k_embed_wide<FP32> (512 landmarks per pass over a row tile)"
        return f"k_embed_s3<{prec.upper()}> (32 x 32 x 16 split products, 512 landmarks per pass)"
    return f"k_embed<{prec.upper()}> (128 landmarks per pass over a row tile)"


def counters_for(kernel_tag):
    """Traffic measured by rocprofv3 --pmc for the current kernel source, or
    None if the source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    src = open(os.path.join(ROOT, "paper_2007_11919_amd", "csrc", "embed.hip"), "rb").read()
    if vals.get("embed_hip_sha256") != hashlib.sha256(src).hexdigest():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_info():
    """CPU model, usable cores and the BLAS the oracle runs on."""
    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = []
    try:
        from threadpoolctl import threadpool_info
        for i in threadpool_info():
            if i.get("user_api") == "blas":
                blas.append(f"{i.get('internal_api')} {i.get('version')} ({i.get('num_threads')} threads)")
    except Exception:  # threadpoolctl absent: report what numpy was built with
        blas.append("unknown")
    return {"cpu_model": model, "cores": len(os.sched_getaffinity(0)), "blas": "; ".join(blas)}


def one_thread():
    """Context that limits the BLAS to one thread (for a per-core rate)."""
    from threadpoolctl import threadpool_limits
    return threadpool_limits(limits=1, user_api="blas")


def max_row_error(Y, R, scale):
    """Worst RMS and worst max over columns of |Y - R| / scale_k (device
    tensors; scale: column RMS of the reference over the whole pool)."""
    d = (Y.double() - R.double()).abs() / scale
    return float(d.pow(2).mean(0).sqrt().max()), float(d.max())


def serving_run(mds, torch, model, Xd, prec, count, seed, budget, Y64, fit_o, X):
    """Poisson load at three fractions of the measured saturated capacity.
    Requests are slices of the pool at random offsets.  Every served result
    is compared with the oracle-validated GPU FP64 embed of the same pool
    rows (Y64), and every 10th request's first rows (up to 256) with the
    host oracle itself (fit_o, X)."""
    import oracle
    from paper_2007_11919_amd.serve import Server
    from synth import generators as gen
    n = Xd.shape[0]
    sizes = gen.request_sizes(count, 200_000, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    offs = rng.integers(0, n - sizes + 1)
    total = int(sizes.sum())
    Yall = torch.empty((total, model.r), dtype=torch.float32, device=Xd.device)
    ystart = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    srv = Server(budget_bytes=budget, max_slots=256, tiles_per_step=2048)
    mid = srv.add_model(model)

    def run(arrivals):
        tickets = []
        t0 = srv.now() + 0.002
        for i in range(count):
            if arrivals is not None:
                target = t0 + arrivals[i]
                while srv.now() < target:
                    pass
            s, o, y0 = int(sizes[i]), int(offs[i]), int(ystart[i])
            tickets.append(srv.submit(mid, Xd[o:o + s], prec, Yall[y0:y0 + s]))
        for t in tickets:
            srv.wait(t, timeout=600.0)
        recs = [srv.poll(t) for t in tickets]
        done = np.array([r["t_done"] for r in recs])
        if arrivals is None:
            start = min(r["t_submit"] for r in recs)
            return (done.max() - start), None
        sched = t0 + arrivals
        lat = done - sched
        return done.max() - t0, lat

    run(None)  # warm-up
    makespan, _ = run(None)
    cap_rps = count / makespan
    out = {"precision": prec, "requests": count, "points": total, "mean_points": float(sizes.mean()),
           "saturated_points_per_s": float(total / makespan),
           "saturated_requests_per_s": float(cap_rps), "loads": []}
    for rho in (0.5, 0.8, 0.95):
        arr = gen.poisson_arrivals(count, rho * cap_rps, seed + 7)
        span, lat = run(arr)
        out["loads"].append({
            "rho": rho, "rate_requests_per_s": float(rho * cap_rps),
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "points_per_s": float(total / span)})
    srv.close()
    # results of the last run against the references
    scale = Y64.double().pow(2).mean(0).sqrt()
    worst_rms, worst_max = 0.0, 0.0
    for i in range(count):
        s, o, y0 = int(sizes[i]), int(offs[i]), int(ystart[i])
        a, b = max_row_error(Yall[y0:y0 + s], Y64[o:o + s], scale)
        worst_rms, worst_max = max(worst_rms, a), max(worst_max, b)
    sc = scale.cpu().numpy()
    o_rms, o_max, o_rows = 0.0, 0.0, 0
    for i in range(0, count, 10):
        s, o, y0 = min(int(sizes[i]), 256), int(offs[i]), int(ystart[i])
        Yo = oracle.interpolate(fit_o, X[o:o + s].astype(np.float64))
        d = np.abs(Yall[y0:y0 + s].cpu().numpy().astype(np.float64) - Yo) / sc
        o_rms = max(o_rms, float(np.sqrt((d * d).mean(0)).max()))
        o_max = max(o_max, float(d.max()))
        o_rows += s
    out["error"] = {
        "every_request_vs_gpu_fp64": {"rms": worst_rms, "max": worst_max},
        "every_10th_request_vs_oracle": {"rms": o_rms, "max": o_max, "rows": o_rows},
        "reading": "per request, worst column of RMS and of max |served - reference| over the "
                   "column RMS of the reference on the whole pool"}
    del Yall
    return out


def serving_multi(mds, torch, count, seed, budget, pool_rows=500_000, precs=("fp32", "split_bf16")):
    """Multi-tenant serving: 48 fitted models (p in {10, 50, 100, 784} x r in
    {2, 5, 10, 20} x 3, l log-uniform in [500, 4000]) resident under a byte
    budget; a stream of requests (sizes log-uniform in [1, 500,000], model
    uniform) at 0.8 of the measured saturated rate.  A sample of results is
    compared bit for bit with a plain mds_embed of the same rows, and for
    each (p, r) the model with the fewest landmarks is refitted by the host
    oracle, which checks up to 512 rows of that model's largest request."""
    import oracle
    from paper_2007_11919_amd.serve import Server
    from synth import errors
    from synth import generators as gen
    rng = np.random.Generator(np.random.PCG64(seed))
    pools = {
        10: gen.gaussian_columns(pool_rows, gen.SIGMAS_SMALL, 21, dtype=np.float32),
        50: gen.gaussian_columns(pool_rows, gen.SIGMAS_P50, 22, dtype=np.float32),
        100: gen.wide_gaussian(pool_rows, seed=23),
        784: gen.image_mixture(pool_rows, seed=24),
    }
    dpools = {p: torch.from_numpy(x).cuda() for p, x in pools.items()}
    models, specs = [], []
    t = time.perf_counter()
    for rep in range(3):
        for p in (10, 50, 100, 784):
            for r in (2, 5, 10, 20):
                l = int(round(np.exp(rng.uniform(np.log(500), np.log(4000)))))
                fseed = rep * 100 + p + r
                models.append((p, mds.fit_landmarks(dpools[p], l, r, seed=fseed)))
                specs.append((p, r, l, fseed))
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t
    out = {"models": len(models), "budget_bytes": budget, "fit_all_s": fit_s, "pool_rows": pool_rows,
           "model_bytes": int(sum(m.nbytes for _, m in models)), "runs": []}
    sizes = gen.request_sizes(count, 500_000, seed + 1)
    which = rng.integers(0, len(models), size=count)
    offs = [int(rng.integers(0, pool_rows - s + 1)) for s in sizes]
    # per (p, r): the model with the fewest landmarks, and its largest request
    checks = {}
    for mi, (p, r, l, _) in enumerate(specs):
        if (p, r) not in checks or l < specs[checks[(p, r)]][2]:
            checks[(p, r)] = mi
    fits_o = {}
    t = time.perf_counter()
    for (p, r), mi in checks.items():
        _, _, l, fseed = specs[mi]
        fits_o[mi] = oracle.fit_landmarks(pools[p], l, r, seed=fseed)
    oracle_fit_s = time.perf_counter() - t
    for prec in precs:
        srv = Server(budget_bytes=budget, max_slots=512, tiles_per_step=4096)
        ids = [srv.add_model(m) for _, m in models]
        ys = [None] * count

        def run(arrivals):
            tickets = []
            t0 = srv.now() + 0.002
            for i in range(count):
                if arrivals is not None:
                    while srv.now() < t0 + arrivals[i]:
                        pass
                p, m = models[which[i]]
                s, o = int(sizes[i]), offs[i]
                if ys[i] is None:
                    ys[i] = torch.empty((s, m.r), dtype=torch.float32, device="cuda")
                tickets.append(srv.submit(ids[which[i]], dpools[p][o:o + s], prec, ys[i]))
            for tk in tickets:
                srv.wait(tk, timeout=1200.0)
            recs = [srv.poll(tk) for tk in tickets]
            done = np.array([r["t_done"] for r in recs])
            if arrivals is None:
                return done.max() - min(r["t_submit"] for r in recs), None
            return done.max() - t0, done - (t0 + arrivals)

        makespan, _ = run(None)
        cap = count / makespan
        arr = gen.poisson_arrivals(count, 0.8 * cap, seed + 2)
        span, lat = run(arr)
        # bit-for-bit check of a sample against plain mds_embed
        same = True
        for i in range(0, count, max(1, count // 50)):
            p, m = models[which[i]]
            s, o = int(sizes[i]), offs[i]
            ref = mds.embed(m, dpools[p][o:o + s], prec=prec)
            same &= bool(torch.equal(ref, ys[i]))
        # oracle check per (p, r)
        per_class = []
        for (p, r), mi in sorted(checks.items()):
            reqs = np.flatnonzero(which == mi)
            if len(reqs) == 0:
                continue
            i = int(reqs[np.argmax(sizes[reqs])])
            s, o = min(int(sizes[i]), 512), offs[i]
            Yo = oracle.interpolate(fits_o[mi], pools[p][o:o + s].astype(np.float64))
            e = errors.column_errors(ys[i][:s].cpu().numpy(), Yo)
            per_class.append({"p": p, "r": r, "l": specs[mi][2], "rows": s,
                              "r_eff": int(models[mi][1].r_eff),
                              "rms_rel": e["rms_rel"], "maxabs_rms": e["maxabs_rms"]})
        st = srv.stats()
        srv.close()
        out["runs"].append({
            "precision": prec, "requests": count, "points": int(sizes.sum()),
            "saturated_points_per_s": float(sizes.sum() / makespan),
            "rate_requests_per_s": float(0.8 * cap),
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "points_per_s_at_load": float(sizes.sum() / span),
            "steps": int(st["steps"]), "bitwise_equal_to_plain_embed": same,
            "err_vs_oracle_per_class": per_class})
        del ys
    out["oracle_fit_s"] = oracle_fit_s
    for _, m in models:
        m.free()
    return out


def sqdist_leg(mds, torch, model, Xd, Y32, iters):
    """mds_embed_from_sqdist on the n x l block of squared distances from
    every row to the landmarks (FP32, built on the device beforehand as
    input).  Memory-bound: reported against the HBM peak."""
    idx = torch.from_numpy(model.landmarks()).to(Xd.device)
    M = Xd[idx]
    n, l = Xd.shape[0], M.shape[0]
    A2 = torch.empty((n, l), dtype=torch.float32, device=Xd.device)
    mn = (M * M).sum(1)
    for s in range(0, n, 100_000):
        xb = Xd[s:s + 100_000]
        A2[s:s + 100_000] = ((xb * xb).sum(1, keepdim=True) + mn[None, :] - 2.0 * (xb @ M.T)).clamp_min_(0)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    Y = mds.embed_from_sqdist(model, A2, prec="fp32")
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(iters):
        mds.embed_from_sqdist(model, A2, prec="fp32", Y=Y)
    e1.record(st)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / iters
    nbytes = 4.0 * n * l + 4.0 * n * model.r
    from synth import errors
    err = errors.column_errors(Y.cpu().numpy(), Y32.cpu().numpy())
    del A2
    return {"ms": t * 1e3, "points_per_s": n / t,
            "roofline": {"bound": "hbm", "achieved": nbytes / t / 1e9, "peak": PEAK_HBM / 1e9,
                         "unit": "GB/s", "frac": nbytes / t / PEAK_HBM,
                         "bytes_per_launch": nbytes},
            "rms_rel_vs_fp32_embed": err["rms_rel"]}


def affine_leg(mds, torch, model, Xd, Y64, iters):
    """mds_embed_affine (y = A x + b, squared Euclidean only) on the same
    rows and model, FP32: a streaming kernel, reported against the HBM
    peak, with its error against the FP64 distance path."""
    from synth import errors
    st = torch.cuda.current_stream()
    Y = mds.embed_affine(model, Xd, prec="fp32")
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(iters):
        mds.embed_affine(model, Xd, prec="fp32", Y=Y)
    e1.record(st)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / iters
    n, p = Xd.shape
    nbytes = 4.0 * n * (p + model.r)
    e = errors.column_errors(Y.cpu().numpy(), Y64)
    return {"ms": t * 1e3, "points_per_s": n / t,
            "roofline": {"bound": "hbm", "achieved": nbytes / t / 1e9, "peak": PEAK_HBM / 1e9,
                         "unit": "GB/s", "frac": nbytes / t / PEAK_HBM, "bytes_per_launch": nbytes},
            "err_vs_gpu_fp64_distance_path": {k: e[k] for k in ("rms_rel", "maxabs_rms")},
            "note": "separate mode (affine form of eq. (2)); not the distance-block path"}


def pivot_leg(mds, torch, Xd, X, iters, cpu):
    """MaxMin selection of l = 200 landmarks (one pass over X per landmark)
    and pivot MDS with l = 200 random pivots, r = 10 (Section 4.1's pivot
    MDS setting), on the 10^6 x 100 rows."""
    from synth import errors
    import oracle
    from oracle import pivot as opv
    n, p = Xd.shape
    l, r = 200, 10
    st = torch.cuda.current_stream()
    mds.maxmin_landmarks(Xd, 8, 0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    mm = mds.maxmin_landmarks(Xd, l, 0)
    t_mm = time.perf_counter() - t
    mm_bytes = (l - 1) * (4.0 * n * p + 16.0 * n)
    Y, lam, r_eff = mds.pivot_mds(Xd, l, r, seed=4)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(iters):
        mds.pivot_mds(Xd, l, r, seed=4, Y=Y)
    t_pv = (time.perf_counter() - t) / iters
    out = {"maxmin": {"l": l, "ms": t_mm * 1e3, "ms_per_landmark": t_mm * 1e3 / (l - 1),
                      "roofline": {"bound": "hbm", "achieved": mm_bytes / t_mm / 1e9,
                                   "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                                   "frac": mm_bytes / t_mm / PEAK_HBM,
                                   "bytes": mm_bytes}},
           "pivot_mds": {"l": l, "r": r, "pivots": "random", "ms": t_pv * 1e3,
                         "points_per_s": n / t_pv, "lam_over_n": [float(v) / n for v in lam],
                         "r_eff": r_eff}}
    pidx = np.array(oracle.sample_landmarks(n, l, 4))
    rows = np.sort(np.random.default_rng(0).choice(n, 3000, replace=False))
    t = time.perf_counter()
    Yo, lamo, _ = opv.pivot_mds_large(X, pidx, r, rows=rows)
    t_orc = time.perf_counter() - t
    e = errors.column_errors(Y.cpu().numpy()[rows], Yo)
    out["pivot_mds"]["err_vs_oracle_rows"] = {"rows": len(rows),
                                              **{k: e[k] for k in ("rms_rel", "maxabs_rms")}}
    if cpu:
        out["pivot_mds"]["cpu_baseline"] = {
            "value": n / t_orc, "unit": "points/s", "cores": len(os.sched_getaffinity(0)),
            "kind": "oracle",
            "sample": f"oracle (chunked FP64 expansion, all {n} rows for C'C, {len(rows)} rows "
                      f"output) {t_orc:.1f} s, counted as a whole pass (output of the other rows "
                      f"not included)"}
    return out


DC = dict(n=1_000_000, k=100, h=10, l=400, c=50, r=10,
          desc="divide-and-conquer MDS, 1,000,000 x 100 rows of the simulation design "
               "(10 columns of variance 15, 90 of variance 1), l=400, c=5r=50, r=10; "
               "FP32 input, FP64 arithmetic")


def dc_flops(n, p, l, c, r):
    """FP64 flops of divide-and-conquer MDS through the p x p Gram matrix:
    per part of m rows, Gram 2 m p^2, Householder tridiagonalisation
    4/3 p^3, back-transformation 4 p^2 r, coordinates 2 m p r."""
    from oracle import dc as odc
    P = odc.num_parts(n, l, c)
    tot = 0.0
    for j in range(P):
        m = l if j < P - 1 else n - (P - 1) * (l - c)
        tot += 2.0 * m * p * p + 4.0 / 3.0 * p ** 3 + 4.0 * p * p * r + 2.0 * m * p * r
    return tot, P


def dc_leg(mds, torch, iters, cpu):
    """mds_divide_conquer at the largest simulation scenario of Section 4.1
    with the paper's divide-and-conquer settings (l = 400, c = 5r)."""
    from synth import generators as gen
    from synth import errors
    from oracle import dc as odc
    d = DC
    X = gen.paper_design(d["n"], d["k"], d["h"], seed=15, dtype=np.float32)
    Xd = torch.from_numpy(X).cuda()
    st = torch.cuda.current_stream()
    Y, lam_bar, r_eff = mds.divide_conquer(Xd, d["l"], d["c"], d["r"], seed=6)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    t = time.perf_counter()
    for _ in range(iters):
        mds.divide_conquer(Xd, d["l"], d["c"], d["r"], seed=6, Y=Y)
    wall = (time.perf_counter() - t) / iters
    e1.record(st)
    torch.cuda.synchronize()
    dev_s = e0.elapsed_time(e1) / 1e3 / iters
    flops, P = dc_flops(d["n"], d["k"], d["l"], d["c"], d["r"])
    out = {"config": d["desc"], "parts": P, "ms": wall * 1e3, "ms_stream": dev_s * 1e3,
           "points_per_s": d["n"] / wall, "lam_bar": [float(v) for v in lam_bar], "r_eff": r_eff,
           "fp64": {"algorithmic_gflop": flops / 1e9, "achieved_tflops": flops / wall / 1e12,
                    "peak_tflops": 78.6, "frac": flops / wall / 78.6e12}}
    Yn = Y.cpu().numpy()
    parts = {1, P // 2, P - 1}
    X64 = X.astype(np.float64)
    t = time.perf_counter()
    ref = odc.dc_mds(X64, d["l"], d["c"], d["r"], 6, parts=parts)
    t_orc = time.perf_counter() - t
    rows = np.flatnonzero(~np.isnan(ref.Y[:, 0]))
    e = errors.column_errors(Yn[rows], ref.Y[rows])
    out["err_vs_oracle_parts"] = {"parts": sorted(parts | {0}),
                                  **{k: e[k] for k in ("rms_rel", "maxabs_rms", "frob_rel")}}
    if cpu:
        # partition plus 4 parts of classical MDS and alignment on the host,
        # scaled to all parts
        per_part = t_orc / 4.0
        whole = per_part * P
        out["cpu_baseline"] = {"value": d["n"] / whole, "unit": "points/s",
                               "cores": len(os.sched_getaffinity(0)), "kind": "oracle",
                               "sample": f"oracle on 4 of {P} parts ({t_orc:.2f} s, partition "
                                         f"of all rows included), scaled to all parts"}
    del Xd
    return out


def cpu_baseline(name, X, w, sample_rows, one_thread_rows, Ys_gpu):
    """The FP64 oracle, as it stands, on the host cores: the full fit (once)
    plus the embed of a random sample of rows (median of 3), scaled to rows
    per second of a whole pass; also the embed rate of one thread on a
    smaller sample.  Returns the oracle fit, the sample rows and the GPU
    results' error on them."""
    import oracle
    from synth import errors
    info = host_info()
    t = time.perf_counter()
    fit = oracle.fit_landmarks(X, w["l"], w["r"], seed=0)
    t_fit = time.perf_counter() - t
    rows = np.sort(np.random.Generator(np.random.PCG64(99)).choice(X.shape[0], sample_rows,
                                                                   replace=False))
    Xs = X[rows]
    t_emb = []
    for _ in range(3):
        t = time.perf_counter()
        Yo = oracle.interpolate(fit, Xs)
        t_emb.append(time.perf_counter() - t)
    t_med = float(np.median(t_emb))
    per_row = t_med / sample_rows
    whole = t_fit + per_row * X.shape[0]
    with one_thread():
        t = time.perf_counter()
        oracle.interpolate(fit, Xs[:one_thread_rows])
        t1 = time.perf_counter() - t
    errs = {}
    for prec, Y in Ys_gpu.items():
        e = errors.column_errors(Y[rows], Yo)
        errs[prec] = {k: e[k] for k in ("rms_rel", "maxabs_rms", "frob_rel")}
    base = {"value": float(X.shape[0] / whole), "unit": "points/s", "cores": info["cores"],
            "kind": "oracle",
            "sample": f"oracle fit on all {w['l']} landmarks, timed once ({t_fit:.2f} s) + embed of "
                      f"{sample_rows} random rows (median of 3: {t_med:.2f} s), scaled to "
                      f"{X.shape[0]} rows",
            "cpu_model": info["cpu_model"], "blas": info["blas"],
            "fit_s": t_fit, "embed_s_per_row": per_row, "embed_runs_s": t_emb,
            "one_thread": {"rows": one_thread_rows, "s": t1,
                           "embed_points_per_s": one_thread_rows / t1}}
    return base, errs, fit, rows, Yo


def lo_parts_zero(X):
    """True when every value is an integer of magnitude <= 256, so that its
    BF16 (and FP16) value is exact and both split lo parts are zero (the
    landmark rows are rows of X)."""
    return bool(np.all(np.abs(X) <= 256.0) and np.array_equal(X, np.rint(X)))


def workload_run(mds, torch, name, args, dev, cpu):
    """The step (sampler + fit + FP32 embed of every row) on one workload,
    timed over args.steps after args.warmup, then the fit and each embed
    precision alone, errors against the GPU FP64 embed (all rows) and the
    host oracle (a sample).  Returns the report and what later legs reuse."""
    from synth import errors
    w = WORKLOADS[name]
    log(f"[{name}] generating data")
    X = make_data(name)
    Xd = torch.from_numpy(X).to(dev)
    torch.cuda.synchronize()
    n = w["n"]

    def step():
        model = mds.fit_landmarks(Xd, w["l"], w["r"], seed=0)
        Y = mds.embed(model, Xd, prec="fp32")
        torch.cuda.synchronize()
        model.free()
        return Y

    log(f"[{name}] warm-up")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[{name}] timed steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0

    # fit alone (median of five) and the embed kernels alone, on one model
    fit_times = []
    for _ in range(5):
        torch.cuda.synchronize()
        t = time.perf_counter()
        model = mds.fit_landmarks(Xd, w["l"], w["r"], seed=0)
        torch.cuda.synchronize()
        fit_times.append((time.perf_counter() - t) * 1e3)
        if len(fit_times) < 5:
            model.free()
    fit_stats = model.fit_stats()
    log(f"[{name}] embeds")
    t32, Y32 = time_embed(mds, torch, model, Xd, "fp32", args.embed_iters)
    tbf, Ybf = time_embed(mds, torch, model, Xd, "split_bf16", args.embed_iters)
    t16, Y16 = time_embed(mds, torch, model, Xd, "split_fp16", args.embed_iters)
    t64, Y64 = time_embed(mds, torch, model, Xd, "fp64", max(3, args.embed_iters // 4))
    Y64n = Y64.cpu().numpy()
    err_vs64 = {}
    for prec, Y in (("fp32", Y32), ("split_bf16", Ybf), ("split_fp16", Y16)):
        e = errors.column_errors(Y.cpu().numpy(), Y64n)
        err_vs64[prec] = {k: e[k] for k in ("rms_rel", "maxabs_rms", "frob_rel")}

    fpp = flops_per_point(w["p"], w["l"], w["r"])
    flops = fpp * n
    lo_zero = lo_parts_zero(X)
    roof = {"bound": "mfma", "achieved": flops / t32 / 1e12, "peak": PEAK_FP32_MFMA / 1e12,
            "unit": "TFLOP/s", "frac": flops / t32 / PEAK_FP32_MFMA,
            "traffic": counters_for(f"embed_fp32_{name}"),
            "kernel": embed_kernel("fp32", w["p"], w["l"], w["r"]),
            "flops_per_point": fpp, "points_per_launch": n}
    rep = {
        "ms_per_step": total / args.steps * 1e3, "points_per_s": n * args.steps / total,
        "config": {"workload": w["desc"], "n": n, "p": w["p"], "l": w["l"], "r": w["r"]},
        "roofline": roof,
        "fit_ms": float(np.median(fit_times)), "fit_lanczos_steps": fit_stats["lanczos_steps"],
        "embed_fp32_ms": t32 * 1e3, "embed_fp32_points_per_s": n / t32,
        "split_bf16": {
            "embed_ms": tbf * 1e3, "points_per_s": n / tbf, "speedup_vs_fp32": t32 / tbf,
            "algorithmic_tflops": flops / tbf / 1e12,
            "frac_of_bf16_peak_algorithmic": flops / tbf / PEAK_BF16_MFMA,
            "kernel": embed_kernel("bf16", w["p"], w["l"], w["r"]),
            "lo_passes_skipped": lo_zero,
            "products": ("hi.hi only: data and landmarks are integers 0..255, exact in BF16, so "
                         "every lo part is zero and the lo products are skipped"
                         if lo_zero else
                         "hi.hi + lo.hi + hi.lo + lo.lo (data lo parts nonzero)")},
        "split_fp16": {"embed_ms": t16 * 1e3, "points_per_s": n / t16, "speedup_vs_fp32": t32 / t16},
        "embed_fp64_ms": t64 * 1e3,
        "err_vs_gpu_fp64_all_rows": err_vs64,
    }
    fit_o = None
    if cpu:
        log(f"[{name}] cpu baseline (oracle)")
        base, errs, fit_o, _, _ = cpu_baseline(
            name, X, w, args.cpu_sample,
            100_000 if name == "wide" else 50_000,
            {"fp32": Y32.cpu().numpy(), "split_bf16": Ybf.cpu().numpy(),
             "split_fp16": Y16.cpu().numpy(), "fp64": Y64n})
        rep["cpu_baseline"] = base
        rep["err_vs_oracle_sample"] = errs
    return rep, dict(X=X, Xd=Xd, model=model, Y32=Y32, Y64=Y64, Y64n=Y64n, fit_o=fit_o)


def small_leg(mds, torch, dev, cpu):
    """Latency at 5,000 x 10, FP64 (fit and embed), each landmark seed: GPU
    medians of 10 (wall time around a synchronous fit; HIP events around the
    embed), the host oracle's medians of 10 (all cores, and one thread),
    and the error against the oracle."""
    import oracle
    from synth import errors
    from synth import generators as gen
    s = SMALL
    X = gen.small_gaussian(s["n"], seed=11)
    Xd = torch.from_numpy(X).to(dev)
    st = torch.cuda.current_stream()
    out = {"config": s["desc"], "seeds": []}
    for seed in s["seeds"]:
        fits = []
        for _ in range(11):
            torch.cuda.synchronize()
            t = time.perf_counter()
            model = mds.fit_landmarks(Xd, s["l"], s["r"], seed=seed)
            fits.append((time.perf_counter() - t) * 1e3)
            model.free()
        model = mds.fit_landmarks(Xd, s["l"], s["r"], seed=seed)
        Y = mds.embed(model, Xd, prec="fp64")
        torch.cuda.synchronize()
        embs, whole = [], []
        for _ in range(10):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            mds.embed(model, Xd, prec="fp64", Y=Y)
            e1.record(st)
            torch.cuda.synchronize()
            embs.append(e0.elapsed_time(e1))
        for _ in range(10):
            torch.cuda.synchronize()
            t = time.perf_counter()
            m2 = mds.fit_landmarks(Xd, s["l"], s["r"], seed=seed)
            mds.embed(m2, Xd, prec="fp64", Y=Y)
            torch.cuda.synchronize()
            whole.append((time.perf_counter() - t) * 1e3)
            m2.free()
        rec = {"landmark_seed": seed, "fit_ms_median": float(np.median(fits[1:])),
               "embed_ms_median": float(np.median(embs)),
               "fit_plus_embed_ms_median": float(np.median(whole)),
               "points_per_s": s["n"] / (np.median(whole) / 1e3)}
        fit_o = oracle.fit_landmarks(X, s["l"], s["r"], seed=seed)
        Yo = oracle.interpolate(fit_o, X)
        e = errors.column_errors(Y.cpu().numpy(), Yo)
        rec["err_vs_oracle"] = {k: e[k] for k in ("rms_rel", "maxabs_rms")}
        rec["landmarks_equal_oracle"] = bool(np.array_equal(model.landmarks(), fit_o.idx))
        if cpu:
            def oracle_once():
                f = oracle.fit_landmarks(X, s["l"], s["r"], seed=seed)
                oracle.interpolate(f, X)
            tt = []
            for _ in range(10):
                t = time.perf_counter()
                oracle_once()
                tt.append((time.perf_counter() - t) * 1e3)
            with one_thread():
                t1 = []
                for _ in range(10):
                    t = time.perf_counter()
                    oracle_once()
                    t1.append((time.perf_counter() - t) * 1e3)
            rec["oracle_ms_median"] = float(np.median(tt))
            rec["oracle_one_thread_ms_median"] = float(np.median(t1))
        model.free()
        out["seeds"].append(rec)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="image",
                    help="headline workload (the other one runs as a leg unless --no-wide)")
    ap.add_argument("--embed-iters", type=int, default=20)
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-sqdist", action="store_true")
    ap.add_argument("--serve-multi", type=int, default=20000,
                    help="requests in the 48-model multi-tenant mix (0: skip it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-wide", action="store_true", help="skip the legs on the other workload")
    ap.add_argument("--no-small", action="store_true", help="skip the 5,000 x 10 FP64 latency leg")
    ap.add_argument("--cpu-sample", type=int, default=200_000)
    ap.add_argument("--only-embed", choices=["fp32", "split_bf16", "split_fp16", "fp64"])
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--only-fit", action="store_true", help="run --iters fits only (profiling)")
    ap.add_argument("--copy-calib", type=int, default=0)
    ap.add_argument("--no-dc", action="store_true")
    ap.add_argument("--no-affine", action="store_true")
    ap.add_argument("--no-pivot", action="store_true")
    ap.add_argument("--dc-iters", type=int, default=5)
    ap.add_argument("--only-dc", action="store_true", help="run --iters divide-and-conquer calls only")
    ap.add_argument("--only-affine", action="store_true", help="run --iters affine embeds only")
    ap.add_argument("--only-sqdist", action="store_true",
                    help="run --iters embeds from squared dissimilarities only")
    ap.add_argument("--only-pivot", action="store_true",
                    help="run one MaxMin selection and --iters pivot MDS calls only")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(rows would shard across GPUs after one broadcast of the model). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2007_11919_amd as mds
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")

    if args.copy_calib:
        n = args.copy_calib // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes": n * 4, "launches": 5}))
        return

    if args.only_dc:
        from synth import generators as gen
        X = gen.paper_design(DC["n"], DC["k"], DC["h"], seed=15, dtype=np.float32)
        Xd = torch.from_numpy(X).to(dev)
        for _ in range(args.iters):
            mds.divide_conquer(Xd, DC["l"], DC["c"], DC["r"], seed=6)
        torch.cuda.synchronize()
        print(json.dumps({"only_dc": args.iters}))
        return

    if args.only_fit or args.only_affine or args.only_sqdist or args.only_pivot or args.only_embed:
        w = WORKLOADS[args.workload]
        log(f"generating {args.workload} data")
        X = make_data(args.workload)
        Xd = torch.from_numpy(X).to(dev)
        torch.cuda.synchronize()
        if args.only_fit:
            for _ in range(args.iters):
                mds.fit_landmarks(Xd, w["l"], w["r"], seed=0).free()
            torch.cuda.synchronize()
            print(json.dumps({"only_fit": args.iters}))
            return
        if args.only_pivot:
            mds.maxmin_landmarks(Xd, 200, 0)
            for _ in range(args.iters):
                mds.pivot_mds(Xd, 200, 10, seed=4)
            torch.cuda.synchronize()
            print(json.dumps({"only": "pivot", "iters": args.iters}))
            return
        model = mds.fit_landmarks(Xd, w["l"], w["r"], seed=0)
        if args.only_embed:
            Y = mds.embed(model, Xd, prec=args.only_embed)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.iters):
                mds.embed(model, Xd, prec=args.only_embed, Y=Y)
            e1.record()
            torch.cuda.synchronize()
            print(json.dumps({"only_embed": args.only_embed, "iters": args.iters,
                              "ms_per_launch": e0.elapsed_time(e1) / max(1, args.iters)}))
            return
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        if args.only_affine:
            Y = mds.embed_affine(model, Xd, prec="fp32")
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.iters):
                mds.embed_affine(model, Xd, prec="fp32", Y=Y)
            e1.record()
        else:
            idx = torch.from_numpy(model.landmarks()).to(dev)
            M = Xd[idx]
            A2 = torch.empty((w["n"], w["l"]), dtype=torch.float32, device=dev)
            mn = (M * M).sum(1)
            for s0 in range(0, w["n"], 100_000):
                xb = Xd[s0:s0 + 100_000]
                A2[s0:s0 + 100_000] = ((xb * xb).sum(1, keepdim=True) + mn[None, :]
                                       - 2.0 * (xb @ M.T)).clamp_min_(0)
            Y = mds.embed_from_sqdist(model, A2, prec="fp32")
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.iters):
                mds.embed_from_sqdist(model, A2, prec="fp32", Y=Y)
            e1.record()
        torch.cuda.synchronize()
        print(json.dumps({"only": "affine" if args.only_affine else "sqdist", "iters": args.iters,
                          "ms_per_launch": e0.elapsed_time(e1) / max(1, args.iters)}))
        return

    cpu = not args.no_cpu_baseline
    head, h = workload_run(mds, torch, args.workload, args, dev, cpu)
    w = WORKLOADS[args.workload]
    out = {
        "metric": "embedded points/s, FP32 vs split-BF16 at stated err; serving p50/p99 latency",
        "value": head["points_per_s"], "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
    }
    out.update({k: v for k, v in head.items() if k not in ("ms_per_step", "points_per_s")})
    if not cpu:
        out["cpu_baseline"] = None
    out["paper_context"] = ("paper (R, one i9-10900K): interpolation MDS of 814,255 x 784 images "
                            "with l=250 in 98.55 s (about 8,260 points/s), and of 10^6 x 100 rows "
                            "with l=250 in 18.34 s (about 54,500 points/s); other l, not a target")
    if args.workload == "image" and not args.no_affine:
        log("[image] affine form")
        out["embed_affine"] = affine_leg(mds, torch, h["model"], h["Xd"], h["Y64n"], args.embed_iters)
    h["model"].free()
    del h

    if not args.no_wide and args.workload == "image":
        torch.cuda.empty_cache()
        wide, g = workload_run(mds, torch, "wide", args, dev, cpu)
        model, Xd, X = g["model"], g["Xd"], g["X"]
        if not args.no_sqdist:
            log("[wide] embedding from squared dissimilarities")
            wide["embed_from_sqdist"] = sqdist_leg(mds, torch, model, Xd, g["Y32"], args.embed_iters)
        if not args.no_affine:
            log("[wide] affine form")
            wide["embed_affine"] = affine_leg(mds, torch, model, Xd, g["Y64n"], args.embed_iters)
        if not args.no_pivot:
            log("[wide] maxmin and pivot MDS")
            wide["maxmin_pivot"] = pivot_leg(mds, torch, Xd, X, args.dc_iters, cpu)
        if not args.no_serve:
            log("[wide] serving runs")
            fit_o = g["fit_o"]
            if fit_o is None:
                import oracle
                fit_o = oracle.fit_landmarks(X, WORKLOADS["wide"]["l"], WORKLOADS["wide"]["r"], seed=0)
            budget = 8 << 30
            out["serving"] = {"model": WORKLOADS["wide"]["desc"], "budget_bytes": budget, "runs": [
                serving_run(mds, torch, model, Xd, prec, args.serve_requests, 5, budget, g["Y64"],
                            fit_o, X)
                for prec in ("fp32", "split_bf16")]}
        model.free()
        del g, model, Xd, X
        torch.cuda.empty_cache()
        if not args.no_dc:
            log("divide-and-conquer MDS")
            wide["divide_conquer"] = dc_leg(mds, torch, args.dc_iters, cpu)
        out["wide"] = wide
    if not args.no_small:
        log("5,000 x 10 FP64 latency")
        out["small_fp64"] = small_leg(mds, torch, dev, cpu)
    if args.serve_multi:
        log("multi-tenant serving")
        torch.cuda.empty_cache()
        out["serving_multi"] = serving_multi(mds, torch, args.serve_multi, 31, 24 << 30)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
