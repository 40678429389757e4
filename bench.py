"""Benchmark: Gaussian log-likelihood evaluations per second at n = 99,856 on one MI355X.

One step = one whole evaluation of eq. (2) through the C-ABI one-shot entry point with the
inputs resident in HBM: Z-order ordering of the locations, Matérn covariance tiles, the
mixed-precision tile Cholesky with the fused forward solve, log-determinant and reduction.

The timed (headline) path is the paper's own method at its own precision: the two-tier band
plan of Algorithm 1, FP64 within 2 tiles of the diagonal and FP32 beyond, tile 512.  Beside
it, on the same inputs, each leg with its own dtype and roofline: the three-precision-tier
plan (the paper's future work: FP64 band 2, FP32 for the next 8 tiles, FP16 operands beyond,
power-of-two scaled per tile row, FP32 accumulation) and the all-FP64 path; the log-likelihood
error of each mixed path against the FP64 path is reported.

Inputs: a jittered 316 x 316 grid in ]0,1[^2 (n = 99,856), theta = (1, 0.1, 0.5), and z a
draw of the Matérn field at theta (z = L eps with L the library's FP64 factor, drawn once
before timing).  The CPU baseline times the FP64 oracle on a smaller grid of the same kind
and scales the time by (n / n_sample)^3.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "log-lik evals/sec + Cholesky TFLOP/s at n=100k (mixed vs FP64); p50/p99 latency"
PEAK_FP16_MATRIX = 2516.6  # TFLOP/s, MI355X dense FP16 / BF16 matrix
PEAK_FP32_MATRIX = 157.3   # TFLOP/s, MI355X dense FP32 matrix
PEAK_FP64_MATRIX = 78.6    # TFLOP/s, MI355X dense FP64 matrix
PEAKS = {"update_lowp": PEAK_FP16_MATRIX, "update_fp32": PEAK_FP32_MATRIX,
         "update_fp64": PEAK_FP64_MATRIX}
PEAK_HBM_GBS = 8000.0      # GB/s, MI355X HBM3E
# committed rocprofv3 FETCH_SIZE / WRITE_SIZE summaries, one per update kernel, each naming
# the kernel source it was measured on (the figure is void once that source changed)
TRAFFIC_PROFILES = {
    "update_lowp": (["update_lowp_hbm_traffic_matern-n99856-nb512-band2-band32_8-fp16.md",
                     "update_lowp_hbm_traffic_matern-n99856-nb512-band2-band32_10-fp16.md"], "lowp.hip"),
    "update_fp32": (["update_fp32_hbm_traffic_matern-n99856-nb512-band2.md"], "gemm.hip"),
}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of an update kernel from its committed rocprofv3 counter summary,
    or None when there is none for this workload or the kernel source changed since."""
    import hashlib
    import re
    if kernel not in TRAFFIC_PROFILES:
        return None
    fnames, src = TRAFFIC_PROFILES[kernel]
    source = os.path.join(ROOT, "paper_2003_05324_amd", "csrc", src)
    digest = hashlib.sha256(open(source, "rb").read()).hexdigest()
    for fname in fnames:
        path = os.path.join(ROOT, "profiles", fname)
        if not os.path.exists(path):
            continue
        text = open(path).read()
        wl = re.search(r"workload: (\S+)", text)
        sha = re.search(r"sha256 at measurement: ([0-9a-f]+)", text)
        val = re.search(r"traffic_bytes_per_launch: ([0-9.e+]+)", text)
        if wl and wl.group(1) == workload and sha and sha.group(1) == digest and val:
            return float(val.group(1))
    return None


def roofline(stats, workload):
    """Roofline of the dominant kernel: the update class with the largest share of the
    algorithmic flops.  Its bound follows from its arithmetic intensity: below the ridge
    point peak_flops / peak_bandwidth it is HBM-bound and is rated in GB/s of algorithmic
    bytes, above it MFMA-bound and rated in TFLOP/s."""
    updates = [s for s in stats if s["name"] in PEAKS and s["launches"]]
    dom = max(updates, key=lambda s: s["flops"])
    peak_flops = PEAKS[dom["name"]]
    intensity = dom["flops"] / dom["bytes"]
    ridge = peak_flops * 1e12 / (PEAK_HBM_GBS * 1e9)
    tflops = dom["flops"] / dom["seconds"] / 1e12
    gbs = dom["bytes"] / dom["seconds"] / 1e9
    out = {"kernel": dom["name"]}
    if intensity < ridge:
        out.update({"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": gbs / PEAK_HBM_GBS})
    else:
        out.update({"bound": "mfma", "achieved": tflops, "peak": peak_flops, "unit": "TFLOP/s",
                    "frac": tflops / peak_flops})
    traffic = measured_traffic(dom["name"], workload)
    out.update({
        "traffic": traffic,
        "algorithmic_bytes_per_launch": dom["bytes"] / dom["launches"],
        "flops_per_launch": dom["flops"] / dom["launches"],
        "intensity_flop_per_byte": intensity,
        "ridge_flop_per_byte": ridge,
        "tflops": tflops,
        "tflops_frac_of_matrix_peak": tflops / peak_flops,
        "avg_launch_ms": 1e3 * dom["seconds"] / dom["launches"],
        "launches": dom["launches"],
    })
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--three-tier-steps", type=int, default=3)
    ap.add_argument("--legs", default="two_tier,three_tier,three_tier_wide,fp64",
                    help="comma list of the paths to time: two_tier (the headline: --steps/--warmup), "
                         "three_tier and three_tier_wide (--three-tier-steps), fp64 (--fp64-steps); profiling runs may "
                         "leave out the headline, and then print no value")
    ap.add_argument("--band32", type=int, default=8,
                    help="FP32 tiles beyond the FP64 band in the three-tier leg")
    ap.add_argument("--band32-wide", type=int, default=10,
                    help="FP32 width of a second three-tier leg (three_tier_wide; 0: none)")
    ap.add_argument("--lowp", default="fp16", choices=["fp16", "bf16", "none"])
    ap.add_argument("--m", type=int, default=316, help="grid side (n = m*m)")
    ap.add_argument("--tile", type=int, default=512)
    ap.add_argument("--band", type=int, default=2)
    ap.add_argument("--cpu-sample-m", type=int, default=160)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--heldout", type=int, default=2000, help="kriging sites (0: skip)")
    ap.add_argument("--batch", type=int, default=0,
                    help="instead of the headline: a batch of this many independent problems "
                         "(n log-uniform in [500, 8000]) through the batched entry point, against "
                         "one-at-a-time evaluation; one JSON line")
    ap.add_argument("--serve", type=int, default=0,
                    help="instead of the headline: this many requests (Poisson arrivals, theta along "
                         "Nelder-Mead trajectories) for 16 resident datasets (n log-uniform in "
                         "[2000, 60000], the small ones through the persistent queue) through the "
                         "serving loop, three-tier, two-tier and FP64 plans; one JSON line")
    ap.add_argument("--serve-rate", type=float, default=4.0, help="arrivals per second")
    ap.add_argument("--serve-theta", default="trajectory", choices=["trajectory", "lognormal"],
                    help="request theta: along Nelder-Mead trajectories, or log-normal around theta_0 "
                         "with nu = 1/2 fixed")
    ap.add_argument("--serve-queue-max-n", type=int, default=4096,
                    help="datasets up to this n are served through the persistent queue (0: none)")
    ap.add_argument("--small", action="store_true",
                    help="instead of the headline: the n = 1,600 plain-method workload (40 x 40 "
                         "jittered grid, tile 160, FP64 band 2): --repeats evaluations at the true "
                         "theta and its 8 corners on the FP64 and band paths (p50/p99 latency, "
                         "evals/s) and the maximum-likelihood fit on the GPU beside the oracle's; one "
                         "JSON line")
    ap.add_argument("--repeats", type=int, default=100)
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the headline: the n = 40,000 band sweep (6 fields x bands "
                         "0, 1, 4, 16, all), one JSON line")
    ap.add_argument("--sweep-fields", default="",
                    help="comma list of sweep field indices (0-5) to run (default: all)")
    ap.add_argument("--sweep-mle", action="store_true",
                    help="with --sweep: also the maximum-likelihood fit of theta at bands 0, 4 and "
                         "all (Nelder-Mead from theta_0 * (1.5, 0.5, 1.2), xtol 1e-5 in log-theta)")
    return ap.parse_args()


def percentile(xs, q):
    xs = sorted(xs)
    if len(xs) == 1:
        return xs[0]
    pos = (len(xs) - 1) * q
    lo = int(math.floor(pos))
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (pos - lo)


def time_path(mp, ctx, locs, z, theta, tile, band, steps, warmup, band32=-1, lowp=None):
    """warmup + timed steps of the one-shot evaluation; returns wall time and per-step results."""
    import torch
    for _ in range(warmup):
        ctx.loglik(locs, z, theta, tile, band, band32=band32, lowp=lowp)
    ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [ctx.loglik(locs, z, theta, tile, band, timing=True, band32=band32, lowp=lowp)
               for _ in range(steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, results, ctx.kernel_stats()


def leg_summary(wall, res, steps, n, ll_ref=None, stats=None, workload=None, dtype=None):
    chol_flops = n ** 3 / 3.0
    out = {
        "evals_per_s": steps / wall,
        "ms_per_step": 1e3 * wall / steps,
        "cholesky_tflops": chol_flops / statistics.median([r["t_factor"] for r in res]) / 1e12,
        "p50_s": percentile([r["t_total"] for r in res], 0.5),
        "p99_s": percentile([r["t_total"] for r in res], 0.99),
        "loglik": res[-1]["loglik"],
        "logdet": res[-1]["logdet"],
    }
    if ll_ref is not None:
        out["dloglik_rel_vs_fp64"] = abs(res[-1]["loglik"] - ll_ref) / abs(ll_ref)
        out["dloglik_relmax_vs_fp64"] = abs(res[-1]["loglik"] - ll_ref) / max(abs(ll_ref), n)
    if dtype is not None:
        out["dtype"] = dtype
    if workload is not None:
        out["workload"] = workload
    if stats:
        out["roofline"] = roofline(stats, workload)
        out["kernel_streams"] = stream_occupancy(stats)
    return out


def stream_occupancy(stats):
    """Per kernel class: launches and HIP-event time between the events around each launch on
    its stream.  Kernels of the three streams share the compute units, so these times include
    waiting for units held by other kernels: stream occupancy, not kernel rates."""
    return {"note": "HIP-event seconds per kernel class on its own stream, including waits for "
                    "compute units held by concurrent kernels (occupancy, not kernel rates)",
            "classes": {s["name"]: {"launches": s["launches"], "seconds": s["seconds"],
                                    "algorithmic_tflops": (s["flops"] / s["seconds"] / 1e12) if s["seconds"] else None,
                                    "algorithmic_gbs": (s["bytes"] / s["seconds"] / 1e9) if s["seconds"] else None}
                        for s in stats if s["launches"]}}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(m_sample, n_full, theta):
    """The oracle's evaluation of eq. (2) on a bounded sample of the workload, timed in its two
    parts (covariance matrix: n^2 kernel evaluations; Cholesky + triangular solve: n^3/3 flops)
    and each part scaled to n_full by its own order.  Both parts use the host's cores: the
    covariance matrix as row blocks of the oracle's own eq. (1) (cross distances, Matérn) on a
    thread pool (its Bessel routine releases the interpreter lock), the factorization through
    the multi-threaded LAPACK the oracle calls."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import threadpoolctl

    import oracle
    from synthetic import jittered_grid, normals
    locs = jittered_grid(m_sample, 901)
    n = len(locs)
    z = normals(n, 902)
    blas = max((i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()
                if i.get("user_api") == "blas"), default=1)
    workers = max(1, min(blas, len(os.sched_getaffinity(0))))
    sig = np.empty((n, n))
    rows = np.array_split(np.arange(n), 8 * workers)

    def fill(r):
        sig[r] = oracle.matern(oracle.cross_distances(locs[r], locs), *theta)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=workers) as pool:
        list(pool.map(fill, rows))
    t_cov = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.likelihood.loglik_parts(sig, z)
    t_fac = time.perf_counter() - t0
    del sig
    s2, s3 = (n_full / n) ** 2, (n_full / n) ** 3
    t_full = t_cov * s2 + t_fac * s3
    return {
        "value": 1.0 / t_full,
        "unit": "evals/s",
        "cores": int(workers),
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": (f"oracle eq. (2) on a {m_sample}x{m_sample} jittered grid (n={n}) on {workers} "
                   f"threads of a {cpu_model()}: covariance matrix (scipy K_nu, row blocks on a "
                   f"thread pool) {t_cov:.2f} s, scaled by (n_full/n)^2 = {s2:.1f}; LAPACK Cholesky "
                   f"+ triangular solve ({blas} BLAS threads) {t_fac:.2f} s, scaled by "
                   f"(n_full/n)^3 = {s3:.1f}; {t_full:.0f} s per evaluation at n={n_full}"),
        "sample_seconds": t_cov + t_fac,
    }


def small_bench(args):
    """The n = 1,600 workload of the plain method: 40 x 40 jittered grid (seed 101), theta_0 =
    (1, 0.1, 0.5), z the oracle's draw of the field stored in tests/golden/small_z.txt (the
    input of the oracle's stored fit; the Nelder-Mead end point moves by about 1e-2 in theta
    when z changes by rounding, the likelihood being that flat near its maximum), tile 160,
    FP64 band 2.  Each of the 9 theta (theta_0 and the corners
    theta_0 (1 +- 0.1)) is evaluated --repeats times on the all-FP64 and the band path of a
    resident dataset; latency is the host wall time of each synchronous call.  Then the
    Nelder-Mead fit of theta on the GPU (both paths) beside the oracle's fit of the same
    workload, stored by tests/golden/make_golden.py (which calls only the oracle)."""
    import numpy as np
    import torch

    import paper_2003_05324_amd as mp
    from synthetic import SMALL, perturbed_thetas
    w = SMALL
    ctx = mp.Context(0)
    zfile = os.path.join(ROOT, "tests", "golden", "small_z.txt")
    if os.path.exists(zfile):   # the oracle's draw, the input of its stored fit
        z = np.loadtxt(zfile)
    else:
        gen = mp.Dataset(ctx, w.locations(), None)
        z = gen.simulate(w.theta, w.eps(), w.tile, -1)
        gen.close()
    ds = mp.Dataset(ctx, w.locations(), z)
    thetas = [w.theta] + perturbed_thetas(w.theta)
    out = {"small": w.name, "n": w.n, "tile": w.tile, "band64": w.band64, "repeats": args.repeats,
           "thetas": len(thetas)}
    ll = {}
    for name, band in (("fp64", -1), ("band2", w.band64)):
        for th in thetas:
            ds.loglik(th, w.tile, band)                                    # warm-up
        lat = []
        torch.cuda.synchronize()
        t_all = time.perf_counter()
        for th in thetas:
            for _ in range(args.repeats):
                t0 = time.perf_counter()
                r = ds.loglik(th, w.tile, band)
                lat.append(time.perf_counter() - t0)
            ll[(name, th)] = r["loglik"]
        wall = time.perf_counter() - t_all
        out[name] = {"p50_latency_s": percentile(lat, 0.5), "p99_latency_s": percentile(lat, 0.99),
                     "evals_per_s": 1.0 / percentile(lat, 0.5), "throughput_evals_per_s": len(lat) / wall,
                     "loglik_theta0": ll[(name, w.theta)]}
        print(f"[small] {name}: {out[name]}", file=sys.stderr, flush=True)
    out["max_rel_dloglik_band2_vs_fp64"] = max(abs(ll[("band2", th)] - ll[("fp64", th)]) / abs(ll[("fp64", th)])
                                               for th in thetas)
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "mle_small.json")))
    start = [min(max(t * sc, lo), hi) for t, sc, lo, hi in
             zip(w.theta, (1.5, 0.5, 1.2), (0.01, 0.001, 0.1), (10.0, 2.0, 3.0))]
    out["mle"] = {"start": start, "oracle": {k: gold[k] for k in ("theta_hat", "loglik_hat", "evals", "iters",
                                                                 "seconds")}}
    for name, band in (("fp64", -1), ("band2", w.band64)):
        t0 = time.perf_counter()
        fit = ds.mle(start, w.tile, band)
        sec = time.perf_counter() - t0
        out["mle"][name] = {"theta_hat": list(fit["theta"]), "loglik_hat": fit["loglik"], "evals": fit["evals"],
                            "iters": fit["iters"], "seconds": sec,
                            "max_rel_dtheta_vs_oracle": max(abs(a - b) / abs(b) for a, b in
                                                            zip(fit["theta"], gold["theta_hat"]))}
        print(f"[small] mle {name}: {out['mle'][name]}", file=sys.stderr, flush=True)
    ds.close()
    ctx.close()
    if not args.no_cpu_baseline:
        # the oracle's evaluation of eq. (2) at theta_0 on the same workload, repeated for ~10 s
        import oracle
        locs = w.locations()
        zz = oracle.simulate_field(locs, w.theta, w.eps())
        reps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < 10.0:
            oracle.loglik(locs, zz, w.theta)
            reps += 1
        sec = (time.perf_counter() - t0) / reps
        out["cpu_baseline"] = {"value": 1.0 / sec, "unit": "evals/s", "cores": len(os.sched_getaffinity(0)),
                               "cpu_model": cpu_model(), "kind": "oracle",
                               "sample": f"oracle eq. (2) at theta_0 on the n = 1,600 workload, {reps} "
                                         f"evaluations in {reps * sec:.1f} s"}
    print(json.dumps(out), flush=True)


def band_sweep(args):
    """n = 40,000 band sweep: sigma2 = 1, beta in {0.03, 0.1, 0.3} x nu in {0.5, 1.0}, each field
    drawn by the library's FP64 sampler; for every FP64 band b the log-likelihood at the true
    theta, its error against the all-FP64 path and against the oracle's eq. (2) at the true
    theta (stored in tests/golden/sweep_n40000.json by a script that calls only the oracle; the
    oracle's z = L eps comes from its own factor, equal to the library's draw to rounding), SPD
    failures and the factor rate; with --sweep-mle the maximum-likelihood fit of theta at bands
    0, 4 and all."""
    import torch

    import paper_2003_05324_amd as mp
    from synthetic import SWEEP
    gold_path = os.path.join(ROOT, "tests", "golden", "sweep_n40000.json")
    gold = {}
    if os.path.exists(gold_path):
        gold = {f["field"]: f for f in json.load(open(gold_path))["fields"]}
    fields = [int(x) for x in args.sweep_fields.split(",")] if args.sweep_fields else range(len(SWEEP))
    ctx = mp.Context(0)
    dev = torch.device("cuda:0")
    rows, fits = [], []
    for fi in fields:
        w = SWEEP[fi]
        locs = torch.from_numpy(w.locations()).to(dev)
        gen = mp.Dataset(ctx, locs, None)
        z = gen.simulate(w.theta, torch.from_numpy(w.eps()).to(dev), w.tile, -1)
        gen.close()
        ds = mp.Dataset(ctx, locs, z)
        ref = None
        og = gold.get(w.name)
        for band in sorted(w.bands, key=lambda b: (b < 0, b), reverse=True):   # all-FP64 first
            st, _ = ds.try_loglik(w.theta, w.tile, band)                       # warm-up
            times, res = [], None
            if st == 0:
                for _ in range(args.steps):
                    res = ds.loglik(w.theta, w.tile, band, timing=False)
                    times.append(res["t_factor"])
            row = {"field": w.name, "beta": w.theta[1], "nu": w.theta[2], "band64": band,
                   "status": mp.status_string(st)}
            if res is not None:
                t = statistics.median(times)
                row.update({"loglik": res["loglik"], "logdet": res["logdet"], "quad": res["quad"],
                            "t_factor_s": t, "cholesky_tflops": w.n ** 3 / 3.0 / t / 1e12})
                if og is not None:
                    row["dloglik_rel_vs_oracle"] = abs(res["loglik"] - og["loglik"]) / abs(og["loglik"])
                    row["dlogdet_rel_vs_oracle"] = abs(res["logdet"] - og["logdet"]) / abs(og["logdet"])
                if band < 0:
                    ref = res
                elif ref is not None:
                    row["dloglik_rel_vs_fp64"] = abs(res["loglik"] - ref["loglik"]) / abs(ref["loglik"])
                    row["dlogdet_rel"] = abs(res["logdet"] - ref["logdet"]) / abs(ref["logdet"])
                    row["dquad_rel"] = abs(res["quad"] - ref["quad"]) / ref["quad"]
            rows.append(row)
            print(f"[sweep] {row}", file=sys.stderr, flush=True)
        if args.sweep_mle:
            start = [min(max(t * sc, lo), hi) for t, sc, lo, hi in
                     zip(w.theta, (1.5, 0.5, 1.2), (0.01, 0.001, 0.1), (10.0, 2.0, 3.0))]
            fit_ref = None
            for band in (-1, 4, 0):
                t0 = time.perf_counter()
                try:
                    fit = ds.mle(start, w.tile, band, xtol=1e-5)
                except mp.MpgeoError as e:
                    fit = {"error": str(e)}
                sec = time.perf_counter() - t0
                f = {"field": w.name, "band64": band, "start": start, "seconds": sec}
                f.update(fit)
                if "theta" in fit:
                    if band < 0:
                        fit_ref = fit
                    elif fit_ref is not None:
                        f["max_rel_dtheta_vs_fp64_fit"] = max(abs(a - b) / abs(b) for a, b in
                                                              zip(fit["theta"], fit_ref["theta"]))
                fits.append(f)
                print(f"[sweep] mle {f}", file=sys.stderr, flush=True)
        ds.close()
    for r in rows:
        base = next(x for x in rows if x["field"] == r["field"] and x["band64"] < 0)
        if "t_factor_s" in r and "t_factor_s" in base:
            r["speedup_vs_fp64"] = base["t_factor_s"] / r["t_factor_s"]
    ctx.close()
    out = {"sweep": "matern-n40000-nb512", "steps": args.steps, "rows": rows}
    if args.sweep_mle:
        out["mle"] = fits
    print(json.dumps(out), flush=True)


def batch_bench(args):
    """Batched evaluation: `args.batch` problems with their own sites, theta and data (a draw of
    each problem's field), all-FP64 plan, tiles from the autotuner (tuned on an untimed first batch), against evaluating the
    same problems one after another through the one-shot entry point (tile 512); then the
    persistent task queue, all-FP64 and with FP64-band/FP32 tiles whose band the tuner picks per
    class of n."""
    import numpy as np
    import torch

    import oracle
    import paper_2003_05324_amd as mp
    from synthetic import batch_instances
    ctx = mp.Context(0)
    # each problem's data: a draw of its own field by the library's FP64 sampler (its normal
    # vector as eps), as the paper's synthetic data are drawn from the model
    probs = []
    for locs, eps, theta in batch_instances(args.batch, 11):
        gen = mp.Dataset(ctx, locs, None)
        probs.append((locs, np.asarray(gen.simulate(theta, eps, 128, -1)), theta))
        gen.close()
    ns = np.array([len(z) for _, z, _ in probs])
    flops = float(np.sum(ns.astype(np.float64) ** 3 / 3.0))
    print(f"[batch] {len(probs)} problems, n in [{ns.min()}, {ns.max()}], sum n^3/3 = {flops:.3e}",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    st, _, tiles = ctx.batch_loglik(probs, tile=0, band64=-1)          # tunes the tile sizes
    t_tune = time.perf_counter() - t0
    walls = []
    for _ in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, res, tiles = ctx.batch_loglik(probs, tile=0, band64=-1)
        walls.append(time.perf_counter() - t0)
    wall = statistics.median(walls)
    print(f"[batch] batched: {wall:.3f} s (tuning pass {t_tune:.2f} s)", file=sys.stderr, flush=True)
    # the same batch as one persistent kernel over a device task queue (tile 128)
    st_q, res_q, _ = ctx.batch_loglik(probs, tile=0, band64=-1, queue=True)   # warm-up
    walls_q = []
    for _ in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st_q, res_q, _ = ctx.batch_loglik(probs, tile=0, band64=-1, queue=True)
        walls_q.append(time.perf_counter() - t0)
    wall_q = statistics.median(walls_q)
    print(f"[batch] task queue: {wall_q:.3f} s", file=sys.stderr, flush=True)
    # the same queue with FP64-band/FP32 tiles, the band of each class chosen by the tuner
    # (MPGEO_TUNE_BAND; the first call probes, untimed), problems that are not positive definite
    # at their band widened (MPGEO_ESCALATE)
    ctx.batch_loglik(probs, tile=0, queue=True, tune_band=True, escalate=True)
    walls_b = []
    for _ in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st_b, res_b, _ = ctx.batch_loglik(probs, tile=0, queue=True, tune_band=True, escalate=True)
        walls_b.append(time.perf_counter() - t0)
    wall_b = statistics.median(walls_b)
    bands = {}
    for r in res_b:
        key = "all" if r["band64"] < 0 else str(r["band64"])
        bands[key] = bands.get(key, 0) + 1
    print(f"[batch] task queue, tuned bands {bands}: {wall_b:.3f} s", file=sys.stderr, flush=True)
    for locs, z, theta in probs[:2]:
        ctx.loglik(locs, z, theta, 512, -1)                              # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq = [ctx.loglik(locs, z, theta, 512, -1) for locs, z, theta in probs]
    t_seq = time.perf_counter() - t0
    print(f"[batch] one at a time: {t_seq:.3f} s", file=sys.stderr, flush=True)
    dev = max(abs(a["loglik"] - b["loglik"]) / max(abs(b["loglik"]), len(p[1]))
              for a, b, p in zip(res, seq, probs))
    dev_q = max(abs(a["loglik"] - b["loglik"]) / max(abs(b["loglik"]), len(p[1]))
                for a, b, p in zip(res_q, seq, probs))
    errs_b = [abs(a["loglik"] - b["loglik"]) / abs(b["loglik"]) for a, b in zip(res_b, seq)]
    dev_b = max(errs_b)
    # the same errors against the size of eq. (2)'s terms, the tuner's scale (l itself passes
    # through zero for the smoothest fields)
    terms_b = [abs(a["loglik"] - b["loglik"]) /
               (0.5 * (len(p[1]) * np.log(2 * np.pi) + abs(b["logdet"]) + abs(b["quad"])))
               for a, b, p in zip(res_b, seq, probs)]
    # oracle spot check on the three smallest problems
    small = np.argsort(ns)[:3]
    want = {q: oracle.loglik(*probs[q])["loglik"] for q in small}
    orc = max(abs(res[q]["loglik"] - want[q]) / abs(want[q]) for q in small)
    orc_q = max(abs(res_q[q]["loglik"] - want[q]) / abs(want[q]) for q in small)
    orc_b = max(abs(res_b[q]["loglik"] - want[q]) / abs(want[q]) for q in small)
    hist = {}
    for t in tiles:
        hist[str(t)] = hist.get(str(t), 0) + 1
    ctx.close()
    print(json.dumps({
        "batch": "matern-batch512-n500-8000" if args.batch == 512 else f"matern-batch{args.batch}-n500-8000",
        "problems": len(probs), "status": st, "sum_n3_over_3": flops,
        "batched_s": wall, "batched_evals_per_s": len(probs) / wall,
        "batched_tflops": flops / wall / 1e12,
        "sequential_s": t_seq, "sequential_evals_per_s": len(probs) / t_seq,
        "speedup": t_seq / wall, "tuning_pass_s": t_tune, "tiles": hist,
        "max_dloglik_batched_vs_sequential": dev, "max_rel_dloglik_vs_oracle_3_smallest": orc,
        "lanes": int(os.environ.get("MPGEO_BATCH_LANES", "4")),
        "queue": {"status": st_q, "seconds": wall_q, "evals_per_s": len(probs) / wall_q,
                  "tflops": flops / wall_q / 1e12, "speedup_vs_lanes": wall / wall_q,
                  "speedup_vs_sequential": t_seq / wall_q, "tile": 128,
                  "max_dloglik_vs_sequential": dev_q,
                  "max_rel_dloglik_vs_oracle_3_smallest": orc_q},
        "queue_tuned_band": {"status": st_b, "seconds": wall_b, "evals_per_s": len(probs) / wall_b,
                             "escalated": int(sum(1 for r in res_b if r["escalations"] > 0)),
                             "tflops_cholesky_equivalent": flops / wall_b / 1e12,
                             "speedup_vs_fp64_queue": wall_q / wall_b, "bands": bands, "tile": 128,
                             "max_rel_dloglik_vs_sequential_fp64": dev_b,
                             "median_rel_dloglik_vs_sequential_fp64": float(np.median(errs_b)),
                             "problems_over_1e-5": int(sum(e > 1e-5 for e in errs_b)),
                             "max_dloglik_over_terms_vs_sequential_fp64": max(terms_b),
                             "max_rel_dloglik_vs_oracle_3_smallest": orc_b}}), flush=True)


def serve_bench(args):
    """Serving loop: Poisson arrivals of likelihood requests for 16 datasets (n log-uniform in
    [2,000, 60,000], z a draw of the Matern field at theta_0 = (1, 0.1, 0.5) by the library's FP64
    sampler), every fourth a kriging request (predictions and variances at 500 new sites), HBM
    budget 96 GB, 4 lanes.  The theta of the requests for a dataset follow, in order, a seeded
    Nelder-Mead trajectory: the library's own maximum-likelihood search (mpgeo_dataset_mle_trace,
    all-FP64, tile 128) on a 30 x 30 field drawn at theta_0 with the dataset's seed, from
    theta_0 * (1.5, 0.5, 1.2).  Datasets of n <= 4,096 are served through the persistent queue
    (tile 128, FP64 within the same distance of the diagonal as the leg's plan, FP32 beyond;
    ready requests batched into one launch), the others on the lanes with the leg's plan at tile
    512: the three-tier plan (FP64 band 2, FP32 next 8 tiles, FP16 operands beyond), the two-tier
    plan (FP64 band 2, FP32 beyond) and the all-FP64 plan, the same trace each time."""
    import numpy as np

    import paper_2003_05324_amd as mp
    from synthetic import jittered_grid, normals, uniform_sites
    rng = np.random.default_rng(21)
    sizes = [int(round(np.exp(rng.uniform(np.log(2000), np.log(60000))))) for _ in range(16)]
    theta0 = (1.0, 0.1, 0.5)
    ctx = mp.Context(0)
    data = []
    for q, n in enumerate(sizes):
        m = int(np.ceil(np.sqrt(n)))
        locs = jittered_grid(m, 700 + q)[:n].copy()
        gen = mp.Dataset(ctx, locs, None)
        z = gen.simulate(theta0, normals(n, 800 + q), 512, -1)
        gen.close()
        data.append((locs, np.asarray(z)))
    # one optimiser trajectory per dataset
    start = (1.5 * theta0[0], 0.5 * theta0[1], 1.2 * theta0[2])
    trajectories = []
    for q in range(len(sizes)):
        tl = jittered_grid(30, 1700 + q)
        gen = mp.Dataset(ctx, tl, None)
        tz = gen.simulate(theta0, normals(len(tl), 1800 + q), 128, -1)
        gen.close()
        tds = mp.Dataset(ctx, tl, tz)
        fit = tds.mle_trace(start, 128, -1, xtol=1e-4, max_evals=400)
        tds.close()
        trajectories.append([th for th, ll in zip(fit["trace"], fit["trace_loglik"]) if np.isfinite(ll)])
    arrivals = np.cumsum(rng.exponential(1.0 / args.serve_rate, args.serve))
    picks = rng.integers(0, len(sizes), args.serve)
    used = [0] * len(sizes)
    thetas = []
    for d in picks:
        tr = trajectories[d]
        thetas.append(tuple(tr[used[d] % len(tr)]))
        used[d] += 1
    if args.serve_theta == "lognormal":
        trng = np.random.default_rng(22)
        thetas = [(float(np.exp(trng.normal(0, 0.15))), float(0.1 * np.exp(trng.normal(0, 0.15))), 0.5)
                  for _ in range(args.serve)]
    flops = float(sum(sizes[d] ** 3 / 3.0 for d in picks))
    kriging = [q % 4 == 3 for q in range(args.serve)]
    new_sites = [uniform_sites(500, 950 + q) for q in range(len(sizes))]
    small = [n <= args.serve_queue_max_n for n in sizes]
    out = {"serve": f"matern-serve{args.serve}-16sets-n2000-60000", "requests": args.serve,
           "rate_per_s": args.serve_rate, "dataset_sizes": sizes, "sum_n3_over_3": flops,
           "queued_datasets": int(sum(small)),
           "queued_requests": int(sum(1 for d, k in zip(picks, kriging) if small[d] and not k)),
           "trajectory_evals": [len(t) for t in trajectories]}
    for name, band, band32, lowp in (("three_tier_b2_c8", 2, 8, "fp16"), ("two_tier_b2", 2, -1, None),
                                     ("fp64", -1, -1, None)):
        srv = mp.Server(ctx, 96 * 2 ** 30, 4)
        qband = -1 if band < 0 else (band + 1) * 512 // 128 - 1   # the same FP64 distance at tile 128
        ids = [srv.add_dataset(locs, z, 128, qband, queue=True) if sm else
               srv.add_dataset(locs, z, 512, band, band32, lowp)
               for (locs, z), sm in zip(data, small)]
        for q in range(args.serve):
            if kriging[q]:
                srv.submit_krige(ids[picks[q]], thetas[q], new_sites[picks[q]], float(arrivals[q]),
                                 variance=True)
            else:
                srv.submit(ids[picks[q]], thetas[q], float(arrivals[q]))
        print(f"[serve] {name}: {args.serve} requests over {arrivals[-1]:.1f} s", file=sys.stderr, flush=True)
        st, res = srv.run()
        srv.close()
        lat = np.array([r["finish_s"] - r["arrival_s"] for r in res])
        klat = np.array([r["finish_s"] - r["arrival_s"] for r, k in zip(res, kriging) if k])
        qlat = np.array([r["finish_s"] - r["arrival_s"] for r, d, k in zip(res, picks, kriging)
                         if small[d] and not k])
        wait = np.array([r["start_s"] - r["arrival_s"] for r in res])
        span = max(r["finish_s"] for r in res)
        failed = int(sum(1 for r in res if r["info"] >= 0))
        out[name] = {"status": st, "status_string": mp.status_string(st), "failed_requests": failed,
                     "p50_latency_s": float(np.percentile(lat, 50)),
                     "p99_latency_s": float(np.percentile(lat, 99)),
                     "kriging_requests": int(sum(kriging)),
                     "kriging_p50_latency_s": float(np.percentile(klat, 50)) if len(klat) else None,
                     "queued_p50_latency_s": float(np.percentile(qlat, 50)) if len(qlat) else None,
                     "mean_wait_s": float(wait.mean()), "makespan_s": span,
                     "evals_per_s": args.serve / span, "tflops": flops / span / 1e12,
                     "loglik_first": res[0]["loglik"]}
        print(f"[serve] {name}: {out[name]}", file=sys.stderr, flush=True)
    ctx.close()
    if all(out[k]["status"] == 0 for k in ("fp64", "two_tier_b2", "three_tier_b2_c8")):
        out["p50_speedup_vs_fp64"] = out["fp64"]["p50_latency_s"] / out["two_tier_b2"]["p50_latency_s"]
        out["p50_speedup_three_tier_vs_fp64"] = out["fp64"]["p50_latency_s"] / out["three_tier_b2_c8"]["p50_latency_s"]
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              f"sharding of the path is a design note, not a build", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve_bench(args)
        return
    if args.sweep:
        band_sweep(args)
        return
    if args.small:
        small_bench(args)
        return
    if args.batch:
        batch_bench(args)
        return
    import torch

    import numpy as np

    import paper_2003_05324_amd as mp
    from synthetic import jittered_grid, normals, uniform_sites

    m = args.m
    n = m * m
    theta = (1.0, 0.1, 0.5)
    locs_h = jittered_grid(m, 301)
    eps_h = normals(n, 302)
    dev = torch.device("cuda:0")
    locs = torch.from_numpy(locs_h).to(dev)
    eps = torch.from_numpy(eps_h).to(dev)
    ctx = mp.Context(0)
    # the field is drawn jointly at the n observed and the held-out kriging sites
    m_h = args.heldout
    sites_h = uniform_sites(m_h, 303) if m_h else np.zeros((0, 2))
    all_locs = torch.from_numpy(np.concatenate([locs_h, sites_h])).to(dev)
    all_eps = torch.from_numpy(np.concatenate([eps_h, normals(m_h, 304)])).to(dev)
    print(f"[bench] n={n} tile={args.tile} band={args.band}: drawing z from the FP64 field "
          f"(+{m_h} held-out sites)", file=sys.stderr, flush=True)
    gen = mp.Dataset(ctx, all_locs, None)
    z_all = gen.simulate(theta, all_eps, args.tile, -1)
    gen.close()
    del gen
    z = z_all[:n].contiguous()
    z_heldout = z_all[n:].cpu().numpy()
    sites = all_locs[n:].contiguous()
    torch.cuda.synchronize()

    lowp = None if args.lowp == "none" else args.lowp
    band32 = args.band32 if lowp else -1

    def workload_of(band64, b32, fmt):
        return (f"matern-n{n}-nb{args.tile}-band{band64}" + (f"-band32_{b32}-{fmt}" if fmt else "")
                if band64 >= 0 else f"matern-n{n}-nb{args.tile}-fp64")

    # the timed headline: the two-tier plan (the paper's method at its own precision); then
    # the legs beside it on the same inputs
    want = set(args.legs.split(","))
    legs = []
    if "two_tier" in want and args.steps > 0:
        legs.append(("two_tier", args.band, -1, None, args.steps, args.warmup, "f64+f32"))
    if "three_tier" in want and lowp and args.three_tier_steps > 0:
        legs.append(("three_tier", args.band, band32, lowp, args.three_tier_steps, 1,
                     "f64+f32+" + lowp.replace("fp", "f")))
    if "three_tier_wide" in want and lowp and args.three_tier_steps > 0 and args.band32_wide > 0:
        legs.append(("three_tier_wide", args.band, args.band32_wide, lowp, args.three_tier_steps, 1,
                     "f64+f32+" + lowp.replace("fp", "f")))
    if "fp64" in want and args.fp64_steps > 0:
        legs.append(("fp64", -1, -1, None, args.fp64_steps, 1, "f64"))
    runs = {}
    for name, b64, b32, fmt, steps, warm, dt in legs:
        print(f"[bench] {name} path (band64 {b64}, band32 {b32}, {fmt})", file=sys.stderr, flush=True)
        wall, res, stats = time_path(mp, ctx, locs, z, theta, args.tile, b64, steps, warm, b32, fmt)
        print(f"[bench] {name}: {wall / steps:.3f} s/step", file=sys.stderr, flush=True)
        runs[name] = (wall, res, steps, stats, workload_of(b64, b32, fmt), dt)
    kriging = None
    if m_h:
        # simple-kriging predictions at the held-out sites from the factor of each plan
        # (resident dataset, outside the timed region)
        print("[bench] kriging at held-out sites", file=sys.stderr, flush=True)
        ds = mp.Dataset(ctx, locs, z)
        kriging = {"sites": m_h}
        for name, b64, b32, fmt in (("two_tier", args.band, -1, None), ("three_tier", args.band, band32, lowp),
                                    ("three_tier_wide", args.band, args.band32_wide, lowp),
                                    ("fp64", -1, -1, None)):
            if name.startswith("three_tier") and (fmt is None or b32 <= 0 or name not in runs):
                continue
            ds.loglik(theta, args.tile, b64, band32=b32, lowp=fmt)
            t0 = time.perf_counter()
            pred = ds.krige(sites).cpu().numpy()
            kriging[name] = {"seconds": time.perf_counter() - t0,
                             "pmse": float(np.mean((pred - z_heldout) ** 2)), "pred": pred}
        ref = kriging["fp64"]["pred"]
        for name in list(kriging):
            if isinstance(kriging[name], dict):
                kriging[name]["max_abs_dpred_vs_fp64"] = float(np.max(np.abs(kriging[name].pop("pred") - ref)))
        ds.close()
    ctx.close()

    ll64 = runs["fp64"][1][-1]["loglik"] if "fp64" in runs else None
    summaries = {name: leg_summary(w, r, st, n, ll64 if name != "fp64" else None, stats, wl, dt)
                 for name, (w, r, st, stats, wl, dt) in runs.items()}
    if "two_tier" not in summaries:   # a profiling run of the other legs: no headline
        print(json.dumps({"legs": summaries, "kriging": kriging}), flush=True)
        return
    head = summaries["two_tier"]
    value = head["evals_per_s"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": head["workload"],
                   "n": n, "grid": f"{m}x{m} jittered", "theta": list(theta), "tile": args.tile,
                   "band64": args.band, "band32": -1, "lowp": None},
        "cholesky_tflops": head["cholesky_tflops"],
        "p50_s": head["p50_s"],
        "p99_s": head["p99_s"],
        "loglik": head["loglik"],
        "roofline": head["roofline"],
        "kernel_streams": head["kernel_streams"],
    }
    if ll64 is not None:
        out["dloglik_rel_vs_fp64"] = head["dloglik_rel_vs_fp64"]
    for name in ("three_tier", "three_tier_wide", "fp64"):
        if name in summaries:
            out[name] = summaries[name]
            out["speedup_" + name + "_vs_two_tier"] = summaries[name]["evals_per_s"] / value
    if "fp64" in summaries:
        out["speedup_vs_fp64"] = value / summaries["fp64"]["evals_per_s"]
    if kriging:
        out["kriging"] = kriging
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_m, n, theta)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
