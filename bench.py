#!/usr/bin/env python
"""Benchmark of the two-stage k-means hot path on one MI355X.

A step is one complete two-stage fit -- fast-stage sampling, the fast stage on
the subset, the slow stage on all points, the final labelling pass -- of a
Gaussian-mixture workload (default: the largest single-GPU one,
100,000,000 x 128-D BF16, k = 1024), with X resident in HBM before the timed
region.  ``value`` is distance evaluations per second of the whole job:
k*(m*Q_f + n*Q_s) + k*n evaluations per fit (section 3 of the paper counts the
method's cost in these units) over the fit's wall time.

The roofline object covers the dominant kernel, the slow stage's assignment
kernel (for BF16 data with d >= 32, its BF16 MFMA screen; for d <= 16 and
k <= 128, the fused pass on the split BF16 screen): its duration is measured
live with HIP events on the stream it runs on (the library's pass profiler).
Its algorithmic work per launch is 2*n*k*d flops and n*d*s bytes (s = bytes
per element of X).  It is priced against the unit its products run on:
T_roof = max(bytes / HBM peak, flops / peak of that unit) -- dense BF16 MFMA
for the BF16 screens (the split screen included), FP32 MFMA for the FP32 MFMA
pass, FP32 vector otherwise -- and frac = T_roof / measured duration.  The
VALU issue load of the kernel, from the committed counter summary, is a field
of its own.  Measured peaks (a streaming read, a BF16 MFMA loop) are reported
beside the datasheet ones.  The CPU baseline is the FP64 oracle timed on a
bounded sample of the same workload on the host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "gmm128d_n1e8_k1024_bf16"
PEAK_FP32_TFLOPS = 157.3        # MI355X published FP32 vector/matrix peak
PEAK_BF16_TFLOPS = 2500.0       # MI355X published dense BF16 MFMA peak
PEAK_HBM_GBS = 8000.0           # MI355X HBM3E
# VALU issue: one wave64 instruction per SIMD per 4 cycles, 1024 SIMDs at 2.4 GHz
VALU_ISSUE_PER_S = 1024 * 2.4e9 / 4
# rows of the CPU-baseline sample per workload (about 10-30 s of oracle work)
CPU_ROWS = {"gmm2d_n1e5_k8": 100_000, "gmm16d_n1e7_k64": 2_000_000,
            "gmm128d_n1e8_k1024_bf16": 80_000, "gmm4d_n5e8_k32": 20_000_000}
METRIC = "distance evals/s & % roofline per Lloyd iter; batched p50/p99 solve latency"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "km_internal.h"):
        with open(os.path.join(ROOT, "paper_1108_1351_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profile_kv(name: str):
    """key value lines of a committed counter summary, or None when it is absent
    or the kernel source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        parts = line.strip().split(None, 1)
        if len(parts) == 2 and not line.startswith("#"):
            kv[parts[0]] = parts[1]
    if kv.get("kernel_src_sha256") != kernel_source_hash():
        return None
    return kv


def read_traffic(workload: str):
    """HBM bytes per launch of the dominant kernel (FETCH_SIZE + WRITE_SIZE,
    scaled by a plain copy's readings), or None."""
    kv = _profile_kv(f"traffic_assign_{workload}.txt")
    try:
        return float(kv["hbm_bytes_per_launch"]) if kv else None
    except (KeyError, ValueError):
        return None


def read_valu(workload: str):
    """SQ_INSTS_VALU per launch of the dominant kernel, or None."""
    kv = _profile_kv(f"valu_assign_{workload}.txt")
    try:
        return float(kv["valu_insts_per_launch"]) if kv else None
    except (KeyError, ValueError):
        return None


def plan_unit(dtype: str, d: int, k: int, precision: str):
    """The pass the library plans for the slow stage, and the unit its products
    run on: (kernel description, unit name, unit peak TFLOP/s, dtype label)."""
    screen = precision == "bf16_rerank" or (precision == "auto" and dtype == "bf16" and d >= 32)
    small = d <= 16 and k <= 128
    if small and precision in ("auto", "bf16_rerank"):
        if precision == "auto":
            return ("slow-stage fused pass on the split BF16 screen (c'hi x^ + c'lo x^ + c'hi xlo "
                    "on BF16 MFMA, FP32 accumulate, certified top-3 keys, FP64 decisions, J and "
                    "exact cluster sums)", "bf16 mfma", PEAK_BF16_TFLOPS, "bf16x3-split")
        return ("slow-stage fused pass on the BF16 screen", "bf16 mfma", PEAK_BF16_TFLOPS, "bf16")
    if screen and d <= 256:
        return ("slow-stage BF16 MFMA screen (slot-pair top-2 keys, certified candidates, "
                "FP64 re-rank)", "bf16 mfma", PEAK_BF16_TFLOPS, "bf16")
    if d <= 32 and k <= 128:
        return ("slow-stage fused pass on FP32 MFMA (assign + cluster sums)", "fp32 mfma",
                PEAK_FP32_TFLOPS, "f32")
    return ("slow-stage FP32 assignment kernel", "fp32 valu", PEAK_FP32_TFLOPS, "f32")


def measured_peaks():
    """A streaming read of 2 GiB and a BF16 MFMA loop, timed on this GPU."""
    import torch

    import paper_1108_1351_amd as km
    buf = torch.empty(1 << 31, dtype=torch.uint8, device="cuda")
    hbm = km.km_probe_stream_read(buf, reps=10)
    del buf
    return {"hbm_read_GBs": hbm, "bf16_mfma_TFLOPs": km.km_probe_mfma_bf16(20000)}


def cpu_baseline(w, rows: int):
    import oracle
    Xs = w.data(n=rows)
    t0 = time.perf_counter()
    f = oracle.fit(Xs, w.k, w.subset_frac, w.fit_seed, w.max_iter, w.tol)
    dt = time.perf_counter() - t0
    return {"value": f.info["dist_evals"] / dt, "unit": "distance evals/s",
            "cores": oracle.get_threads(), "kind": "oracle",
            "sample": (f"full two-stage fit of the first {rows:,} rows of {w.name} "
                       f"(same k, subset fraction, seed, max_iter, tol): "
                       f"{f.info['dist_evals']:.3e} evals in {dt:.2f} s, "
                       f"passes {f.info['iters']}")}


SERVE_POOL = 500  # distinct requests generated before the clock starts


def serve_stream(count: int, rate: float, budget: int, pool: int = SERVE_POOL) -> dict:
    """The serving workload: `count` requests submitted to one server, with
    Poisson arrivals at `rate` per second (rate 0: all at once, the closed-loop
    capacity).  The requests follow the serving stream's distribution (mixed n,
    d, k; data from each request's seed); the first `pool` of them are generated
    on the host before the clock starts and request i reuses request i % pool's
    shape and data with its own fit seed, so that the host generator does not
    bound the arrival rate.  Latency = admission wait + run, from the server's
    own clock."""
    import threading
    import numpy as np
    import torch

    import paper_1108_1351_amd as km
    import synth

    reqs = synth.serving_stream(min(count, pool), 1.0)
    tensors = []
    for r in reqs:
        w = r.workload
        Xh = w.data()
        X = torch.from_numpy(Xh.view(np.int16) if w.dtype == "bf16" else Xh)
        tensors.append((X.view(torch.bfloat16) if w.dtype == "bf16" else X, w))
    print(f"[serve] {len(tensors)} distinct requests generated", file=sys.stderr, flush=True)
    rng = np.random.default_rng(5)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=count)) if rate > 0 else \
        np.zeros(count)
    tickets = [None] * count
    lat, evals, errs = [], 0, 0
    with km.Server(hbm_budget_bytes=budget) as srv:
        # warm the autotuner for every (dtype, d, k bucket) the stream can use
        for d in (2, 8, 32, 128):
            for kb in (8, 16, 32, 64, 128, 256):
                km.km_tune_query(torch.float32 if d < 32 else torch.bfloat16, d, kb)
        t0 = time.perf_counter()

        def produce():
            for i in range(count):
                X, w = tensors[i % len(tensors)]
                now = time.perf_counter() - t0
                if arrivals[i] > now:
                    time.sleep(arrivals[i] - now)
                tickets[i] = srv.submit(X, w.k, w.subset_frac, i, w.max_iter, w.tol,
                                        labels=False)
                if i % 1000 == 0:
                    print(f"[serve] submitted {i + 1}/{count}", file=sys.stderr, flush=True)

        th = threading.Thread(target=produce)
        th.start()
        for i in range(count):
            while tickets[i] is None:
                time.sleep(0.0002)
            try:
                _, _, info = srv.wait(tickets[i])
                lat.append(info["queue_seconds"] + info["run_seconds"])
                evals += info["dist_evals"]
            except km.KMeansError:
                errs += 1
            if i % 1000 == 0:
                print(f"[serve] completed {i + 1}/{count}", file=sys.stderr, flush=True)
        th.join()
        t1 = time.perf_counter()
        st = srv.stats()
    lat = np.array(lat)
    return {"requests": count, "distinct": len(tensors), "rate_per_s": rate, "failed": errs,
            "offered_per_s": count / max(1e-9, float(arrivals[-1])) if rate > 0 else None,
            "completed_per_s": count / (t1 - t0),
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "wall_s": t1 - t0,
            "evals_per_s": evals / (t1 - t0), "rounds": st["rounds"],
            "peak_active": st["peak_active"], "peak_bytes": st["peak_bytes"]}


SPEEDUP_TOLS = [10.0 ** -e for e in range(1, 11)]
SPEEDUP_FRACS = [0.10, 0.15, 0.20, 0.30, 0.40]
SPEEDUP_SIZES = [1_000_000, 2_000_000, 5_000_000, 10_000_000]


def speedup_specs():
    """The sweep's data: (grid name, mixture spec, k, data seed)."""
    import synth
    spec10 = synth.MixtureSpec(10, 10, "uniform", -10.0, 10.0, sigma_lo=0.5, sigma_hi=2.0)
    spec12 = synth.MixtureSpec(12, 12, "uniform", -10.0, 10.0, sigma_lo=0.5, sigma_hi=2.0)
    return {"table2": ("table2_10d", spec10, 10, 1010), "sec61": ("sec61_12d", spec12, 12, 1012)}


SPEEDUP_FIT_SEED = 7


def speedup_sweep(reps: int = 3, max_iter: int = 1000, table2_n: int = 100_000,
                  fracs=None, tols=None, sizes=None, sec61_frac: float = 0.01,
                  sec61_tol: float = 1e-4) -> list:
    """The two-stage method against normal k-means (the slow stage alone, from the
    same initial centers) on the same kernels (section 6 and its Table 2;
    section 6.1).  Stand-ins for the paper's data (not available): a 10-D
    mixture of 100,000 points (10 equally weighted components, means
    U[-10,10]^10, sigma_c U[0.5,2], k = 10) swept over the subset fraction and
    the stopping tolerance (the same tolerance in both stages and in normal
    k-means); and 12-D mixtures of 1e6..1e7 points (12 components, the same
    distribution in 12-D, k = 12, 1% subset, tolerance 1e-4).  Each cell runs
    both fits `reps` times and keeps the median wall time; the evals ratio is
    the machine-independent form of the speed-up (section 3's cost model)."""
    import numpy as np
    import torch

    import paper_1108_1351_amd as km
    import synth

    def load(spec, n, seed):
        Xh = synth.generate(spec, seed, n, "f32")
        return torch.from_numpy(Xh).to("cuda")

    def fit(X, k, f, tol, normal):
        ts, info = [], None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, info = km.kmeans_fit_ex(X, k, f, SPEEDUP_FIT_SEED, max_iter, tol,
                                          skip_stage1=normal,
                                          labels=True)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), info

    def cell(name, X, k, f, tol):
        t2, i2 = fit(X, k, f, tol, False)
        t1, i1 = fit(X, k, f, tol, True)
        row = {"grid": name, "n": int(X.shape[0]), "d": int(X.shape[1]), "k": k,
               "subset_frac": f, "tol": tol, "max_iter": max_iter,
               "two_stage": {"s": t2, "passes": i2["iters"], "evals": i2["dist_evals"],
                             "J": i2["J"]},
               "normal": {"s": t1, "passes": i1["iters"][1], "evals": i1["dist_evals"],
                          "J": i1["J"]},
               "speedup_time": t1 / t2, "speedup_evals": i1["dist_evals"] / i2["dist_evals"]}
        print(f"[speedup] {name} n={row['n']} f={f:g} tol={tol:g}: time x{row['speedup_time']:.2f}"
              f" evals x{row['speedup_evals']:.2f}", file=sys.stderr, flush=True)
        return row

    rows = []
    specs = speedup_specs()
    name, spec, k, seed = specs["table2"]
    X = load(spec, table2_n, seed)
    for f in fracs or SPEEDUP_FRACS:
        for tol in tols or SPEEDUP_TOLS:
            rows.append(cell(name, X, k, f, tol))
    del X
    name, spec, k, seed = specs["sec61"]
    for n in sizes or SPEEDUP_SIZES:
        X = load(spec, n, seed)
        rows.append(cell(name, X, k, sec61_frac, sec61_tol))
        del X
    return rows


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--precision", default="auto", choices=["auto", "fp32", "bf16_rerank"],
                    help="the library's precision choice (fp32: the plain FP32 path)")
    ap.add_argument("--no-peaks", action="store_true", help="skip the measured-peak probes")
    ap.add_argument("--cpu-rows", type=int, default=0,
                    help="rows of the CPU-baseline sample (default: per workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (HBM counter scale)")
    ap.add_argument("--serve", type=int, default=0, metavar="REQUESTS",
                    help="run the serving stream of REQUESTS requests instead of the fit bench")
    ap.add_argument("--serve-rate", type=float, default=100.0,
                    help="arrivals per second (0: all at once, the closed-loop capacity)")
    ap.add_argument("--serve-protocol", action="store_true",
                    help="closed-loop capacity C, then Poisson arrivals at 0.5 C and 0.9 C")
    ap.add_argument("--serve-budget", type=int, default=0, help="server HBM budget (bytes)")
    ap.add_argument("--speedup", action="store_true",
                    help="run the two-stage vs normal k-means sweep instead of the fit bench")
    args = ap.parse_args()
    if args.speedup:
        if args.gpus != 1:
            print("bench.py measures one GPU", file=sys.stderr)
            return 2
        for row in speedup_sweep():
            print(json.dumps(row), flush=True)
        return 0
    if args.serve:
        if args.gpus != 1:
            print("bench.py measures one GPU", file=sys.stderr)
            return 2
        rates = [args.serve_rate]
        if args.serve_protocol:
            cap = serve_stream(args.serve, 0.0, args.serve_budget)
            c = cap["completed_per_s"]
            print(json.dumps({"serving_capacity": cap}), flush=True)
            rates = [0.5 * c, 0.9 * c]
        for rate in rates:
            r = serve_stream(args.serve, rate, args.serve_budget)
            out = {"metric": METRIC, "value": r["evals_per_s"], "unit": "distance evals/s",
                   "n_gpus": 1, "higher_is_better": True, "scaling": "weak",
                   "vs_baseline": None, "dtype": "f32+bf16", "data": "synthetic",
                   "config": {"workload": f"serving_stream_{args.serve}req_{rate:g}per_s"},
                   "latency": {"p50_s": r["p50_s"], "p99_s": r["p99_s"], "mean_s": r["mean_s"]},
                   "serving": r}
            print(json.dumps(out), flush=True)
        return 0
    if args.copy_calibration:
        import torch
        a = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4}))
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is described, not built)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1108_1351_amd as km
    import synth

    w = synth.WORKLOADS[args.workload]
    print(f"[bench] generating {w.name}: n={w.n} d={w.d} k={w.k} {w.dtype}", file=sys.stderr,
          flush=True)
    host = torch.empty((w.n, w.d), dtype=torch.float32 if w.dtype == "f32" else torch.int16,
                       pin_memory=True)
    hv = host.numpy() if w.dtype == "f32" else host.numpy().view(np.uint16)
    chunk = 10_000_000
    prm = synth.params(w.spec, w.data_seed)
    for r0 in range(0, w.n, chunk):
        r1 = min(w.n, r0 + chunk)
        synth.generate(w.spec, w.data_seed, r1 - r0, w.dtype, row0=r0, out=hv[r0:r1], prm=prm)
        if w.n > chunk:
            print(f"[bench] generated rows {r0:,}..{r1:,}", file=sys.stderr, flush=True)
    X = host.to("cuda", non_blocking=False)
    if w.dtype == "bf16":
        X = X.view(torch.bfloat16)
    del host
    torch.cuda.synchronize()

    def step():
        return km.kmeans_fit_ex(X, w.k, w.subset_frac, w.fit_seed, w.max_iter, w.tol,
                                labels=True, precision=args.precision)

    for i in range(args.warmup):
        step()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    evals = 0
    infos = []
    km.kmeans_profile_begin()
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, _, info = step()
        evals += info["dist_evals"]
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = km.kmeans_profile_end()
    print(f"[bench] timed {args.steps} steps in {t1 - t0:.3f} s", file=sys.stderr, flush=True)
    dt = t1 - t0
    value = evals / dt
    info = infos[-1]

    # dominant kernel: the slow stage's assignment kernel (one launch per pass)
    launches = prof["passes"][1]
    avg_s = prof["assign_ms"][1] / 1e3 / max(1, launches)
    rows = prof["rows"][1] / max(1, launches)
    flops = 2.0 * rows * w.k * w.d
    algo_bytes = rows * w.d * (4 if w.dtype == "f32" else 2)
    kernel, unit, peak_flops, dtype_label = plan_unit(w.dtype, w.d, w.k, args.precision)
    traffic = read_traffic(w.name) if args.precision == "auto" else None
    # T_roof = max(bytes / HBM peak, flops / peak of the unit the products run on)
    t_hbm = algo_bytes / (PEAK_HBM_GBS * 1e9)
    t_unit = flops / (peak_flops * 1e12)
    if t_hbm >= t_unit:
        achieved = algo_bytes / avg_s / 1e9
        roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    else:
        achieved = flops / avg_s / 1e12
        roofline = {"bound": "mfma" if "mfma" in unit else "alu",
                    "achieved": achieved, "peak": peak_flops, "unit": "TFLOP/s"}
    valu = read_valu(w.name) if args.precision == "auto" else None
    roofline.update({
        "frac": roofline["achieved"] / roofline["peak"], "traffic": traffic,
        "kernel": kernel, "products_on": unit,
        "T_roof_us": max(t_hbm, t_unit) * 1e6,
        "launches": launches, "avg_launch_us": avg_s * 1e6,
        "flops_per_launch": flops, "algo_bytes_per_launch": algo_bytes,
        "achieved_TFLOPs": flops / avg_s / 1e12, "algo_hbm_GBs": algo_bytes / avg_s / 1e9,
        # VALU instructions per launch (counters) over what the SIMDs can issue
        # in the measured duration: the issue load, not a roofline
        "valu_issue_util": (valu / (avg_s * VALU_ISSUE_PER_S)) if valu else None})
    if not args.no_peaks:
        mp = measured_peaks()
        roofline["measured_peaks"] = mp
        roofline["frac_of_measured"] = (
            roofline["achieved"] / (mp["hbm_read_GBs"] if roofline["bound"] == "hbm"
                                    else mp["bf16_mfma_TFLOPs"])
            if roofline["bound"] != "alu" else None)
    pass_s = prof["pass_ms"][1] / 1e3 / max(1, launches)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "distance evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # products in BF16 (the split screen: high and low BF16 parts), FP32
        # accumulation; FP64 decisions near ties; "f32" for the FP32 kernels
        "dtype": dtype_label,
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "k": w.k,
                   "precision": args.precision,
                   "subset_frac": w.subset_frac, "max_iter": w.max_iter, "tol": w.tol,
                   "passes": info["iters"], "m": info["m"],
                   "dist_evals_per_fit": info["dist_evals"],
                   "fp64_full_checks_per_fit": info["uncertain"],
                   "fp64_pair_decisions_per_fit": info["fp64_pairs"]},
        "per_pass": {"slow_stage_pass_us": pass_s * 1e6,
                     "slow_stage_evals_per_s": rows * w.k / pass_s,
                     "assign_evals_per_s": rows * w.k / avg_s},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        cpu_rows = min(w.n, args.cpu_rows or CPU_ROWS.get(w.name, 1_000_000))
        print(f"[bench] cpu baseline on {cpu_rows} rows", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, cpu_rows)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
