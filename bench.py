#!/usr/bin/env python3
"""Throughput of the sketched leverage-score path on one MI355X.

One step = slso_leverage (column equilibration, CountSketch, FP64 Householder
QR of the sketch, rank screen, Pi_2 and triangular solve, scores) followed by
slso_order (dec ordering), on the image-like workload: dense FP32 X with
n = 60000, d = 784 (entries in [0, 1], rank 50 + noise, 10 clusters),
CountSketch r = 16384, k = 64. X is resident in HBM before the clock starts.

Prints one JSON line: rows/s over the timed steps, p50/p99 step latency, the
max relative score error and Kendall tau of the last step against the FP64
oracle, the roofline of the dominant kernel (HIP events recorded live around
every launch in the timed region) and the oracle's own CPU throughput.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"hbm": 8.0e12, "fp64": 78.6e12, "fp32": 157.3e12}

N, D, R, K, SEED = 60000, 784, 16384, 64, 2001


def qr_update_flops(m: int, d: int, w: int = 16) -> float:
    """Algorithmic flops of the blocked Householder trailing updates
    (Y^T C and C - Y W: 4 m' w n' per panel)."""
    f = 0.0
    for j0 in range(0, d, w):
        wj = min(w, d - j0)
        f += 4.0 * (m - j0) * wj * (d - j0 - wj)
    return f


def qr_node_flops(m: int, d: int, w: int = 16) -> float:
    """Algorithmic flops of the panel factorisations (unblocked Householder
    on (m - j0) x w panels: 2 m' w^2 - 2/3 w^3)."""
    f = 0.0
    for j0 in range(0, d, w):
        wj = min(w, d - j0)
        f += 2.0 * (m - j0) * wj * wj - (2.0 / 3.0) * wj ** 3
    return f


# profiler name -> (kernel symbol in the PMC summary, source file)
KERNEL_SRC = {
    "cq2_gram": ("gram_block_kernel<false,true>", "k_cholqr.hip"),
    "cq2_solve": ("stripe_solve_kernel<64>", "k_cholqr.hip"),
    "cq_update": ("cq_update_kernel", "k_cqr.hip"),
    "cq_z": ("cq_z_kernel", "k_cqr.hip"),
    "cq_q1": ("cq_q1_kernel", "k_cqr.hip"),
    "cq_gram": ("cq_gram_kernel", "k_cqr.hip"),
    "qr_node": ("qr_node_kernel", "k_qr.hip"),
    "qr_update": ("qr_update_kernel", "k_qr.hip"),
    "score": ("score_mfma_kernel<3,true>", "k_score.hip"),
    "countsketch": ("countsketch_colmax_kernel<float,false>", "k_sketch.hip"),
    "colmax": ("colmax_dense_kernel<float>", "k_sketch.hip"),
}
PMC_SUMMARY = os.path.join(ROOT, "profiles",
                           "pmc_traffic_image_like_n60000_d784.txt")


def measured_traffic(name: str):
    """Calibrated HBM bytes per launch from the committed rocprofv3 PMC
    summary, or None when there is none or the kernel's source has changed
    since the counters were taken."""
    import hashlib
    if name not in KERNEL_SRC or not os.path.exists(PMC_SUMMARY):
        return None
    sym, src = KERNEL_SRC[name]
    path = os.path.join(ROOT, "paper_1812_07903_amd", "csrc", src)
    with open(path, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    with open(PMC_SUMMARY) as f:
        for line in f:
            t = line.split()
            if len(t) == 8 and t[0] == "traffic" and t[1] == sym:
                return float(t[7]) if t[2] == src and t[3] == sha else None
    return None


def roofline_for(name: str, ms_per_launch: float, launches_per_step: float):
    """Algorithmic work per launch of a kernel at this workload."""
    r = _roofline(name, ms_per_launch, launches_per_step)
    if r is not None:
        r["traffic"] = measured_traffic(name)
    return r


def cq_panels(m: int = R, d: int = D):
    """(active rows, trailing columns) of each 64-column Cholesky-QR2 panel."""
    return [(m - j0, d - j0 - 64) for j0 in range(0, d - 63, 64)]


def _fp64(flops_per_launch: float, sec: float):
    a = flops_per_launch / sec
    return {"bound": "mfma", "achieved": a / 1e12, "peak": PEAK["fp64"] / 1e12,
            "unit": "TFLOP/s", "frac": a / PEAK["fp64"], "traffic": None}


def _roofline(name: str, ms_per_launch: float, launches_per_step: float):
    sec = ms_per_launch * 1e-3
    if name == "cq2_gram":
        # the upper triangle of A^T A: d (d + 1) / 2 entries of m products
        # each when the last column block is at most 16 wide (its products
        # are formed by the same launch), else the part inside full
        # 128-column blocks (c = 128 floor(d / 128))
        c = D if D % 128 <= 16 else 128 * (D // 128)
        return _fp64(float(R) * c * (c + 1), sec)
    if name == "cq2_gram_edge":
        # the rest of the upper triangle (columns past c), plus the sum of
        # the partial blocks
        c = 128 * (D // 128)
        return _fp64(float(R) * (D * (D + 1) - c * (c + 1)), sec)
    if name == "cq2_solve":
        # Q1 = A R1^{-1}: m d^2 flop
        return _fp64(float(R) * D * D, sec)
    if name in ("cq2_chol", "cq2_r"):
        # d^3 / 3 flop (Cholesky of G1; R = R2 R1 with triangular R2, R1)
        a = D ** 3 / 3.0 / sec
        return {"bound": "alu", "achieved": a / 1e12,
                "peak": PEAK["fp64"] / 1e12, "unit": "TFLOP/s",
                "frac": a / PEAK["fp64"], "traffic": None}
    if name in ("cq_update", "cq_z"):
        # C -= Q1 K  /  Z = Q1^T C: 2 m' 64 n' flop per panel
        f = sum(2.0 * mp * 64 * nc for mp, nc in cq_panels() if nc > 0)
        return _fp64(f / launches_per_step, sec)
    if name == "cq_q1":
        # Q1 = P R1^{-1} and G2 = Q1^T Q1: 2 x 2 m' 64^2 flop per panel
        return _fp64(sum(4.0 * mp * 64 * 64 for mp, _ in cq_panels())
                     / launches_per_step, sec)
    if name == "cq_gram":
        return _fp64(sum(2.0 * mp * 64 * 64 for mp, _ in cq_panels())
                     / launches_per_step, sec)
    if name in ("cq_recon", "cq_chol"):
        # one workgroup per panel: Cholesky (64^3 / 3), triangular inverses,
        # the sign-choosing LU (2 64^3 / 3) and several 64^3 products
        f = {"cq_chol": 64 ** 3, "cq_recon": 14 * 64 ** 3}[name]
        a = f / sec
        return {"bound": "alu", "achieved": a / 1e12,
                "peak": PEAK["fp64"] / 1e12, "unit": "TFLOP/s",
                "frac": a / PEAK["fp64"], "traffic": None}
    if name == "qr_update":
        flops = qr_update_flops(R, D) / launches_per_step
        a = flops / sec
        return {"bound": "alu", "achieved": a / 1e12, "peak": PEAK["fp64"] / 1e12,
                "unit": "TFLOP/s", "frac": a / PEAK["fp64"], "traffic": None}
    if name == "qr_node":
        flops = qr_node_flops(R, D) / launches_per_step
        a = flops / sec
        return {"bound": "alu", "achieved": a / 1e12, "peak": PEAK["fp64"] / 1e12,
                "unit": "TFLOP/s", "frac": a / PEAK["fp64"], "traffic": None}
    if name == "score":
        # X M as six split-BF16 products: 12 n d k flop on the BF16 MFMA take
        # less time at its peak than reading X once, so the pass is priced
        # against HBM: X once (4 n d), M's three BF16 parts (6 d k) and the
        # scores (4 n)
        byts = (N * D * 4 + 6 * D * K + N * 4) / launches_per_step
        a = byts / sec
        return {"bound": "hbm", "achieved": a / 1e9, "peak": PEAK["hbm"] / 1e9,
                "unit": "GB/s", "frac": a / PEAK["hbm"], "traffic": None}
    if name == "countsketch":
        # X once, the sketch written once, the sorted row list once, the
        # per-workgroup column maxima (min(1024, R / 4) x D floats) once
        byts = (N * D * 4 + R * D * 8 + N * 4 + min(1024, R // 4) * D * 4) \
            / launches_per_step
        a = byts / sec
        return {"bound": "hbm", "achieved": a / 1e9, "peak": PEAK["hbm"] / 1e9,
                "unit": "GB/s", "frac": a / PEAK["hbm"], "traffic": None}
    if name == "colmax":
        byts = N * D * 4 / launches_per_step
        a = byts / sec
        return {"bound": "hbm", "achieved": a / 1e9, "peak": PEAK["hbm"] / 1e9,
                "unit": "GB/s", "frac": a / PEAK["hbm"], "traffic": None}
    return None


def copy_calibration(mib: int) -> int:
    """A plain elementwise copy y = 1.0 * x of known size, five launches."""
    import torch
    n = mib * (1 << 20) // 4
    x = torch.rand(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(5):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 4,
                      "copy_calibration_bytes_written": n * 4,
                      "launches": 5}), flush=True)
    return 0


def serving_bench(args) -> int:
    """Continuous serving: jobs arrive as a Poisson stream and are admitted
    by the library's server (slots under an HBM budget); reports aggregate
    rows/s and p50/p99 latency from arrival to resident outputs per rate."""
    import numpy as np
    import torch

    import synth
    import paper_1812_07903_amd as slso

    rates = [float(v) for v in args.rates.split(",") if v]
    t_gen = time.perf_counter()
    pool = synth.serving_pool(n=args.pool_n)
    torch.cuda.synchronize()
    print(f"[serving] pool of {len(pool)} base matrices ready in "
          f"{time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    per_rate = {}
    checked = None
    for rate in rates:
        jobs = synth.serving_jobs(args.jobs, rate, pool_n=args.pool_n)
        srv = slso.Server(0, slots=args.slots, hbm_budget=96 << 30)
        tickets = []
        t0 = time.perf_counter()
        for jb in jobs:
            delay = t0 + jb["arrival_s"] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            x = pool[(jb["d"], jb["dtype"])][jb["row0"]:jb["row0"] + jb["n"]]
            tickets.append(srv.submit(x, jb["seed"], jb["r"], jb["k"]))
        res = [srv.wait(t) for t in tickets]
        stats = srv.stats()
        srv.close()
        bad = [r for r in res if r["status"] < 0]
        lat = np.array([r["latency_ms"] for r in res])
        span_ms = max(r["end_ms"] for r in res) - min(r["submit_ms"] for r in res)
        rows = sum(jb["n"] for jb in jobs)
        per_rate[str(int(rate))] = {
            "rows_per_s": rows / (span_ms * 1e-3), "jobs": len(jobs),
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "max_running": stats["max_running"], "failed": len(bad)}
        print(f"[serving] rate {rate:g}/s: {per_rate[str(int(rate))]}",
              file=sys.stderr, flush=True)
        if checked is None and not args.no_cpu_baseline:
            # accuracy of the three smallest jobs against the FP64 oracle
            from oracle import leverage as olv
            from oracle import metrics as omet
            errs, taus = [], []
            for i in sorted(range(len(jobs)), key=lambda i: jobs[i]["n"])[:3]:
                jb, t = jobs[i], tickets[i]
                xv = t.x.double().cpu().numpy()
                ref = olv.sketched_leverage(xv, jb["seed"], jb["r"], jb["k"])
                got = t.scores.cpu().numpy()
                errs.append(omet.max_rel_err(got, ref["scores"]))
                taus.append(omet.kendall_tau(got, ref["scores"]))
            checked = (max(errs), min(taus))
        del tickets, res
    top = per_rate[str(int(rates[-1]))]
    out = {
        "metric": "rows/sec leverage-scored at stated rel err vs FP64; "
                  "p50/p99 job latency",
        "value": top["rows_per_s"], "unit": "rows/s", "n_gpus": 1,
        "steps": args.jobs, "warmup": 0,
        "ms_per_step": None,
        "p50_ms": top["p50_ms"], "p99_ms": top["p99_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32+bf16", "data": "synthetic",
        "config": {"workload": "serving: Poisson stream of leverage jobs, n "
                               "log-uniform [1e4, 2e6], d in {64..1024}, "
                               "FP32/BF16, CountSketch r=4d..8d, k=32, "
                               "scores + dec ordering",
                   "jobs_per_rate": args.jobs, "slots": args.slots,
                   "pool_rows": args.pool_n},
        "per_rate": per_rate,
    }
    if checked is not None:
        out["rel_err_vs_fp64"], out["kendall_tau_vs_fp64"] = checked
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=("image", "serving"),
                    default="image",
                    help="image: the image-like single-job workload (default); "
                         "serving: a Poisson stream of mixed jobs")
    ap.add_argument("--sketch", choices=("countsketch", "osnap", "srht"),
                    default="countsketch",
                    help="image: the sketch (OSNAP: --nnz nonzeros per column "
                         "of S)")
    ap.add_argument("--nnz", type=int, default=2,
                    help="image, --sketch osnap: nonzeros per column of S")
    ap.add_argument("--rates", default="50,200,800",
                    help="serving: arrival rates in jobs/s")
    ap.add_argument("--jobs", type=int, default=1024,
                    help="serving: jobs per rate")
    ap.add_argument("--slots", type=int, default=4,
                    help="serving: concurrent jobs (server slots)")
    ap.add_argument("--pool-n", type=int, default=2_000_000,
                    help="serving: rows of each base matrix")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times "
                         "(reads MIB, writes MIB per launch): the reference "
                         "kernel for scaling HBM byte counters")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.workload == "serving":
        if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
            print("bench.py measures one GPU only; run with --gpus 1",
                  file=sys.stderr)
            return 2
        return serving_bench(args)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the leverage path runs on a "
              "single MI355X (rows would shard across GPUs with one reduction "
              "of the sketch); run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    import paper_1812_07903_amd as slso

    x_host = synth.config1(N, D)
    x = torch.from_numpy(x_host).cuda()
    ctx = slso.Context(0)
    scores = torch.empty(N, dtype=torch.float32, device="cuda")
    perm = torch.empty(N, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    osnap = args.sketch == "osnap"
    kind = {"countsketch": slso.COUNTSKETCH, "osnap": slso.OSNAP,
            "srht": slso.SRHT}[args.sketch]
    nnz = args.nnz if osnap else 0

    def step():
        _, info = ctx.leverage(x, SEED, R, K, out=scores, stream=stream,
                               sketch=kind, nnz=nnz)
        ctx.order(scores, out=perm, stream=stream)
        return info

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # per-kernel breakdown: a short pass with every launch bracketed by events
    # (outside the timed region, since the events themselves cost time)
    slso.profile_read()
    slso.profile_only(None)
    slso.profile_enable(True)
    nb = max(2, min(5, args.steps))
    for _ in range(nb):
        step()
    prof = slso.profile_read()
    kernels = {k: {"ms_per_step": v[0] / nb, "launches_per_step": v[1] / nb}
               for k, v in prof.items() if v[1] > 0}
    dname = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    # timed region: events around the dominant kernel's launches only
    slso.profile_only(dname)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        info = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    dprof = slso.profile_read()
    slso.profile_enable(False)
    slso.profile_only(None)

    ms_step = 1e3 * total / args.steps
    rows_per_s = N * args.steps / total
    lat_ms = np.array(lat) * 1e3

    dms, dcount = dprof[dname]
    roof = roofline_for(dname, dms / max(dcount, 1), dcount / args.steps)

    got = scores.cpu().numpy().astype(np.float64)
    perm_h = perm.cpu().numpy().astype(np.int64)
    perm_ok = bool(np.array_equal(perm_h, np.argsort(-got.astype(np.float32),
                                                      kind="stable")))

    out = {
        "metric": "rows/sec leverage-scored at stated rel err vs FP64; "
                  "p50/p99 job latency",
        "value": rows_per_s,
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "image-like dense FP32 X (n=60000, d=784, "
                               "values in [0,1], rank 50 + noise, 10 clusters); "
                               + {"countsketch": "CountSketch ",
                                  "osnap": f"OSNAP (s={nnz}) ",
                                  "srht": "SRHT "}[args.sketch]
                               + "r=16384, FP64 QR, k=64, scores + dec ordering",
                   "n": N, "d": D, "r": R, "k": K, "seed": SEED,
                   "rank": int(info["rank"])},
        "perm_matches_stable_sort": perm_ok,
        "kernels": kernels,
        "roofline": dict(kernel=dname, **roof) if roof else None,
        "roofline_other": {
            k: dict(kernel=k, **rr)
            for k in ("cq2_solve", "cq2_chol", "countsketch", "score", "colmax",
                      "cq_update", "cq_z")
            if k in kernels and k != dname
            for rr in [roofline_for(
                k, kernels[k]["ms_per_step"] / kernels[k]["launches_per_step"],
                kernels[k]["launches_per_step"])] if rr},
    }

    if not args.no_cpu_baseline:
        # the oracle, untouched, on whole jobs of the same workload until
        # about 10 s of CPU work has been timed (a bounded sample)
        from oracle import leverage as olv
        from oracle import metrics as omet
        from oracle import order as oorder
        try:
            from threadpoolctl import threadpool_info
            cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
        except Exception:
            cores = os.cpu_count() or 1
        reps, t_cpu, ref = 0, 0.0, None
        while reps < 40 and t_cpu < 10.0:
            tc = time.perf_counter()
            ref = olv.sketched_leverage(x_host, SEED, R, K, kind=args.sketch,
                                        nnz=max(nnz, 1))
            oorder.dec_order(ref["scores"].astype(np.float32))
            t_cpu += time.perf_counter() - tc
            reps += 1
        out["cpu_baseline"] = {
            "value": N * reps / t_cpu, "unit": "rows/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"{reps} full job(s) of the same workload (n={N}): "
                      "oracle sketched leverage (numpy FP64) + dec ordering"}
        out["rel_err_vs_fp64"] = omet.max_rel_err(got, ref["scores"])
        out["kendall_tau_vs_fp64"] = omet.kendall_tau(got, ref["scores"])
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
