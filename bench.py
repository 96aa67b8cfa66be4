#!/usr/bin/env python3
"""Throughput of the sketched leverage-score path on one MI355X.

One step = slso_leverage (sketch, QR of the sketch, rank screen, refinement
where asked, Pi_2 and the triangular factor, scores) followed by slso_order
(dec ordering) on one synthetic job whose input is resident in HBM before
the clock starts.

Workloads (``--workload``):
* ``precision`` (default): dense X with n = 4e6, d = 512 (rank 256 with
  sigma_j = j^-1.5, noise 1e-4, row scales e^N(0, 1.5^2)); Gaussian sketch
  r = 2048, Cholesky-QR refinement, k = 64. The headline runs BF16 input; the
  FP8-e4m3 input (per-column scales) and the plain FP32 path (FP32 input,
  FP32 MFMA sketch, no refinement) are timed beside it. The text-like CSR
  and serving workloads follow as extra keys unless ``--headline-only``.
* ``image``: dense FP32 image-like X (n = 60000, d = 784), CountSketch
  r = 16384, k = 64.
* ``text``: CSR X (n = 5e5, d = 4096, 0.5 % dense, tf-idf-like), CountSketch
  on CSR r = 32768, k = 64.
* ``serving``: a Poisson stream of mixed jobs through the library's server.

Prints one JSON line: rows/s over the timed steps, p50/p99 step latency, the
max relative score error and Kendall tau against the FP64 oracle on a
bounded sample job of the same workload, the roofline of the dominant kernel
(HIP events recorded live around its launches in the timed region) and the
oracle's own CPU throughput.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from dataclasses import dataclass

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"hbm": 8.0e12, "fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15,
        "fp8": 5.0e15}
METRIC = ("rows/sec leverage-scored at stated rel err vs FP64; "
          "p50/p99 job latency")


@dataclass
class Shape:
    """A job's sizes, as the roofline formulas need them."""
    n: int
    d: int
    r: int
    k: int
    xbytes: int          # bytes per stored element of X (CSR: per nonzero)
    dtype: str           # "f32", "bf16", "fp8", "f64", "csr"
    nnz: int = 0
    qr_passes: int = 2   # Cholesky-QR passes of the sketch (1: one pass)


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---- rooflines ----------------------------------------------------------------
# per workload: the committed PMC summary and, per profiler name, the kernel
# symbol in it (the BF16 / FP32 form that the bench line's roofline times;
# for the scoring the two-buffer ring: every ring reads the same bytes)
PMC_SUMMARIES = {
    "image": ("pmc_traffic_image_like_n60000_d784.txt", {
        "cq2_gram": "gram_block_kernel<false,true>",
        "cq2_solve": "q1_gemm_kernel",
        "score": "score_mfma_kernel<3,true>",
        "countsketch": "countsketch_colmax_kernel<float,false,4,4>"}),
    "precision_bf16": ("pmc_traffic_precision_n4000000_d512.txt", {
        "gauss_sketch": "gauss_q_kernel<1,true>",
        "gram": "gram_q_kernel<1,true>",
        "score": "score_q_kernel<1,2,512,2>"}),
    "precision_fp8": ("pmc_traffic_precision_n4000000_d512.txt", {
        "gauss_sketch": "gauss_q_kernel<2,true>",
        "gram": "gram_q_kernel<2,true>",
        "score": "score_q_kernel<2,2,512,2>"}),
    "precision_f32": ("pmc_traffic_precision_n4000000_d512.txt", {
        "gauss_sketch": "gauss_sketch_kernel",
        "score": "score_mfma_kernel<3,true>"}),
    "text": ("pmc_traffic_text_like_n500000_d4096.txt", {
        "countsketch": "countsketch_csr_kernel",
        "cq2_gram": "gram_sk_kernel",
        "cq2_solve": "stripe_solve_kernel<64>",
        "score": "score_csr_kernel"}),
}


def measured_traffic(name: str, workload: str):
    """Calibrated HBM bytes per launch from the workload's committed
    rocprofv3 PMC summary, or None when there is none, when the kernel is
    not in it, or when the kernel's source has changed since the counters
    were taken."""
    if workload not in PMC_SUMMARIES:
        return None
    fname, syms = PMC_SUMMARIES[workload]
    path = os.path.join(ROOT, "profiles", fname)
    if name not in syms or not os.path.exists(path):
        return None
    want = syms[name]
    with open(path) as f:
        for line in f:
            t = line.split()
            if len(t) == 8 and t[0] == "traffic" and t[1] == want:
                src = os.path.join(ROOT, "paper_1812_07903_amd", "csrc", t[2])
                with open(src, "rb") as g:
                    sha = hashlib.sha256(g.read()).hexdigest()[:16]
                return float(t[7]) if t[3] == sha else None
    return None


def _rate(bound: str, work: float, sec: float, peak_key: str):
    a = work / sec
    p = PEAK[peak_key]
    if bound == "hbm":
        return {"bound": "hbm", "achieved": a / 1e9, "peak": p / 1e9,
                "unit": "GB/s", "frac": a / p, "traffic": None}
    return {"bound": bound, "achieved": a / 1e12, "peak": p / 1e12,
            "unit": "TFLOP/s", "frac": a / p, "traffic": None}


def _roofline(name: str, sh: Shape, sec: float, launches: float):
    """Algorithmic work of one launch of a kernel at this job's shape."""
    n, d, r, k = sh.n, sh.d, sh.r, sh.k
    if name == "gauss_sketch":
        # S X: 2 r n d flop on the MFMA of the input's precision (BF16 for
        # BF16 and FP8 input, FP32 for FP32 input)
        key = "fp32" if sh.dtype == "f32" else "bf16"
        return _rate("mfma", 2.0 * r * n * d / launches, sec, key)
    if name == "gram":
        # refinement Gram (X D)^T (X D): X read once (n d xbytes); the
        # d (d + 1) n flop of its upper triangle take less time on the MFMA
        return _rate("hbm", float(n) * d * sh.xbytes / launches, sec, "hbm")
    if name == "score":
        # X once, M's parts (three BF16 parts of d x 64 for FP32 input, one
        # FP32 copy otherwise), the scores
        if sh.dtype == "csr":
            b = sh.nnz * 8.0 + (n + 1) * 8.0 + d * k * 4.0 + n * 4.0
        else:
            mb = 6.0 * d * 64 if sh.dtype == "f32" else 4.0 * d * k
            b = float(n) * d * sh.xbytes + mb + n * 4.0
        return _rate("hbm", b / launches, sec, "hbm")
    if name == "countsketch":
        if sh.dtype == "csr":
            # CSR once (values, column indices, row pointers), the sorted
            # row list, the sketch written once
            b = sh.nnz * 8.0 + (n + 1) * 8.0 + n * 4.0 + r * d * 8.0
        else:
            # X once, the sketch written once, the sorted row list, the
            # per-workgroup column maxima (min(1024, r / 4) x d floats)
            b = (float(n) * d * sh.xbytes + r * d * 8.0 + n * 4.0
                 + min(1024, r // 4) * d * 4.0)
        return _rate("hbm", b / launches, sec, "hbm")
    if name == "cq2_gram":
        # the upper triangle of A^T A over the r x d sketch: d (d + 1) / 2
        # entries of r products each when the last column block is at most
        # 16 wide (formed by the same launch), else the part inside full
        # 128-column blocks (c = 128 floor(d / 128))
        # Each job launches both passes; after one pass the second launch
        # exits at once, so the work of a launch is the passes' work over the
        # launches
        c = d if d % 128 <= 16 else 128 * (d // 128)
        return _rate("mfma", sh.qr_passes * float(r) * c * (c + 1) / launches,
                     sec, "fp64")
    if name == "cq2_solve":
        # Q1 = A R1^{-1}: r d^2 flop (not run after one pass)
        if sh.qr_passes == 1:
            return None
        return _rate("mfma", float(r) * d * d, sec, "fp64")
    if name in ("cq2_chol", "cq2_r"):
        # d^3 / 3 flop
        out = _rate("alu", d ** 3 / 3.0, sec, "fp64")
        return out
    return None


def roofline_for(name, sh, ms_per_launch, launches_per_step, workload):
    rr = _roofline(name, sh, ms_per_launch * 1e-3, launches_per_step)
    if rr is not None:
        rr["traffic"] = measured_traffic(name, workload)
    return rr


# ---- host facts ------------------------------------------------------------------
def host_facts() -> dict:
    model, mem = "unknown", None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for ln in f:
                if ln.startswith("MemTotal"):
                    mem = int(ln.split()[1]) * 1024
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "usable_cpus": usable,
            "host_ram_gib": None if mem is None else round(mem / 2 ** 30, 1)}


def blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count() or 1


# ---- one job, timed --------------------------------------------------------------
def tune_job(slso, ctx, x, r, k, sketch, nnz=0) -> dict:
    """slso_tune on the job's input (outside any timed region): the launch
    shape recorded per tunable pass for (d, dtype), -1 where the input does
    not take the pass."""
    ctx.tune(x, r, k, sketch=sketch, nnz=nnz)
    m = slso._matrix(x)
    return {"score_ring": slso.tune_get(slso.TUNE_SCORE, m.d, m.dtype),
            "countsketch_rows": slso.tune_get(slso.TUNE_COUNTSKETCH, m.d,
                                              m.dtype)}


def time_job(slso, ctx, x, n, seed, r, k, steps, warmup, sketch, refine=False,
             nnz=0, label=""):
    """Launch shapes tuned on the input, warm-up, a per-kernel breakdown
    pass, then ``steps`` timed steps with HIP events around the dominant
    kernel's launches only."""
    import numpy as np
    import torch
    scores = torch.empty(n, dtype=torch.float32, device="cuda")
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    tuned = tune_job(slso, ctx, x, r, k, sketch, nnz)

    def step():
        _, info = ctx.leverage(x, seed, r, k, out=scores, stream=stream,
                               sketch=sketch, refine=refine, nnz=nnz)
        ctx.order(scores, out=perm, stream=stream)
        return info

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    slso.profile_read()
    slso.profile_only(None)
    slso.profile_enable(True)
    nb = max(2, min(3, steps))
    for _ in range(nb):
        step()
    prof = slso.profile_read()
    kernels = {kk: {"ms_per_step": v[0] / nb, "launches_per_step": v[1] / nb}
               for kk, v in prof.items() if v[1] > 0}
    dname = max(kernels, key=lambda kk: kernels[kk]["ms_per_step"])
    slso.profile_only(dname)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        info = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    dprof = slso.profile_read()
    slso.profile_enable(False)
    slso.profile_only(None)
    got = scores.cpu().numpy()
    perm_h = perm.cpu().numpy().astype(np.int64)
    perm_ok = bool(np.array_equal(perm_h, np.argsort(-got, kind="stable")))
    lat_ms = np.array(lat) * 1e3
    dms, dcount = dprof[dname]
    log(f"{label}: {1e3 * total / steps:.3f} ms/step, dominant {dname} "
        f"{dms / max(dcount, 1):.3f} ms/launch")
    return {"ms_per_step": 1e3 * total / steps, "rows_per_s": n * steps / total,
            "p50_ms": float(np.percentile(lat_ms, 50)),
            "p99_ms": float(np.percentile(lat_ms, 99)),
            "kernels": kernels, "dominant": dname,
            "dominant_ms_per_launch": dms / max(dcount, 1),
            "dominant_launches_per_step": dcount / steps,
            "rank": int(info["rank"]), "flags": int(info["flags"]),
            "tuned": tuned,
            "perm_matches_stable_sort": perm_ok, "scores": got}


def rooflines(res, sh, workload, others=()):
    dname = res["dominant"]
    roof = roofline_for(dname, sh, res["dominant_ms_per_launch"],
                        res["dominant_launches_per_step"], workload)
    other = {}
    for kk in others:
        if kk in res["kernels"] and kk != dname:
            kv = res["kernels"][kk]
            rr = roofline_for(kk, sh, kv["ms_per_step"] / kv["launches_per_step"],
                              kv["launches_per_step"], workload)
            if rr:
                other[kk] = dict(kernel=kk, **rr)
    return (dict(kernel=dname, **roof) if roof else None), other


def gpu_scores(slso, ctx, x, seed, r, k, sketch, refine=False, nnz=0):
    import torch
    sc, info = ctx.leverage(x, seed, r, k, sketch=sketch, refine=refine,
                            nnz=nnz)
    torch.cuda.synchronize()
    return sc.cpu().numpy(), info


# ---- workloads ---------------------------------------------------------------------
PREC = dict(n=4_000_000, d=512, r=2048, k=64, seed=2003, data_seed=1003)
IMAGE = dict(n=60000, d=784, r=16384, k=64, seed=2001, data_seed=1001)
TEXT = dict(n=500000, d=4096, r=32768, k=64, seed=2002, data_seed=1002)


def precision_bench(args, slso, ctx) -> dict:
    """The precision form: BF16 (headline), FP8 and plain FP32 paths."""
    import numpy as np
    import torch

    import synth
    P = PREC
    n, d, r, k, seed = P["n"], P["d"], P["r"], P["k"], P["seed"]
    t0 = time.perf_counter()
    x64 = synth.precision_dense_device(n, d, 256, P["data_seed"])
    xb = x64.to(torch.bfloat16)
    codes, cs = synth.to_fp8_e4m3_device(x64)
    x8 = slso.Fp8Matrix(codes, cs)
    xf = x64.to(torch.float32)
    del x64
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"precision inputs ready in {time.perf_counter() - t0:.1f} s")

    bf = time_job(slso, ctx, xb, n, seed, r, k, args.steps, args.warmup,
                  slso.GAUSSIAN, refine=True, label="precision bf16")
    sh_b = Shape(n, d, r, k, 2, "bf16")
    roof, roof_other = rooflines(bf, sh_b, "precision_bf16",
                                 ("gauss_sketch", "gram", "score"))
    side_steps = max(2, min(5, args.steps))
    f8 = time_job(slso, ctx, x8, n, seed, r, k, side_steps, 1, slso.GAUSSIAN,
                  refine=True, label="precision fp8")
    f32 = time_job(slso, ctx, xf, n, seed, r, k, side_steps, 1, slso.GAUSSIAN,
                   refine=False, label="precision f32 plain")
    paths = {}
    for name, res, sh, wl in (
            ("fp8", f8, Shape(n, d, r, k, 1, "fp8"), "precision_fp8"),
            ("f32_plain", f32, Shape(n, d, r, k, 4, "f32"), "precision_f32")):
        rf, ro = rooflines(res, sh, wl, ("gauss_sketch", "gram", "score"))
        paths[name] = {"rows_per_s": res["rows_per_s"],
                       "ms_per_step": res["ms_per_step"],
                       "p50_ms": res["p50_ms"], "p99_ms": res["p99_ms"],
                       "steps": side_steps, "rank": res["rank"],
                       "kernels": res["kernels"], "roofline": rf,
                       "roofline_other": ro, "tuned": res["tuned"],
                       "perm_matches_stable_sort":
                           res["perm_matches_stable_sort"]}
    # property that holds at any size: with the refinement R is the R factor
    # of X D, so X R^-1 has orthonormal columns and the scores sum to
    # ||Pi_2||_F^2 (checked against the oracle's Pi_2 in the CPU leg)
    out = {
        "metric": METRIC, "value": bf["rows_per_s"], "unit": "rows/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": bf["ms_per_step"], "p50_ms": bf["p50_ms"],
        "p99_ms": bf["p99_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "precision form: dense BF16 X (n=4e6, d=512, "
                               "rank 256, sigma_j=j^-1.5, noise 1e-4, row "
                               "scales e^N(0,1.5^2)); Gaussian sketch r=2048 "
                               "on MFMA, Cholesky-QR refinement, FP64 QR/rank/"
                               "R^-1, k=64, scores + dec ordering",
                   "n": n, "d": d, "r": r, "k": k, "seed": seed,
                   "refine": True, "rank": bf["rank"]},
        "perm_matches_stable_sort": bf["perm_matches_stable_sort"],
        "kernels": bf["kernels"], "roofline": roof,
        "roofline_other": roof_other, "paths": paths, "tuned": bf["tuned"],
    }
    if not args.no_cpu_baseline:
        out.update(precision_check(args, slso, ctx, xb, x8, xf, bf, f8))
    del xb, x8, xf, codes, cs
    torch.cuda.empty_cache()
    return out


def precision_check(args, slso, ctx, xb, x8, xf, bf, f8) -> dict:
    """The oracle leg: timed on a bounded sample job (the first rows of the
    same X as a job of their own), which also gives the error figures; the
    full-size scores are checked by the sum identity."""
    import numpy as np
    import torch

    import synth
    from oracle import leverage as olv
    from oracle import metrics as omet
    from oracle import order as oorder
    from oracle import streams as ost
    from threadpoolctl import threadpool_limits
    P = PREC
    d, r, k, seed = P["d"], P["r"], P["k"], P["seed"]
    ns = args.sample_rows
    res = {}
    # BF16: oracle timed on the sample (all BLAS threads)
    xb_s = xb[:ns].contiguous()
    got_b, _ = gpu_scores(slso, ctx, xb_s, seed, r, k, slso.GAUSSIAN, True)
    xv = synth.bf16_bits_to_f64(xb_s.view(torch.int16).cpu().numpy()
                                .view(np.uint16))
    threads = blas_threads()
    tc = time.perf_counter()
    ref = olv.sketched_leverage(xv, seed, r, k, refine=True)
    oorder.dec_order(ref["scores"].astype(np.float32))
    t_all = time.perf_counter() - tc
    res["rel_err_vs_fp64"] = omet.max_rel_err(got_b, ref["scores"])
    res["kendall_tau_vs_fp64"] = omet.kendall_tau(got_b, ref["scores"])
    log(f"bf16 sample: err {res['rel_err_vs_fp64']:.3e} "
        f"tau {res['kendall_tau_vs_fp64']:.6f}, oracle {t_all:.1f} s")
    # one BLAS thread on a quarter of the sample
    n1 = max(d + 1, ns // 4)
    with threadpool_limits(limits=1):
        tc = time.perf_counter()
        r1 = olv.sketched_leverage(xv[:n1], seed, r, k, refine=True)
        oorder.dec_order(r1["scores"].astype(np.float32))
        t_one = time.perf_counter() - tc
    facts = host_facts()
    res["cpu_baseline"] = {
        "value": ns / t_all, "unit": "rows/s", "cores": threads,
        "kind": "oracle",
        "sample": f"one job of the first {ns} rows of the BF16 input (same "
                  "seed, r, k; refined): oracle sketched leverage (numpy "
                  "FP64, Householder QR of X D) + dec ordering",
        "one_thread": {"value": n1 / t_one, "unit": "rows/s", "cores": 1,
                       "sample": f"the first {n1} rows as a job"},
        **facts}
    # FP8 on the same sample
    x8_s = slso.Fp8Matrix(x8.codes[:ns].contiguous(), x8.col_scale)
    got_8, _ = gpu_scores(slso, ctx, x8_s, seed, r, k, slso.GAUSSIAN, True)
    xv8 = synth.fp8_e4m3_to_f64(x8_s.codes.cpu().numpy(),
                                x8.col_scale.cpu().numpy())
    ref8 = olv.sketched_leverage(xv8, seed, r, k, refine=True)
    res["paths_err"] = {"fp8": {
        "rel_err_vs_fp64": omet.max_rel_err(got_8, ref8["scores"]),
        "kendall_tau_vs_fp64": omet.kendall_tau(got_8, ref8["scores"])}}
    # plain FP32: the sketched (unrefined) oracle generates every entry of
    # the Gaussian sketch, so its sample is smaller
    nf = args.sample_rows_f32
    xf_s = xf[:nf].contiguous()
    got_f, _ = gpu_scores(slso, ctx, xf_s, seed, r, k, slso.GAUSSIAN, False)
    reff = olv.sketched_leverage(xf_s.cpu().numpy().astype(np.float64), seed,
                                 r, k, kind="gaussian", precision="f32")
    res["paths_err"]["f32_plain"] = {
        "rel_err_vs_fp64": omet.max_rel_err(got_f, reff["scores"]),
        "kendall_tau_vs_fp64": omet.kendall_tau(got_f, reff["scores"]),
        "sample_rows": nf}
    # full size: sum of the refined scores = ||Pi_2||_F^2
    pi_f2 = float((ost.pi2_matrix(seed, d, k) ** 2).sum())
    res["full_size_check"] = {
        "bf16_sum_over_pi2_frob2": float(bf["scores"].astype(np.float64).sum())
        / pi_f2,
        "fp8_sum_over_pi2_frob2": float(f8["scores"].astype(np.float64).sum())
        / pi_f2}
    res["err_sample"] = (f"a job of the first {ns} rows (BF16, FP8) and "
                         f"{nf} rows (plain FP32) of the same inputs")
    return res


def text_bench(args, slso, ctx, steps=None, warmup=None) -> dict:
    import numpy as np
    import torch

    import synth
    T = TEXT
    n, d, r, k, seed = T["n"], T["d"], T["r"], T["k"], T["seed"]
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    t0 = time.perf_counter()
    c = synth.config2(n, d, T["data_seed"])
    x = slso.CsrMatrix(n, d, torch.from_numpy(c.row_ptr).cuda(),
                       torch.from_numpy(c.col_idx).cuda(),
                       torch.from_numpy(c.val).cuda())
    torch.cuda.synchronize()
    log(f"text-like CSR ready in {time.perf_counter() - t0:.1f} s "
        f"(nnz {c.nnz})")
    res = time_job(slso, ctx, x, n, seed, r, k, steps, warmup,
                   slso.COUNTSKETCH, label="text-like csr")
    sh = Shape(n, d, r, k, 8, "csr", nnz=c.nnz,
               qr_passes=1 if res["flags"] & 32 else 2)
    roof, other = rooflines(res, sh, "text", ("cq2_gram", "cq2_solve",
                                              "cq2_chol", "countsketch",
                                              "score"))
    out = {"rows_per_s": res["rows_per_s"], "ms_per_step": res["ms_per_step"],
           "p50_ms": res["p50_ms"], "p99_ms": res["p99_ms"], "steps": steps,
           "config": {"workload": "text-like CSR X (n=5e5, d=4096, 0.5% "
                                  "dense, Zipf(1.1) columns, tf-idf values); "
                                  "CountSketch on CSR r=32768, FP64 QR, k=64, "
                                  "scores + dec ordering",
                      "n": n, "d": d, "r": r, "k": k, "seed": seed,
                      "nnz": c.nnz, "rank": res["rank"]},
           "flags": res["flags"], "tuned": res["tuned"],
           "perm_matches_stable_sort": res["perm_matches_stable_sort"],
           "kernels": res["kernels"], "roofline": roof,
           "roofline_other": other}
    return out, res, c


def image_bench(args, slso, ctx) -> dict:
    import numpy as np
    import torch

    import synth
    I = IMAGE
    n, d, r, k, seed = I["n"], I["d"], I["r"], I["k"], I["seed"]
    x_host = synth.config1(n, d)
    x = torch.from_numpy(x_host).cuda()
    kind = {"countsketch": slso.COUNTSKETCH, "osnap": slso.OSNAP,
            "srht": slso.SRHT}[args.sketch]
    nnz = args.nnz if args.sketch == "osnap" else 0
    res = time_job(slso, ctx, x, n, seed, r, k, args.steps, args.warmup, kind,
                   nnz=nnz, label="image-like")
    sh = Shape(n, d, r, k, 4, "f32", qr_passes=1 if res["flags"] & 32 else 2)
    roof, other = rooflines(res, sh, "image",
                            ("cq2_solve", "cq2_chol", "countsketch", "score"))
    out = {
        "metric": METRIC, "value": res["rows_per_s"], "unit": "rows/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"], "p50_ms": res["p50_ms"],
        "p99_ms": res["p99_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "image-like dense FP32 X (n=60000, d=784, "
                               "values in [0,1], rank 50 + noise, 10 clusters); "
                               + {"countsketch": "CountSketch ",
                                  "osnap": f"OSNAP (s={nnz}) ",
                                  "srht": "SRHT "}[args.sketch]
                               + "r=16384, FP64 QR, k=64, scores + dec ordering",
                   "n": n, "d": d, "r": r, "k": k, "seed": seed,
                   "rank": res["rank"]},
        "perm_matches_stable_sort": res["perm_matches_stable_sort"],
        "kernels": res["kernels"], "roofline": roof, "roofline_other": other,
        "tuned": res["tuned"],
    }
    if not args.no_cpu_baseline:
        import numpy as np
        from oracle import leverage as olv
        from oracle import metrics as omet
        from oracle import order as oorder
        got = res["scores"].astype(np.float64)
        reps, t_cpu, ref = 0, 0.0, None
        while reps < 40 and t_cpu < 10.0:
            tc = time.perf_counter()
            ref = olv.sketched_leverage(x_host, seed, r, k, kind=args.sketch,
                                        nnz=max(nnz, 1))
            oorder.dec_order(ref["scores"].astype(np.float32))
            t_cpu += time.perf_counter() - tc
            reps += 1
        out["cpu_baseline"] = {
            "value": n * reps / t_cpu, "unit": "rows/s",
            "cores": blas_threads(), "kind": "oracle",
            "sample": f"{reps} full job(s) of the same workload (n={n}): "
                      "oracle sketched leverage (numpy FP64) + dec ordering",
            **host_facts()}
        out["rel_err_vs_fp64"] = omet.max_rel_err(got, ref["scores"])
        out["kendall_tau_vs_fp64"] = omet.kendall_tau(got, ref["scores"])
    return out


def serving_run(args, slso) -> dict:
    """Continuous serving: jobs arrive as a Poisson stream and are admitted
    by the library's server (slots under an HBM budget); aggregate rows/s and
    p50/p99 latency from arrival to resident outputs, per arrival rate."""
    import numpy as np
    import torch

    import synth

    rates = [float(v) for v in args.rates.split(",") if v]
    t_gen = time.perf_counter()
    pool = synth.serving_pool(n=args.pool_n)
    torch.cuda.synchronize()
    log(f"serving pool of {len(pool)} base matrices ready in "
        f"{time.perf_counter() - t_gen:.1f} s")
    # launch shapes tuned per (d, dtype) of the pool before the stream, on a
    # job of the geometric-mean size (141421 rows, r = 6 d, k = 32); the
    # server's contexts read the same table
    tctx = slso.Context(0)
    tuned = {}
    for (dv, dt), xp in sorted(pool.items(), key=lambda kv: str(kv[0])):
        tuned[f"{dv}/{dt}"] = tune_job(slso, tctx, xp[:141421], 6 * dv, 32,
                                       slso.COUNTSKETCH)
    tctx.close()
    torch.cuda.synchronize()
    log(f"serving launch shapes tuned: {tuned}")
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
        bad = [q for q in res if q["status"] < 0]
        lat = np.array([q["latency_ms"] for q in res])
        span_ms = max(q["end_ms"] for q in res) - min(q["submit_ms"] for q in res)
        rows = sum(jb["n"] for jb in jobs)
        per_rate[str(int(rate))] = {
            "rows_per_s": rows / (span_ms * 1e-3), "jobs": len(jobs),
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "max_running": stats["max_running"], "failed": len(bad)}
        log(f"serving rate {rate:g}/s: {per_rate[str(int(rate))]}")
        if checked is None and not args.no_cpu_baseline:
            # accuracy of a stratified sample of jobs (one per d, the
            # smallest n of each) against the FP64 oracle
            from oracle import leverage as olv
            from oracle import metrics as omet
            errs, taus, picked = [], [], []
            for dv in sorted({jb["d"] for jb in jobs}):
                cand = [i for i in range(len(jobs)) if jobs[i]["d"] == dv]
                picked.append(min(cand, key=lambda i: jobs[i]["n"]))
            for i in picked:
                jb, t = jobs[i], tickets[i]
                xv = t.x.double().cpu().numpy()
                ref = olv.sketched_leverage(xv, jb["seed"], jb["r"], jb["k"])
                got = t.scores.cpu().numpy()
                errs.append(omet.max_rel_err(got, ref["scores"]))
                taus.append(omet.kendall_tau(got, ref["scores"]))
            checked = (max(errs), min(taus), len(picked))
        del tickets, res
    out = {"per_rate": per_rate, "jobs_per_rate": args.jobs,
           "slots": args.slots, "pool_rows": args.pool_n, "tuned": tuned,
           "config": {"workload": "serving: Poisson stream of leverage jobs, "
                                  "n log-uniform [1e4, 2e6], d in {64..1024}, "
                                  "FP32/BF16, CountSketch r=4d..8d, k=32, "
                                  "scores + dec ordering"}}
    if checked is not None:
        out["rel_err_vs_fp64"], out["kendall_tau_vs_fp64"] = checked[:2]
        out["jobs_checked"] = checked[2]
    del pool
    torch.cuda.empty_cache()
    return out


# ---- rocprofv3 summaries ------------------------------------------------------
def _kernel_sources() -> dict:
    """kernel function name -> csrc file that defines it"""
    import re
    out = {}
    csrc = os.path.join(ROOT, "paper_1812_07903_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if not f.endswith(".hip"):
            continue
        with open(os.path.join(csrc, f)) as fh:
            text = fh.read()
        for m in re.finditer(r"__global__([^;{]*)", text):
            # the first called-looking name that is not an attribute
            for nm in re.findall(r"\b(\w+)\s*\(", m.group(1)):
                if not nm.startswith("__"):
                    out.setdefault(nm, f)
                    break
    return out


def _short_name(name: str) -> str:
    """'void slso::(anonymous namespace)::k<1, true>(args)' -> 'k<1,true>'"""
    name = name.replace("void ", "").replace("slso::(anonymous namespace)::", "")
    name = name.replace("slso::", "")
    depth, cut = 0, len(name)
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    return name[:cut].replace(" ", "")


def _rocprof_csv(d: str, pattern: str) -> list:
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not files:
        raise SystemExit(f"no {pattern} under {d}")
    with open(files[0]) as fh:
        return list(csv.DictReader(fh))


def _field(row: dict, *names):
    low = {k.lower(): v for k, v in row.items()}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    raise KeyError(names)


def rocprof_stats(d: str, top: int = 40) -> int:
    """Kernel-trace statistics (rocprofv3 --kernel-trace --stats, CSV) as a
    table: calls, total and average duration per kernel."""
    rows = _rocprof_csv(d, "*kernel_stats.csv")
    print(f"{'kernel':58s} {'calls':>6s} {'total_us':>11s} {'avg_us':>10s} {'pct':>6s}")
    for r in rows[:top]:
        print(f"{_short_name(_field(r, 'Name', 'KernelName'))[:58]:58s} "
              f"{int(_field(r, 'Calls')):6d} "
              f"{float(_field(r, 'TotalDurationNs')) / 1e3:11.1f} "
              f"{float(_field(r, 'AverageNs')) / 1e3:10.3f} "
              f"{float(_field(r, 'Percentage')):6.2f}")
    return 0


def _counter_means(d: str, counter: str) -> dict:
    """kernel short name -> (dispatches, mean per dispatch of the counter)"""
    from collections import defaultdict
    per = defaultdict(lambda: defaultdict(float))
    for r in _rocprof_csv(d, "*counter_collection.csv"):
        if _field(r, "Counter_Name", "CounterName") != counter:
            continue
        k = _short_name(_field(r, "Kernel_Name", "KernelName"))
        per[k][_field(r, "Dispatch_Id", "DispatchId")] += float(
            _field(r, "Counter_Value", "CounterValue"))
    return {k: (len(v), sum(v.values()) / len(v)) for k, v in per.items()}


def rocprof_counters(d: str) -> int:
    """Mean per dispatch of every counter of a rocprofv3 --pmc CSV output
    folder, for the library's kernels (one line per kernel)."""
    from collections import defaultdict
    per = defaultdict(lambda: defaultdict(lambda: defaultdict(float)))
    for r in _rocprof_csv(d, "*counter_collection.csv"):
        k = _short_name(_field(r, "Kernel_Name", "KernelName"))
        c = _field(r, "Counter_Name", "CounterName")
        per[k][c][_field(r, "Dispatch_Id", "DispatchId")] += float(
            _field(r, "Counter_Value", "CounterValue"))
    srcs = _kernel_sources()
    for k in sorted(per):
        if k.split("<")[0] not in srcs:
            continue
        cs = per[k]
        nd = max(len(v) for v in cs.values())
        print(f"counters {k} dispatches {nd} " + " ".join(
            f"{c}={sum(v.values()) / len(v):.4g}" for c, v in sorted(cs.items())))
    return 0


def rocprof_traffic(fetch_dir: str, write_dir: str, cfetch_dir: str,
                    cwrite_dir: str, copy_mib: int) -> int:
    """HBM bytes per dispatch of every library kernel from a FETCH_SIZE and a
    WRITE_SIZE run (KiB per dispatch), each scaled by what the counter reads
    for a plain copy of copy_mib MiB (the --copy-calibration kernel): one
    'traffic' line per kernel with its source file and that file's hash."""
    cf = _counter_means(cfetch_dir, "FETCH_SIZE")
    cw = _counter_means(cwrite_dir, "WRITE_SIZE")
    kib = copy_mib * 1024.0
    copy_f = max(cf.values(), key=lambda t: t[1])[1]
    copy_w = max(cw.values(), key=lambda t: t[1])[1]
    ff, wf = kib / copy_f, kib / copy_w
    print(f"# copy kernel: FETCH_SIZE {copy_f:.2f} KiB and WRITE_SIZE "
          f"{copy_w:.2f} KiB per launch for {kib:.0f} KiB read and written")
    fetch = _counter_means(fetch_dir, "FETCH_SIZE")
    write = _counter_means(write_dir, "WRITE_SIZE")
    srcs = _kernel_sources()
    rows = []
    for k, (nd, fv) in fetch.items():
        base = k.split("<")[0]
        if base not in srcs:
            continue
        src = srcs[base]
        with open(os.path.join(ROOT, "paper_1812_07903_amd", "csrc", src), "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()[:16]
        wv = write.get(k, (0, 0.0))[1]
        rows.append((fv * 1024 * ff + wv * 1024 * wf, k, src, sha, nd, fv, wv))
    for b, k, src, sha, nd, fv, wv in sorted(rows, reverse=True):
        print(f"traffic {k} {src} {sha} {nd} {fv:.2f} {wv:.2f} {b:.0f}")
    print(f"calibration fetch_factor {ff:.6f} write_factor {wf:.6f}")
    return 0


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



def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload",
                    choices=("precision", "image", "text", "serving"),
                    default="precision")
    ap.add_argument("--headline-only", action="store_true",
                    help="precision: skip the text-like and serving keys")
    ap.add_argument("--sample-rows", type=int, default=262147,
                    help="precision: rows of the oracle's sample job")
    ap.add_argument("--sample-rows-f32", type=int, default=16411,
                    help="precision: rows of the plain FP32 path's sample job")
    ap.add_argument("--sketch", choices=("countsketch", "osnap", "srht"),
                    default="countsketch", help="image: the sketch")
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
    ap.add_argument("--rocprof-stats", metavar="DIR",
                    help="only print the kernel statistics of a rocprofv3 "
                         "--kernel-trace --stats CSV output folder")
    ap.add_argument("--rocprof-counters", metavar="DIR",
                    help="only print mean counter values per dispatch of the "
                         "library's kernels from a rocprofv3 --pmc CSV folder")
    ap.add_argument("--rocprof-traffic", nargs=5,
                    metavar=("FETCH", "WRITE", "CFETCH", "CWRITE", "MIB"),
                    help="only print HBM bytes per dispatch from rocprofv3 "
                         "--pmc FETCH_SIZE / WRITE_SIZE CSV folders of a run "
                         "and of --copy-calibration MIB")
    args = ap.parse_args()
    if args.rocprof_stats:
        return rocprof_stats(args.rocprof_stats)
    if args.rocprof_counters:
        return rocprof_counters(args.rocprof_counters)
    if args.rocprof_traffic:
        f, w, cf, cw, mib = args.rocprof_traffic
        return rocprof_traffic(f, w, cf, cw, int(mib))
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the leverage path runs on a "
              "single MI355X (rows would shard across GPUs with one reduction "
              "of the sketch); run with --gpus 1", file=sys.stderr)
        return 2

    import paper_1812_07903_amd as slso
    slso.load_library()

    if args.workload == "serving":
        srv = serving_run(args, slso)
        top = srv["per_rate"][args.rates.split(",")[-1].split(".")[0]]
        out = {"metric": METRIC, "value": top["rows_per_s"], "unit": "rows/s",
               "n_gpus": 1, "steps": args.jobs, "warmup": 0,
               "ms_per_step": None, "p50_ms": top["p50_ms"],
               "p99_ms": top["p99_ms"], "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None,
               "dtype": "f64+f32+bf16", "data": "synthetic", **srv}
        print(json.dumps(out), flush=True)
        return 0

    ctx = slso.Context(0)
    if args.workload == "image":
        out = image_bench(args, slso, ctx)
    elif args.workload == "text":
        txt, res, _ = text_bench(args, slso, ctx)
        out = {"metric": METRIC, "value": txt["rows_per_s"], "unit": "rows/s",
               "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": txt["ms_per_step"], "p50_ms": txt["p50_ms"],
               "p99_ms": txt["p99_ms"], "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
               "data": "synthetic", **txt}
    else:
        out = precision_bench(args, slso, ctx)
        if not args.headline_only:
            txt, _, _ = text_bench(args, slso, ctx, steps=max(3, args.steps // 4),
                                   warmup=1)
            out["text_like"] = txt
            ctx.close()
            ctx = None
            out["serving"] = serving_run(args, slso)
    if ctx is not None:
        ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
