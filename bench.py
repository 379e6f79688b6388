#!/usr/bin/env python3
"""Bench: top-k principal components of a packed genotype matrix on one MI355X.

Workload (default): 10,000 individuals x 100,000 SNPs, five Balding-Nichols
subpopulations (F 0.005..0.02), 2% of individuals in related pairs, MAF ~
U(0.01, 0.5), 1% missing, 2-bit packed (250 MB); top k = 20 by FP64 GKL with
partial reorthogonalisation (omega = 1e-8) and thick restart (basis 60).

A step is one pass of the hot path: gkl_create (device column statistics and
internal layout) + gkl_solve (the Lanczos iteration to tolerance, Ritz
extraction, output) + gkl_destroy, with the packed matrix already in HBM.
Prints one JSON line.  `value` is seconds per step (lower is better).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "top-k PC solve time + matvec HBM GB/s, split-BF16 blocked vs FP64 GKL"
HBM_PEAK_GBPS = 8000.0

WORKLOADS = {
    "c2": dict(name="c2", k=20, tol=1e-10, reorth="partial", krylov_dim=60,
               desc="10,000 x 100,000 genotypes, 5 subpopulations + related pairs, 1% missing; "
                    "k=20, FP64 GKL, PRO omega=1e-8, thick restart m=60"),
    "c1": dict(name="c1", k=10, tol=1e-10, reorth="full", krylov_dim=0,
               desc="1,000 x 5,000 genotypes, 2 subpopulations, 1% missing; k=10, FP64 GKL, "
                    "full CGS2, no restart"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(workload, kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when the kernel source changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"{workload}_fp64_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    src = os.path.join(ROOT, rec["kernel_source"])
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    k = rec["per_launch_bytes"].get(kernel)
    return None if k is None else int(k["fetch"] + k["write"])


def cpu_baseline(g, gpu_matvecs, seconds):
    """Time the oracle (plain FP64 CPU GKL, full CGS2) on the same matrix for a
    bounded number of steps and scale its per-product time to the GPU solve's
    product count."""
    import numpy as np

    import oracle
    import synth
    cores = len(os.sched_getaffinity(0))
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    op = oracle.PackedOperator(g.packed, g.n, g.p)
    v0 = synth.start_vector(g.p, 1)
    t0 = time.perf_counter()
    oracle.gkl_svd(op, 1, tol=-1.0, v0=v0, max_steps=1)
    t1 = time.perf_counter() - t0
    steps = max(2, min(200, int(seconds / max(t1, 1e-6))))
    op.matvecs = 0
    t0 = time.perf_counter()
    res = oracle.gkl_svd(op, 1, tol=-1.0, v0=v0, max_steps=steps)
    t = time.perf_counter() - t0
    per_mvp = t / res.matvecs
    return {
        "value": per_mvp * gpu_matvecs,
        "unit": "s",
        "cores": min(threads, cores),
        "kind": "oracle",
        "sample": (f"oracle plain GKL (full CGS2, no restart) on the full matrix: first {steps} "
                   f"steps = {res.matvecs} products in {t:.1f} s ({per_mvp * 1e3:.1f} ms per "
                   f"product incl. its CGS2), scaled to the GPU solve's {gpu_matvecs} products"),
    }


MFMA_BF16_PEAK_TFLOPS = 2500.0
MFMA_INT8_PEAK_TOPS = 5000.0
# product launches are bracketed with HIP events one in TIMING_STRIDE (per
# product): a recorded event stalls the stream for a few microseconds, so
# timing every launch would slow the timed solves themselves
TIMING_STRIDE = 8


def run_mixed(gk, torch, G, n, p, k, args, sigma_fp64, stream, fmt="bf16"):
    """The same top-k solve by the blocked path, its products in split BF16 (fmt
    "bf16", GKL_PREC_MIXED) or exact int8 limbs (fmt "int8", GKL_PREC_MIXED_INT8);
    timed like the FP64 steps."""
    import numpy as np
    import synth
    b = args.block_width
    v0 = torch.from_numpy(np.ascontiguousarray(
        np.random.default_rng([1, 0x6D6978]).standard_normal((b, p)))).cuda()
    precision = gk.GKL_PREC_MIXED if fmt == "bf16" else gk.GKL_PREC_MIXED_INT8
    opts = dict(v0=v0, precision=precision, block_width=b, timing=TIMING_STRIDE, stream=stream)
    sig = torch.empty(k, dtype=torch.float64, device="cuda")
    U = torch.empty((k, n), dtype=torch.float64, device="cuda")
    V = torch.empty((k, p), dtype=torch.float64, device="cuda")
    tol = 1e-8

    def one():
        ctx = gk.Context(G, n, p, k, tol, gk.GKL_REORTH_FULL, **opts)
        try:
            return gk.gkl_solve(ctx.ctx, sig, U, n, V, p)
        finally:
            ctx.close()

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, info = one()
        infos.append(info)
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / args.steps
    s_mixed = sig.cpu().numpy()
    rel = np.abs(s_mixed - sigma_fp64) / sigma_fp64
    mv_ms = sum(i.matvec_kernel_ms for i in infos)
    rmv_ms = sum(i.rmatvec_kernel_ms for i in infos)
    mv_n = sum(i.timed_matvecs for i in infos)
    rmv_n = sum(i.timed_rmatvecs for i in infos)
    last = infos[-1]
    alg_bytes = ((n + 3) // 4) * p + b * (4 * p + 8 * n)
    if fmt == "bf16":
        exec_flop = 8.0 * n * p * b           # g and m operands, each hi + lo
        peak = MFMA_BF16_PEAK_TFLOPS
    else:
        # two operands (codes, missing flags) x limb tiles of 16 columns: 2 tiles
        # for b <= 8, 3 per 16 columns otherwise; 2 ops per multiply-add
        tiles = 2 if b <= 8 else 3 * ((b + 15) // 16)
        exec_flop = 2.0 * 2 * 16 * tiles * n * p
        peak = MFMA_INT8_PEAK_TOPS
    out = {"format": fmt, "block_width": b, "tol": tol, "value_s_per_step": step_s,
           "solve_s": float(np.mean([i.solve_ms for i in infos])) / 1e3,
           "create_s": float(np.mean([i.create_ms for i in infos])) / 1e3,
           "converged": int(last.converged), "matvecs": int(last.matvecs),
           "block_steps": int(last.steps), "restarts": int(last.restarts),
           "sigma_max_rel_err_vs_fp64": float(rel.max()),
           "sigma_rel_err_vs_fp64": [float(x) for x in rel]}
    for name, ms, cnt in (("matmat_mixed (A W)", mv_ms, mv_n), ("rmatmat_mixed (A^T X)", rmv_ms, rmv_n)):
        avg = ms / max(cnt, 1)
        out[name] = {"avg_launch_ms": avg, "launches": int(cnt),
                     "algorithmic_bytes_per_launch": int(alg_bytes),
                     "achieved_GBps": alg_bytes / (avg * 1e-3) / 1e9,
                     "hbm_frac": alg_bytes / (avg * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                     "mfma_executed_TFLOPs": exec_flop / (avg * 1e-3) / 1e12,
                     "mfma_frac": exec_flop / (avg * 1e-3) / 1e12 / peak}
    return out


def run_batched(gk, torch, args):
    """22 chromosome blocks (20,000 individuals, 8,000..80,000 SNPs, 700,000 in all)
    solved together by the batched path (persistent products, one HIP graph per
    Lanczos step, autotuned product geometry), beside the same 22 problems
    solved one after another through the single-problem entry points."""
    import numpy as np
    import synth
    log("[bench] batched: generating 22 chromosome blocks")
    gs = [synth.config("c4", chrom=c) for c in range(1, 23)]
    Gs = [torch.from_numpy(g.packed).cuda() for g in gs]
    ns = [g.n for g in gs]
    ps = [g.p for g in gs]
    k, tol, m = 10, 1e-10, 40
    v0s = [synth.start_vector(g.p, 100 + q) for q, g in enumerate(gs)]
    v0 = torch.from_numpy(np.concatenate(v0s)).cuda()
    t0 = time.perf_counter()
    ctx = gk.BatchedContext(Gs, ns, ps, k, tol=tol, v0=v0, krylov_dim=m, autotune=1, graph=1)
    create_s = time.perf_counter() - t0
    try:
        ctx.solve()                     # warmup (captures the step graph)
        torch.cuda.synchronize()
        times = []
        for _ in range(max(1, args.batched_steps)):
            t0 = time.perf_counter()
            sig, Us, Vs, st, infos = ctx.solve()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        plan = ctx.plan()
    finally:
        ctx.close()
    batch_s = float(np.mean(times))
    log(f"[bench] batched: {batch_s * 1e3:.1f} ms per solve, status {st}")
    bytes_pass = sum(((g.n + 3) // 4) * g.p + 16 * g.p + 16 * g.n for g in gs)
    t0 = time.perf_counter()
    seq_mv = 0
    for q, g in enumerate(gs):
        c1 = gk.Context(Gs[q], g.n, g.p, k, tol=tol, reorth=gk.GKL_REORTH_FULL,
                        v0=v0[sum(ps[:q]):sum(ps[:q + 1])], krylov_dim=m)
        try:
            _, _, _, _, info = c1.solve()
            seq_mv += info.matvecs
        finally:
            c1.close()
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t0
    out = {"workload": "22 chromosome blocks of 20,000 individuals x 8,000..80,000 SNPs "
                       "(701,314 in all), 4 subpopulations, 1% missing; k=10 each, FP64 GKL, "
                       "full CGS2, thick restart m=40",
           "problems": len(gs), "total_snps": int(sum(ps)), "packed_bytes": int(sum(g.nbytes for g in gs)),
           "k": k, "tol": tol, "krylov_dim": m, "status": int(st),
           "value_s_per_solve": batch_s, "create_s_incl_autotune": create_s,
           "converged": int(sum(i.converged for i in infos)),
           "steps_max": int(max(i.steps for i in infos)), "steps_min": int(min(i.steps for i in infos)),
           "restarts_max": int(max(i.restarts for i in infos)),
           "matvecs_total": int(sum(i.matvecs for i in infos)),
           "plan": plan,
           "sequential_single_solves_s": seq_s, "sequential_matvecs_total": int(seq_mv),
           "speedup_vs_sequential": seq_s / batch_s}
    for name, ms in (("batched_matvec (A v, all 22)", plan["mv_ms"]),
                     ("batched_rmatvec (A^T u, all 22)", plan["rmv_ms"])):
        if ms > 0:
            out[name] = {"avg_launch_ms": ms, "algorithmic_bytes_per_launch": int(bytes_pass),
                         "achieved_GBps": bytes_pass / (ms * 1e-3) / 1e9,
                         "hbm_frac": bytes_pass / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS}
    return out


def run_c3(gk, torch, args):
    """50,000 x 500,000 (6.25 GB packed): FP64 GKL (PRO, thick restart m=60) and the
    blocked solves (block width 8, split-BF16 and int8-limb products), one solve each
    after a warmup."""
    import numpy as np
    import synth
    log("[bench] c3: generating 50,000 x 500,000")
    g = synth.config("c3")
    n, p, k = g.n, g.p, 20
    G = torch.from_numpy(g.packed).cuda()
    sig = torch.empty(k, dtype=torch.float64, device="cuda")
    U = torch.empty((k, n), dtype=torch.float64, device="cuda")
    V = torch.empty((k, p), dtype=torch.float64, device="cuda")
    out = {"workload": "50,000 x 500,000 genotypes, 10 subpopulations + 20% admixed, 1% missing; k=20"}
    res = {}
    for label, tol, opts in (
            ("fp64", 1e-10, dict(v0=torch.from_numpy(synth.start_vector(p, 1)).cuda(),
                                 krylov_dim=60, reorth=gk.GKL_REORTH_PARTIAL)),
            ("mixed", 1e-8, dict(v0=torch.from_numpy(np.ascontiguousarray(
                np.random.default_rng([1, 0x6D6978]).standard_normal((8, p)))).cuda(),
                precision=gk.GKL_PREC_MIXED, block_width=8, reorth=gk.GKL_REORTH_FULL)),
            ("mixed_int8", 1e-8, dict(v0=torch.from_numpy(np.ascontiguousarray(
                np.random.default_rng([1, 0x6D6978]).standard_normal((8, p)))).cuda(),
                precision=gk.GKL_PREC_MIXED_INT8, block_width=8, reorth=gk.GKL_REORTH_FULL))):
        reorth = opts.pop("reorth")
        for rep in range(2):
            ctx = gk.Context(G, n, p, k, tol, reorth, timing=TIMING_STRIDE, **opts)
            try:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, info = gk.gkl_solve(ctx.ctx, sig, U, n, V, p)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            finally:
                ctx.close()
        res[label] = sig.cpu().numpy().copy()
        mv = info.matvec_kernel_ms / max(info.timed_matvecs, 1)
        rmv = info.rmatvec_kernel_ms / max(info.timed_rmatvecs, 1)
        out[label] = {"solve_s": dt, "status": int(st), "matvecs": int(info.matvecs),
                      "passes_over_G": int(info.passes_over_G), "restarts": int(info.restarts),
                      "avg_product_ms": [mv, rmv]}
        log(f"[bench] c3 {label}: {dt:.2f} s, {info.matvecs} matvecs")
    for key in ("mixed", "mixed_int8"):
        rel = np.abs(res[key] - res["fp64"]) / res["fp64"]
        out[key]["sigma_max_rel_err_vs_fp64"] = float(rel.max())
        out[key + "_speedup_vs_fp64"] = out["fp64"]["solve_s"] / out[key]["solve_s"]
    return out


def run_c5(gk, torch, args):
    """100,000 x 1,000,000 (25 GB packed), a pure noise bulk with ten planted spikes at
    1.5..20 times the bulk edge: the blocked solves (k = 10, b = 8; split-BF16 and int8-limb products) and the
    FP64 solve (PRO, m = 30), each once after nothing else has touched the matrix;
    reports the spike recovery against the planted ratios."""
    import numpy as np
    import synth
    log("[bench] c5: generating 100,000 x 1,000,000")
    g = synth.config("c5", progress=log)
    n, p, k = g.n, g.p, 10
    log("[bench] c5: copying 25 GB to the device")
    G = torch.from_numpy(g.packed).cuda()
    torch.cuda.synchronize()
    edge = g.meta["edge"]
    ratios = np.sort(np.array(g.meta["spike_ratios"]))[::-1]
    sig = torch.empty(k, dtype=torch.float64, device="cuda")
    U = torch.empty((k, n), dtype=torch.float64, device="cuda")
    V = torch.empty((k, p), dtype=torch.float64, device="cuda")
    out = {"workload": "100,000 x 1,000,000 genotypes, MAF ~ Beta(0.5,0.5) folded, 3% missing, "
                       "10 planted spikes at 1.5..20x the bulk edge; k=10",
           "packed_bytes": int(g.nbytes), "bulk_edge": edge, "planted_ratios": ratios.tolist()}
    res = {}
    for label, tol, opts, reorth in (
            ("mixed", 1e-8, dict(precision=gk.GKL_PREC_MIXED, block_width=8), gk.GKL_REORTH_FULL),
            ("mixed_int8", 1e-8, dict(precision=gk.GKL_PREC_MIXED_INT8, block_width=8),
             gk.GKL_REORTH_FULL),
            ("fp64", 1e-10, dict(v0=torch.from_numpy(synth.start_vector(p, 1)).cuda(), krylov_dim=30),
             gk.GKL_REORTH_PARTIAL)):
        log(f"[bench] c5: {label} create")
        t0 = time.perf_counter()
        ctx = gk.Context(G, n, p, k, tol, reorth, timing=TIMING_STRIDE, **opts)
        torch.cuda.synchronize()
        create_s = time.perf_counter() - t0
        try:
            log(f"[bench] c5: {label} solve")
            t0 = time.perf_counter()
            st, info = gk.gkl_solve(ctx.ctx, sig, U, n, V, p)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        finally:
            ctx.close()
        torch.cuda.empty_cache()
        s = sig.cpu().numpy().copy()
        res[label] = s
        mv = info.matvec_kernel_ms / max(info.timed_matvecs, 1)
        rmv = info.rmatvec_kernel_ms / max(info.timed_rmatvecs, 1)
        out[label] = {"solve_s": dt, "create_s": create_s, "status": int(st),
                      "matvecs": int(info.matvecs), "passes_over_G": int(info.passes_over_G),
                      "restarts": int(info.restarts), "avg_product_ms": [mv, rmv],
                      "sigma_over_edge": (s / edge).tolist(),
                      "sigma_vs_planted_ratio": (s / (ratios * edge) - 1.0).tolist()}
        log(f"[bench] c5 {label}: {dt:.2f} s, {info.matvecs} matvecs, status {st}")
    for key in ("mixed", "mixed_int8"):
        rel = np.abs(res[key] - res["fp64"]) / res["fp64"]
        out[key]["sigma_max_rel_err_vs_fp64"] = float(rel.max())
        out[key + "_speedup_vs_fp64"] = out["fp64"]["solve_s"] / out[key]["solve_s"]
    out["outliers_above_1.05_edge"] = int(np.sum(res["fp64"] > 1.05 * edge))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the blocked (split-BF16 and int8-limb) solves of the same workload")
    ap.add_argument("--block-width", type=int, default=8)
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched solve of the 22 chromosome blocks")
    ap.add_argument("--batched-steps", type=int, default=2)
    ap.add_argument("--c3", action="store_true",
                    help="also compare FP64 and mixed at 50,000 x 500,000 (adds about a minute)")
    ap.add_argument("--c5", action="store_true",
                    help="also solve 100,000 x 1,000,000 (25 GB) by both paths (adds a few minutes)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="after the timed steps, copy BYTES bytes device-to-device 3 times "
                         "(reference dispatch for the HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_1808_03374_amd as gk

    wl = WORKLOADS[args.workload]
    log(f"[bench] generating workload {wl['name']}")
    g = synth.config(wl["name"])
    n, p, k = g.n, g.p, wl["k"]
    G = torch.from_numpy(g.packed).cuda()
    v0 = torch.from_numpy(synth.start_vector(p, 1)).cuda()
    stream = torch.cuda.current_stream().cuda_stream
    reorth = gk.GKL_REORTH_PARTIAL if wl["reorth"] == "partial" else gk.GKL_REORTH_FULL
    opts = dict(v0=v0, krylov_dim=wl["krylov_dim"], timing=TIMING_STRIDE, stream=stream)
    sigma = torch.empty(k, dtype=torch.float64, device="cuda")
    U = torch.empty((k, n), dtype=torch.float64, device="cuda")
    V = torch.empty((k, p), dtype=torch.float64, device="cuda")

    def one_step():
        ctx = gk.Context(G, n, p, k, wl["tol"], reorth, **opts)
        try:
            st, info = gk.gkl_solve(ctx.ctx, sigma, U, n, V, p)
        finally:
            ctx.close()
        return st, info

    for w in range(args.warmup):
        st, info = one_step()
        log(f"[bench] warmup {w}: status {st} solve {info.solve_ms:.1f} ms matvecs {info.matvecs}")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        st, info = one_step()
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for s, info in enumerate(infos):
        log(f"[bench] step {s}: solve {info.solve_ms:.1f} ms create {info.create_ms:.1f} ms "
            f"matvecs {info.matvecs} restarts {info.restarts} conv {info.converged}")
    sec_per_step = elapsed / args.steps

    # dominant product kernel: average duration from the HIP events taken on the
    # library's stream during the timed steps
    mv_ms = sum(i.matvec_kernel_ms for i in infos)
    rmv_ms = sum(i.rmatvec_kernel_ms for i in infos)
    mv_n = sum(i.timed_matvecs for i in infos)
    rmv_n = sum(i.timed_rmatvecs for i in infos)
    bytes_per_product = ((n + 3) // 4) * p + 16 * p + 16 * n
    mv_avg = mv_ms / max(mv_n, 1)
    rmv_avg = rmv_ms / max(rmv_n, 1)
    kernels = {"matvec_kernel (A v)": (mv_ms, mv_avg), "rmatvec_kernel (A^T u)": (rmv_ms, rmv_avg)}
    dom = max(kernels, key=lambda key: kernels[key][0])
    dom_avg = kernels[dom][1]
    achieved = bytes_per_product / (dom_avg * 1e-3) / 1e9
    other = [key for key in kernels if key != dom][0]
    other_avg = kernels[other][1]
    solve_s = float(np.mean([i.solve_ms for i in infos])) / 1e3
    create_s = float(np.mean([i.create_ms for i in infos])) / 1e3
    last = infos[-1]
    line = {
        "metric": METRIC,
        "value": sec_per_step,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_per_step * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "n": n, "p": p, "k": k, "tol": wl["tol"],
                   "reorth": wl["reorth"], "krylov_dim": wl["krylov_dim"],
                   "packed_bytes": int(g.nbytes)},
        "solve_s": solve_s,
        "create_s": create_s,
        "matvecs": int(last.matvecs),
        "restarts": int(last.restarts),
        "reorth_passes": int(last.reorths),
        "converged": int(last.converged),
        "max_residual_rel": last.max_residual_rel,
        "matvec_GBps": bytes_per_product / (mv_avg * 1e-3) / 1e9,
        "rmatvec_GBps": bytes_per_product / (rmv_avg * 1e-3) / 1e9,
        "roofline": {
            "kernel": dom,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": measured_traffic(wl["name"], dom),
            "avg_launch_ms": dom_avg,
            "launches": int(mv_n if dom.startswith("matvec") else rmv_n),
            "timed_one_launch_in": TIMING_STRIDE,
            "algorithmic_bytes_per_launch": int(bytes_per_product),
            "other_kernel": {"kernel": other, "avg_launch_ms": other_avg,
                             "achieved_GBps": bytes_per_product / (other_avg * 1e-3) / 1e9},
        },
    }
    if not args.no_mixed:
        line["mixed"] = run_mixed(gk, torch, G, n, p, k, args, sigma.cpu().numpy(), stream)
        line["mixed_int8"] = run_mixed(gk, torch, G, n, p, k, args, sigma.cpu().numpy(), stream,
                                       fmt="int8")
    if not args.no_batched:
        line["batched"] = run_batched(gk, torch, args)
    if args.c3:
        line["c3"] = run_c3(gk, torch, args)
    if args.c5:
        line["c5"] = run_c5(gk, torch, args)
    if args.copy_calibration > 0:
        src = torch.empty(args.copy_calibration, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = args.copy_calibration
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(g, int(last.matvecs), args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
