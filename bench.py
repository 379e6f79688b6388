#!/usr/bin/env python3
"""Bench: top-k principal components of a packed genotype matrix on one MI355X.

Workload (default): 50,000 individuals x 500,000 SNPs, ten Balding-Nichols
subpopulations (F 0.005..0.02) plus 20% admixed individuals (Dirichlet(0.5)
weights), MAF ~ U(0.01, 0.5), 1% missing, 2-bit packed (6.25 GB); top k = 20.

The timed step (`value`) is one FP64 GKL solve with partial
reorthogonalisation (omega = 1e-8) and thick restart (basis 60) to tolerance
1e-10: gkl_create (column statistics, internal layouts) + gkl_solve (Lanczos
iteration, Ritz extraction, output) + gkl_destroy, with the packed matrix
already in HBM.  Beside it (`compare`) the same top-k problem is solved by the
blocked path whose products run on the BF16 matrix cores with split (hi + lo)
vector tiles, at block widths 8, 16 and 32, and by the FP64 path at the blocked
path's tolerance (equal accuracy); every blocked solve reports its error
against the FP64 solve for each sigma_i and the angle of each left and right
singular vector.  `cpu_baseline` times the CPU oracle on a bounded sample: the
residual certificate of the leading FP64 triplets on the full matrix.

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
MFMA_BF16_PEAK_TFLOPS = 2500.0
MFMA_INT8_PEAK_TOPS = 5000.0
# product launches are bracketed with HIP events one in TIMING_STRIDE (per
# product): a recorded event stalls the stream for a few microseconds, so
# timing every launch would slow the timed solves themselves
TIMING_STRIDE = 8
BLOCKED_TOL = 1e-8
ANGLE_TARGET = 1e-6

WORKLOADS = {
    "c3": dict(name="c3", k=20, tol=1e-10, reorth="partial", krylov_dim=60,
               desc="50,000 x 500,000 genotypes, 10 subpopulations + 20% admixed, 1% missing; "
                    "k=20, FP64 GKL, PRO omega=1e-8, thick restart m=60"),
    "c2": dict(name="c2", k=20, tol=1e-10, reorth="partial", krylov_dim=60,
               desc="10,000 x 100,000 genotypes, 5 subpopulations + related pairs, 1% missing; "
                    "k=20, FP64 GKL, PRO omega=1e-8, thick restart m=60"),
    "c1": dict(name="c1", k=10, tol=1e-10, reorth="full", krylov_dim=0,
               desc="1,000 x 5,000 genotypes, 2 subpopulations, 1% missing; k=10, FP64 GKL, "
                    "full CGS2, no restart"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def fp64_bytes(n, p):
    """Algorithmic bytes of one FP64 product: the packed matrix, the vector in and out."""
    return ((n + 3) // 4) * p + 16 * p + 16 * n


def block_bytes(n, p, b, transpose=False):
    """Algorithmic bytes of one block product of b vectors: the packed matrix,
    the vector block read once as split BF16 (hi + lo, 4 bytes per entry) and
    the FP64 result written (A W: W is p x b, Y n x b; A^T X: X n x b, Z p x b)."""
    rows_in, rows_out = (n, p) if transpose else (p, n)
    return ((n + 3) // 4) * p + b * (4 * rows_in + 8 * rows_out)


# FP64 product format of the FP64 solves: (gkl_fp64_products value, name)
FP64_PRODUCTS = [0, "auto"]
FORMAT_NAMES = {1: "lut", 2: "limbs", 3: "lut+limbs"}


def source_digest(path, region=None):
    """sha256 of a source file, or of the text between two marker strings of it."""
    import hashlib
    text = open(path, "rb").read()
    if region:
        a = text.index(region[0].encode())
        b = text.index(region[1].encode(), a)
        text = text[a:b]
    return hashlib.sha256(text).hexdigest()


def sources_digest(paths):
    """sha256 over the bytes of whole files, in order."""
    import hashlib
    h = hashlib.sha256()
    for path in paths:
        h.update(open(os.path.join(ROOT, path), "rb").read())
    return h.hexdigest()


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summaries of the workload (profiles/<workload>_*hbm_traffic*.md, one JSON
    record per summary), or None when none covers it or the kernel's source
    changed since the counters were taken (a record names either whole files,
    `sources`, or one file and a marked region of it)."""
    import glob
    import re
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"{workload}_*hbm_traffic*.md"))):
        for block in re.findall(r"```json\n(.*?)\n```", open(path).read(), re.S):
            rec = json.loads(block)
            k = rec.get("per_launch_bytes", {}).get(kernel)
            if k is None:
                continue
            try:
                if "sources" in rec:
                    digest = sources_digest(rec["sources"])
                else:
                    digest = source_digest(os.path.join(ROOT, rec["kernel_source"]), rec.get("region"))
            except (OSError, ValueError):
                return None
            if digest != rec["source_sha256"]:
                return None
            return int(k["fetch"] + k["write"])
    return None


def vector_angles(X, Y):
    """Angle (radians) between matching unit columns of X and Y, sign ignored:
    atan2(|x - (x.y) y|, |x.y|) per column (accurate for tiny angles)."""
    import numpy as np
    c = np.sum(X * Y, axis=0)
    r = X - Y * c[None, :]
    return np.arctan2(np.linalg.norm(r, axis=0), np.abs(c))


def relative_gaps(s):
    """delta_i = min_{j != i} |s_i - s_j| / s_i over the returned values."""
    import numpy as np
    d = np.abs(s[:, None] - s[None, :]) + np.diag(np.full(len(s), np.inf))
    return d.min(axis=1) / s


class Workload:
    """One packed matrix resident on the device plus its FP64 reference solve."""

    def __init__(self, gk, torch, wl, progress=True):
        import synth
        self.wl = wl
        log(f"[bench] generating {wl['name']}")
        t0 = time.perf_counter()
        self.g = synth.config(wl["name"], progress=log if progress else None)
        log(f"[bench] generated {self.g.nbytes / 1e9:.2f} GB in {time.perf_counter() - t0:.1f} s")
        self.n, self.p, self.k = self.g.n, self.g.p, wl["k"]
        self.G = torch.from_numpy(self.g.packed).cuda()
        torch.cuda.synchronize()
        self.v0 = torch.from_numpy(synth.start_vector(self.p, 1)).cuda()
        self.sigma = self.U = self.V = None


def fp64_solve(gk, torch, W, tol, steps, warmup, stream, keep=True, label="fp64", probe=None):
    """`steps` timed FP64 solves (create + solve + destroy) after `warmup` untimed ones."""
    import numpy as np
    wl = W.wl
    reorth = gk.GKL_REORTH_PARTIAL if wl["reorth"] == "partial" else gk.GKL_REORTH_FULL
    opts = dict(v0=W.v0, krylov_dim=wl["krylov_dim"], timing=TIMING_STRIDE, stream=stream,
                fp64_products=FP64_PRODUCTS[0])
    n, p, k = W.n, W.p, W.k
    sigma = torch.empty(k, dtype=torch.float64, device="cuda")
    U = torch.empty((k, n), dtype=torch.float64, device="cuda")
    V = torch.empty((k, p), dtype=torch.float64, device="cuda")
    probe_out = {}

    def one():
        ctx = gk.Context(W.G, n, p, k, tol, reorth, **opts)
        try:
            st, info = gk.gkl_solve(ctx.ctx, sigma, U, n, V, p)
        finally:
            ctx.close()
        return st, info

    for w in range(warmup):
        st, info = one()
        log(f"[bench] {label} warmup {w}: status {st} solve {info.solve_ms:.1f} ms "
            f"matvecs {info.matvecs}")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for s in range(steps):
        st, info = one()
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for s, info in enumerate(infos):
        log(f"[bench] {label} step {s}: solve {info.solve_ms:.1f} ms create {info.create_ms:.1f} ms "
            f"matvecs {info.matvecs} restarts {info.restarts} conv {info.converged}")
    if probe is not None:
        # FP64 products of a few random directions, for the blocked products' error
        pw, px = probe
        ctx = gk.Context(W.G, n, p, k, tol, reorth, **opts)
        try:
            probe_out["Y"] = torch.stack([ctx.matvec(pw[:, c].contiguous())
                                          for c in range(pw.shape[1])], dim=1)
            probe_out["Z"] = torch.stack([ctx.rmatvec(px[:, c].contiguous())
                                          for c in range(px.shape[1])], dim=1)
        finally:
            ctx.close()
        torch.cuda.synchronize()
    out = {"sec_per_step": elapsed / steps, "infos": infos, "status": int(st),
           "probe_Y": probe_out.get("Y"), "probe_Z": probe_out.get("Z")}
    if keep:
        out["sigma"] = sigma.cpu().numpy().copy()
        out["U"] = U.cpu().numpy().T.copy()
        out["V"] = V.cpu().numpy().T.copy()
    return out


KERNEL_NAMES = {"lut": ("matvec_lut_kernel (A v)", "rmatvec_lut_kernel (A^T u)"),
                "limbs": ("limb_product_kernel<A v>", "limb_product_kernel<A^T u>"),
                "lut+limbs": ("matvec_lut_kernel (A v)", "limb_product_kernel<A^T u>")}


def product_stats(infos, nbytes, products="lut"):
    """Average launch time of each product from the sampled HIP events, and rates."""
    mv_ms = sum(i.matvec_kernel_ms for i in infos)
    rmv_ms = sum(i.rmatvec_kernel_ms for i in infos)
    mv_n = sum(i.timed_matvecs for i in infos)
    rmv_n = sum(i.timed_rmatvecs for i in infos)
    mv_avg = mv_ms / max(mv_n, 1)
    rmv_avg = rmv_ms / max(rmv_n, 1)
    a, b = KERNEL_NAMES.get(products, ("A v", "A^T u"))
    return {a: {"total_ms": mv_ms, "avg_ms": mv_avg, "launches": mv_n,
                "GBps": nbytes / (mv_avg * 1e-3) / 1e9},
            b: {"total_ms": rmv_ms, "avg_ms": rmv_avg, "launches": rmv_n,
                "GBps": nbytes / (rmv_avg * 1e-3) / 1e9}}


def blocked_solve(gk, torch, W, b, fmt, ref, stream, reps=1, probe=None, probe_Y=None, tol=None):
    """Top-k by the blocked path (block width b, products in split BF16, int8
    limbs, or FP64-exact limb pairs for fmt "fp64") at tolerance tol (default
    BLOCKED_TOL): one warm-up solve, then `reps` timed ones; errors against the
    FP64 reference solve `ref`."""
    import numpy as np
    n, p, k = W.n, W.p, W.k
    tol = BLOCKED_TOL if tol is None else tol
    v0 = torch.from_numpy(np.ascontiguousarray(
        np.random.default_rng([1, 0x6D6978]).standard_normal((b, p)))).cuda()
    precision = {"bf16": gk.GKL_PREC_MIXED, "int8": gk.GKL_PREC_MIXED_INT8,
                 "fp64": gk.GKL_PREC_BLOCK_FP64}[fmt]
    opts = dict(v0=v0, precision=precision, block_width=b, timing=TIMING_STRIDE, stream=stream)
    sig = torch.empty(k, dtype=torch.float64, device="cuda")
    U = torch.empty((k, n), dtype=torch.float64, device="cuda")
    V = torch.empty((k, p), dtype=torch.float64, device="cuda")
    eps_op = eps_rel = None
    infos, times = [], []
    for rep in range(reps + 1):
        ctx = gk.Context(W.G, n, p, k, tol, gk.GKL_REORTH_FULL, **opts)
        try:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, info = gk.gkl_solve(ctx.ctx, sig, U, n, V, p)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if rep == 0 and probe is not None and probe_Y is not None:
                pw, px = probe
                probe_Z = ref["probe_Z"]
                Ym = ctx.matmat_mixed(pw)
                Zm = ctx.rmatmat_mixed(px)
                torch.cuda.synchronize()
                dY = torch.linalg.norm(Ym - probe_Y, dim=0)
                dZ = torch.linalg.norm(Zm - probe_Z, dim=0)
                eps_rel = float(max(torch.max(dY / torch.linalg.norm(probe_Y, dim=0)),
                                    torch.max(dZ / torch.linalg.norm(probe_Z, dim=0))))
                eps_op = float(max(torch.max(dY / torch.linalg.norm(pw, dim=0)),
                                   torch.max(dZ / torch.linalg.norm(px, dim=0)))) / float(ref["sigma"][0])
        finally:
            ctx.close()
        if rep > 0:
            infos.append(info)
            times.append(dt)
    s = sig.cpu().numpy()
    Uh = U.cpu().numpy().T
    Vh = V.cpu().numpy().T
    rel = np.abs(s - ref["sigma"]) / ref["sigma"]
    ang_u = vector_angles(Uh, ref["U"])
    ang_v = vector_angles(Vh, ref["V"])
    gaps = relative_gaps(ref["sigma"])
    # gap rule: a vector is held to the angle target when the bound
    # eps * sigma_1 / (delta_i sigma_i) on its error is itself below the target,
    # with eps the solve tolerance plus the measured product error
    # ||dY|| / (sigma_1 ||w||) on random unit vectors
    eps = tol + (eps_op or 0.0)
    bound = eps * ref["sigma"][0] / (gaps * ref["sigma"])
    gated = bound <= ANGLE_TARGET
    gated[-1] = False          # the gap below sigma_k is not known
    last = infos[-1]
    out = {"format": fmt, "block_width": b, "tol": tol, "status": int(st),
           "solve_s": float(np.mean(times)), "create_s": float(np.mean([i.create_ms for i in infos])) / 1e3,
           "converged": int(last.converged), "matvecs": int(last.matvecs),
           "passes_over_G": int(last.passes_over_G), "block_steps": int(last.steps),
           "restarts": int(last.restarts), "max_residual_rel": last.max_residual_rel,
           "sigma_max_rel_err_vs_fp64": float(rel.max()),
           "sigma_rel_err_vs_fp64": [float(x) for x in rel],
           "angle_u_vs_fp64": [float(x) for x in ang_u],
           "angle_v_vs_fp64": [float(x) for x in ang_v],
           "product_err_rel": eps_rel,
           "product_err_rel_to_sigma1": eps_op,
           "gap_rule_gated": [int(x) for x in gated],
           "gated_max_angle": float(max(ang_u[gated].max(), ang_v[gated].max())) if gated.any() else None}
    if fmt == "bf16":
        # 16 x 16 x 32 MFMAs per 16 rows x 32 K: 2 for b <= 8 (hi and lo share a
        # tile), else 4 per 16 columns; 2 x 16 x 16 x 32 flop each
        exec_flop = 2.0 * 16 * n * p * (2 if b <= 8 else 4 * ((b + 15) // 16))
        peak = MFMA_BF16_PEAK_TFLOPS
    elif fmt == "int8":
        tiles = 2 if b <= 8 else 3 * ((b + 15) // 16)
        exec_flop = 2.0 * 2 * 16 * tiles * n * p
        peak = MFMA_INT8_PEAK_TOPS
    else:
        # one 16-column tile (two vectors' seven limbs) per pass: code and flag
        # MFMAs of 16 x 16 x 64, 2 x 16 ops per genotype and operand
        exec_flop = 2.0 * 2 * 16 * n * p * ((b + 1) // 2)
        peak = MFMA_INT8_PEAK_TOPS
    for name, total, core, cnt in (
            ("A W", sum(i.matvec_kernel_ms for i in infos), sum(i.matvec_core_ms for i in infos),
             sum(i.timed_matvecs for i in infos)),
            ("A^T X", sum(i.rmatvec_kernel_ms for i in infos), sum(i.rmatvec_core_ms for i in infos),
             sum(i.timed_rmatvecs for i in infos))):
        avg = total / max(cnt, 1)
        avg_core = core / max(cnt, 1)
        nbytes = block_bytes(n, p, b, transpose=name == "A^T X")
        d = {"chain_avg_ms": avg, "core_kernel_avg_ms": avg_core, "launches": int(cnt),
             "algorithmic_bytes": int(nbytes),
             "chain_GBps": nbytes / (avg * 1e-3) / 1e9 if avg > 0 else None}
        if avg_core > 0:
            d["core_GBps"] = nbytes / (avg_core * 1e-3) / 1e9
            d["core_hbm_frac"] = d["core_GBps"] / HBM_PEAK_GBPS
            d["core_mfma_executed_TFLOPs"] = exec_flop / (avg_core * 1e-3) / 1e12
            d["core_mfma_frac"] = d["core_mfma_executed_TFLOPs"] / peak
        out[name] = d
    log(f"[bench] blocked {fmt} b={b}: {out['solve_s']:.3f} s, {last.steps} block steps, "
        f"max sigma err {rel.max():.2e}, gated max angle {out['gated_max_angle']}")
    return out


def run_compare(gk, torch, W, ref, args, stream):
    """FP64 at the blocked tolerance (equal accuracy) and the blocked solves."""
    import numpy as np
    out = {"fp64_tol": W.wl["tol"], "blocked_tol": BLOCKED_TOL}
    r = fp64_solve(gk, torch, W, BLOCKED_TOL, max(1, min(args.steps, 3)), 1, stream, keep=True,
                   label="fp64@1e-8")
    rel = np.abs(r["sigma"] - ref["sigma"]) / ref["sigma"]
    out["fp64_at_blocked_tol"] = {"solve_s": r["sec_per_step"], "matvecs": int(r["infos"][-1].matvecs),
                                  "restarts": int(r["infos"][-1].restarts),
                                  "sigma_max_rel_err_vs_fp64": float(rel.max())}
    rng = np.random.default_rng([7, 0x70726F])
    probe = (torch.from_numpy(rng.standard_normal((W.p, 4)) / np.sqrt(W.p)).cuda(),
             torch.from_numpy(rng.standard_normal((W.n, 4)) / np.sqrt(W.n)).cuda())
    probe_Y = ref.get("probe_Y")
    for fmt in args.formats:
        for b in args.widths:
            key = f"{fmt}_b{b}"
            res = blocked_solve(gk, torch, W, b, fmt, ref, stream, reps=args.blocked_reps,
                                probe=probe if b >= 4 else None,
                                probe_Y=probe_Y if b >= 4 else None)
            res["speedup_vs_fp64"] = ref["sec_per_step"] / (res["solve_s"] + res["create_s"])
            res["speedup_vs_fp64_at_equal_tol"] = (out["fp64_at_blocked_tol"]["solve_s"]
                                                   / (res["solve_s"] + res["create_s"]))
            out[key] = res
            torch.cuda.empty_cache()
    # the blocked path with FP64-exact products (seven int8 limbs, two columns
    # per pass) at the FP64 tolerance: the same accuracy as the headline solve
    for b in args.fp64_block_widths:
        res = blocked_solve(gk, torch, W, b, "fp64", ref, stream, reps=args.blocked_reps,
                            tol=W.wl["tol"])
        res["speedup_vs_fp64"] = ref["sec_per_step"] / (res["solve_s"] + res["create_s"])
        out[f"fp64_block_b{b}"] = res
        log(f"[bench] fp64 block b={b}: {res['solve_s']:.3f} s + {res['create_s']:.3f} s create, "
            f"sigma err {res['sigma_max_rel_err_vs_fp64']:.1e}, speedup {res['speedup_vs_fp64']:.2f}")
        torch.cuda.empty_cache()
    return out


def chromosome_blocks():
    import synth
    log("[bench] generating the 22 chromosome blocks")
    return [synth.config("c4", chrom=c) for c in range(1, 23)]


def run_loco(gk, torch, gs, args):
    """Leave-one-chromosome-out PCAs of the 22-block genome: 22 problems (the
    genome without one chromosome each), solved together with block products of
    width 22 on the matrix cores (split BF16), one pass over the genome per
    half-step for all 22."""
    import numpy as np
    import synth
    packed = np.concatenate([g.packed for g in gs], axis=0)
    starts = np.cumsum([0] + [g.p for g in gs])
    n, p = gs[0].n, int(starts[-1])
    G = torch.from_numpy(packed).cuda()
    del packed
    k, tol, m = 10, 1e-8, 40
    v0 = torch.from_numpy(np.concatenate([synth.start_vector(p, 200 + q) for q in range(22)])).cuda()
    t0 = time.perf_counter()
    ctx = gk.LocoContext(G, n, p, starts, k, tol=tol, v0=v0, krylov_dim=m,
                         precision=gk.GKL_PREC_MIXED, graph=1)
    create_s = time.perf_counter() - t0
    try:
        ctx.solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sig, Us, Vs, st, infos = ctx.solve()
        torch.cuda.synchronize()
        solve_s = time.perf_counter() - t0
    finally:
        ctx.close()
    del G, v0
    torch.cuda.empty_cache()
    log(f"[bench] loco: {solve_s:.3f} s, status {st}")
    return {"workload": "leave-one-chromosome-out: 22 problems, each the 20,000 x 701,314 genome "
                        "without one chromosome; k=10, tol 1e-8, basis 40, products as 22-column "
                        "split-BF16 block products of the whole genome",
            "problems": 22, "k": k, "tol": tol, "krylov_dim": m, "status": int(st),
            "solve_s": solve_s, "create_s": create_s,
            "converged": int(sum(i.converged for i in infos)),
            "steps": int(max(i.steps for i in infos)), "restarts": int(max(i.restarts for i in infos)),
            "passes_over_genome": int(2 * max(i.steps for i in infos)),
            "sigma_1": [float(x.cpu()[0]) for x in sig]}


def run_batched(gk, torch, gs, args):
    """22 chromosome blocks (20,000 individuals, 8,000..80,000 SNPs, 700,000 in all)
    solved together by the batched path (persistent products, one HIP graph per
    Lanczos step, autotuned product geometry), beside the same 22 problems
    solved one after another through the single-problem entry points."""
    import numpy as np
    import synth
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
        sig_b = [s.cpu().numpy() for s in sig]
    finally:
        ctx.close()
    batch_s = float(np.mean(times))
    log(f"[bench] batched: {batch_s * 1e3:.1f} ms per solve, status {st}")
    bytes_pass = sum(fp64_bytes(g.n, g.p) for g in gs)
    t0 = time.perf_counter()
    seq_mv = 0
    sig_seq = []
    for q, g in enumerate(gs):
        c1 = gk.Context(Gs[q], g.n, g.p, k, tol=tol, reorth=gk.GKL_REORTH_FULL,
                        v0=v0[sum(ps[:q]):sum(ps[:q + 1])], krylov_dim=m)
        try:
            s1, _, _, _, info = c1.solve()
            seq_mv += info.matvecs
            sig_seq.append(s1.cpu().numpy())
        finally:
            c1.close()
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t0
    agree = max(float(np.max(np.abs(a - b) / b)) for a, b in zip(sig_b, sig_seq))
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
           "speedup_vs_sequential": seq_s / batch_s,
           "sigma_max_rel_diff_batched_vs_sequential": agree}
    for name, ms in (("batched_matvec (A v, all 22)", plan["mv_ms"]),
                     ("batched_rmatvec (A^T u, all 22)", plan["rmv_ms"])):
        if ms > 0:
            out[name] = {"avg_launch_ms": ms, "algorithmic_bytes_per_launch": int(bytes_pass),
                         "achieved_GBps": bytes_pass / (ms * 1e-3) / 1e9,
                         "hbm_frac": bytes_pass / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS}
    del Gs
    torch.cuda.empty_cache()
    return out


def run_paper_model(gk, torch, args, stream):
    """The paper's own experiment matrix: its Section 2 random model at the Fig. 1
    size (41,505 individuals x 81,700 SNPs, r = 10, nsignal = n p, rkins = 0.017;
    848 MB packed), top 25 by FP64 GKL as in its Table 3 -- partial
    reorthogonalisation without restart, and full reorthogonalisation with thick
    restart -- reporting products, time, the summed residual estimates (the
    paper's ||Delta theta||_1), the error of sigma_10 against a solve to 1e-13,
    and the outliers above 1.1 sigma_+."""
    import numpy as np
    import synth
    log("[bench] paper model: generating 41,505 x 81,700")
    g = synth.algorithm1()
    n, p, k = g.n, g.p, 25
    G = torch.from_numpy(g.packed).cuda()
    v0 = torch.from_numpy(synth.start_vector(p, 3)).cuda()
    sig = torch.empty(k, dtype=torch.float64, device="cuda")
    U = torch.empty((k, n), dtype=torch.float64, device="cuda")
    V = torch.empty((k, p), dtype=torch.float64, device="cuda")
    runs = {}
    for label, reorth, tol, m in (("tight", gk.GKL_REORTH_FULL, 1e-13, 0),
                                  ("partial_no_restart", gk.GKL_REORTH_PARTIAL, 1e-10, 0),
                                  ("full_thick_restart", gk.GKL_REORTH_FULL, 1e-10, 60)):
        for rep in range(2):
            ctx = gk.Context(G, n, p, k, tol, reorth, v0=v0, krylov_dim=m, stream=stream)
            try:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, info = gk.gkl_solve(ctx.ctx, sig, U, n, V, p)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            finally:
                ctx.close()
        runs[label] = (sig.cpu().numpy().copy(), info, dt, int(st))
    s_t = runs["tight"][0]
    edge = np.sqrt(n) + np.sqrt(p)
    out = {"workload": "Section 2 model at the Fig. 1 size: 41,505 x 81,700, r=10, nsignal=n*p, "
                       "rkins=0.017, rows read as individuals; top 25, FP64",
           "packed_bytes": int(g.nbytes), "copied_rows": g.meta["copied_rows"],
           "bulk_edge_unit_variance": float(edge),
           "outliers_above_1.1_edge": int(np.sum(s_t > 1.1 * edge)),
           "outliers_above_529.7": int(np.sum(s_t > 529.7)),
           "sigma_tight": [float(x) for x in s_t]}
    for label in ("partial_no_restart", "full_thick_restart"):
        s_l, info, dt, st = runs[label]
        out[label] = {"status": st, "solve_s": dt, "mvps": int(info.matvecs),
                      "restarts": int(info.restarts),
                      "sum_residual_est": info.sum_residual_est,
                      "rel_err_sigma10_vs_tight": float(abs(s_l[9] - s_t[9]) / s_t[9])}
    del G
    torch.cuda.empty_cache()
    log(f"[bench] paper model: {out['outliers_above_1.1_edge']} outliers above 1.1 edge")
    return out


def run_extra(gk, torch, name, args, stream):
    """A second workload (FP64, blocked b = 8 and 16 in split BF16, blocked with
    FP64-exact pairs) reported beside the headline."""
    W = Workload(gk, torch, WORKLOADS[name], progress=False)
    ref = fp64_solve(gk, torch, W, W.wl["tol"], 3, 1, stream, label=f"{name} fp64")
    fmt = FORMAT_NAMES.get(int(ref["infos"][-1].fp64_products), "?")
    prod = product_stats(ref["infos"], fp64_bytes(W.n, W.p), fmt)
    out = {"workload": W.wl["desc"], "fp64_s_per_step": ref["sec_per_step"], "fp64_products": fmt,
           "fp64_matvecs": int(ref["infos"][-1].matvecs), "products": prod}
    for b in (8, 16):
        r = blocked_solve(gk, torch, W, b, "bf16", ref, stream, reps=1)
        r["speedup_vs_fp64"] = ref["sec_per_step"] / (r["solve_s"] + r["create_s"])
        out[f"bf16_b{b}"] = {key: r[key] for key in (
            "solve_s", "create_s", "block_steps", "restarts", "sigma_max_rel_err_vs_fp64",
            "gated_max_angle", "speedup_vs_fp64", "A W", "A^T X")}
    # the blocked GKL with FP64-exact limb pairs at the FP64 tolerance
    for b in args.fp64_block_widths:
        r = blocked_solve(gk, torch, W, b, "fp64", ref, stream, reps=2, tol=W.wl["tol"])
        r["speedup_vs_fp64"] = ref["sec_per_step"] / (r["solve_s"] + r["create_s"])
        out[f"fp64_block_b{b}"] = {key: r[key] for key in (
            "solve_s", "create_s", "block_steps", "restarts", "passes_over_G",
            "sigma_max_rel_err_vs_fp64", "gated_max_angle", "speedup_vs_fp64")}
        log(f"[bench] {name} fp64 block b={b}: {r['solve_s'] * 1e3:.1f} ms + "
            f"{r['create_s'] * 1e3:.1f} ms create (FP64 GKL {ref['sec_per_step'] * 1e3:.1f} ms)")
    out["reorthogonalisation"] = reorth_compare(gk, torch, W, ref, stream)
    del W
    torch.cuda.empty_cache()
    return out


def run_c5(gk, torch, args, stream):
    """100,000 x 1,000,000 (25 GB packed): a noise bulk (MAF ~ Beta(0.5, 0.5) folded,
    3% missing) with ten planted spikes at 1.5..20 times the bulk edge, k = 10.  The
    FP64 GKL (PRO, m = 30, tol 1e-10), the blocked split-BF16 solve (b = 8, tol 1e-8)
    and the blocked FP64-exact solve (b = 2, tol 1e-10), one after the other on the
    resident matrix: time, products, average product time and GB/s, per-sigma error
    against FP64, and the spikes against their planted ratios (a +-5% band: clipping
    and uneven noise make the spiked-model limit approximate)."""
    import numpy as np
    import synth
    log("[bench] c5: generating 100,000 x 1,000,000")
    g = synth.config("c5", progress=log)
    n, p, k = g.n, g.p, 10
    log("[bench] c5: copying 25 GB to the device")
    G = torch.from_numpy(g.packed).cuda()
    torch.cuda.synchronize()
    edge = float(g.meta["edge"])
    ratios = np.sort(np.array(g.meta["spike_ratios"], dtype=np.float64))[::-1]
    v0 = torch.from_numpy(synth.start_vector(p, 1)).cuda()
    sig = torch.empty(k, dtype=torch.float64, device="cuda")
    U = torch.empty((k, n), dtype=torch.float64, device="cuda")
    V = torch.empty((k, p), dtype=torch.float64, device="cuda")
    out = {"workload": "100,000 x 1,000,000 genotypes, MAF ~ Beta(0.5,0.5) folded, 3% missing, "
                       "10 planted spikes at 1.5..20x the bulk edge; k=10",
           "packed_bytes": int(g.nbytes), "bulk_edge": edge, "planted_ratios": ratios.tolist()}
    del g
    res = {}
    runs = (("fp64", 1e-10, gk.GKL_REORTH_PARTIAL, dict(krylov_dim=30)),
            ("bf16_b8", 1e-8, gk.GKL_REORTH_FULL, dict(precision=gk.GKL_PREC_MIXED, block_width=8)),
            ("fp64_block_b2", 1e-10, gk.GKL_REORTH_FULL,
             dict(precision=gk.GKL_PREC_BLOCK_FP64, block_width=2)))
    for label, tol, reorth, opts in runs:
        blocked = "precision" in opts
        t0 = time.perf_counter()
        ctx = gk.Context(G, n, p, k, tol, reorth, stream=stream, timing=1,
                         v0=None if blocked else v0, **opts)
        torch.cuda.synchronize()
        create_s = time.perf_counter() - t0
        try:
            t0 = time.perf_counter()
            st, info = gk.gkl_solve(ctx.ctx, sig, U, n, V, p)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        finally:
            ctx.close()
        torch.cuda.empty_cache()
        s = sig.cpu().numpy().copy()
        res[label] = s
        r = {"status": int(st), "solve_s": dt, "create_s": create_s, "matvecs": int(info.matvecs),
             "passes_over_G": int(info.passes_over_G), "restarts": int(info.restarts),
             "sigma_over_edge": (s / edge).tolist(),
             "sigma_vs_planted_ratio": (s / (ratios * edge) - 1.0).tolist()}
        if not blocked:
            mv = info.matvec_kernel_ms / max(info.timed_matvecs, 1)
            rmv = info.rmatvec_kernel_ms / max(info.timed_rmatvecs, 1)
            byt = fp64_bytes(n, p)
            r["avg_product_ms"] = {"A v": mv, "A^T u": rmv}
            r["product_GBps"] = {"A v": byt / (mv * 1e6), "A^T u": byt / (rmv * 1e6)}
        else:
            r["sigma_max_rel_err_vs_fp64"] = float(np.max(np.abs(s - res["fp64"]) / res["fp64"]))
            r["speedup_vs_fp64"] = out["fp64"]["solve_s"] / dt
        out[label] = r
        log(f"[bench] c5 {label}: {dt:.2f} s + {create_s:.2f} s create, {info.matvecs} products, "
            f"status {st}")
    s = res["fp64"]
    out["spikes_above_1.05_edge"] = int(np.sum(s > 1.05 * edge))
    out["near_edge_spike_recovered"] = bool(s[-1] > 1.05 * edge and abs(s[-1] / (ratios[-1] * edge) - 1) <= 0.05)
    out["all_within_5pct_band"] = bool(np.all(np.abs(s / (ratios * edge) - 1) <= 0.05))
    del G
    torch.cuda.empty_cache()
    return out


def reorth_compare(gk, torch, W, ref, stream):
    """The workload's FP64 solve with full, one-sided and partial
    reorthogonalisation, and with full reorthogonalisation and harmonic Ritz
    restarts (thick restart m = 60, tol as the workload): seconds per solve,
    restarts, Gram-Schmidt passes, products, and the sigma error against `ref`."""
    import numpy as np
    n, p, k = W.n, W.p, W.k
    out = {}
    sig = torch.empty(k, dtype=torch.float64, device="cuda")
    U = torch.empty((k, n), dtype=torch.float64, device="cuda")
    V = torch.empty((k, p), dtype=torch.float64, device="cuda")
    for label, mode, restart in (("full", gk.GKL_REORTH_FULL, gk.GKL_RESTART_RITZ),
                                 ("one_sided", gk.GKL_REORTH_ONESIDED, gk.GKL_RESTART_RITZ),
                                 ("partial", gk.GKL_REORTH_PARTIAL, gk.GKL_RESTART_RITZ),
                                 ("full_harmonic_restart", gk.GKL_REORTH_FULL,
                                  gk.GKL_RESTART_HARMONIC)):
        times = []
        for rep in range(3):
            ctx = gk.Context(W.G, n, p, k, W.wl["tol"], mode, v0=W.v0,
                             krylov_dim=W.wl["krylov_dim"], stream=stream,
                             fp64_products=FP64_PRODUCTS[0], restart=restart)
            try:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, info = gk.gkl_solve(ctx.ctx, sig, U, n, V, p)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            finally:
                ctx.close()
        s = sig.cpu().numpy()
        out[label] = {"status": int(st), "solve_s": float(np.median(times)),
                      "restarts": int(info.restarts),
                      "reorth_passes": int(info.reorths), "matvecs": int(info.matvecs),
                      "sigma_max_rel_err": float(np.max(np.abs(s - ref["sigma"]) / ref["sigma"]))}
    log(f"[bench] reorthogonalisation: {out}")
    return out


def cpu_baseline(W, ref, gpu_matvecs, ntrip):
    """The CPU oracle on the full matrix, bounded: the residual certificate of the
    leading `ntrip` GPU triplets (one A v and one A^T u per triplet).  The
    measured per-product time is scaled to the GPU solve's product count."""
    import numpy as np

    import oracle
    cores = len(os.sched_getaffinity(0))
    threads = min(int(os.environ.get("OMP_NUM_THREADS", cores)), cores)
    op = oracle.PackedOperator(W.g.packed, W.n, W.p)
    t0 = time.perf_counter()
    r1, r2, rq = oracle.certificate(op, ref["sigma"][:ntrip], ref["U"][:, :ntrip], ref["V"][:, :ntrip])
    t = time.perf_counter() - t0
    per = t / (2 * ntrip)
    s1 = ref["sigma"][0]
    res = np.maximum(r1, r2)
    cert = {"triplets": ntrip, "tol": W.wl["tol"],
            "residual_rel": [float(x) for x in res / s1],
            "max_residual_rel": float(res.max() / s1),
            "within_tol": bool(np.all(res <= W.wl["tol"] * s1)),
            "rayleigh_minus_sigma_rel": [float(x) for x in (rq - ref["sigma"][:ntrip]) / s1]}
    base = {"value": per * gpu_matvecs, "unit": "s", "cores": threads, "kind": "oracle",
            "sample": (f"oracle residual certificate of the leading {ntrip} FP64 triplets on the full "
                       f"{W.n:,} x {W.p:,} matrix: {2 * ntrip} products (A v, A^T u) in {t:.1f} s "
                       f"= {per:.2f} s per product, scaled to the GPU solve's {gpu_matvecs} products")}
    return base, cert


def product_bench(gk, torch, wl, widths, reps):
    """Per-call time and error of every product kernel chain on one workload:
    the FP64 products in each format (tables, int8 limbs) and the block products
    (split BF16 and int8 limbs at the given widths), errors against the FP64
    table products.  One JSON line; no solve."""
    import numpy as np
    W = Workload(gk, torch, wl)
    n, p = W.n, W.p
    rng = np.random.default_rng([11, 0x70726F])
    bmax = max(widths) if widths else 1
    Wv = torch.from_numpy(rng.standard_normal((p, bmax)) / np.sqrt(p)).cuda()
    Xv = torch.from_numpy(rng.standard_normal((n, bmax)) / np.sqrt(n)).cuda()
    nbytes = fp64_bytes(n, p)
    out = {"workload": wl["desc"], "reps": reps, "fp64": {}, "blocked": {}}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t0) / reps

    ref = None
    for name, choice in (("lut", gk.GKL_FP64_LUT), ("limbs", gk.GKL_FP64_LIMBS)):
        ctx = gk.Context(W.G, n, p, 1, fp64_products=choice)
        try:
            y, ty = timed(lambda: ctx.matvec(Wv[:, 0].contiguous()))
            z, tz = timed(lambda: ctx.rmatvec(Xv[:, 0].contiguous()))
            if ref is None:
                ref = (y, z)
            out["fp64"][name] = {
                "A v ms": ty * 1e3, "A v GBps": nbytes / ty / 1e9,
                "A^T u ms": tz * 1e3, "A^T u GBps": nbytes / tz / 1e9,
                "A v rel diff vs lut": float(torch.linalg.norm(y - ref[0]) / torch.linalg.norm(ref[0])),
                "A^T u rel diff vs lut": float(torch.linalg.norm(z - ref[1]) / torch.linalg.norm(ref[1]))}
        finally:
            ctx.close()
        log(f"[bench] product bench fp64 {name}: {out['fp64'][name]}")
    if widths:
        f64 = gk.Context(W.G, n, p, 1, fp64_products=gk.GKL_FP64_LUT)
        try:
            Y0 = torch.stack([f64.matvec(Wv[:, c].contiguous()) for c in range(bmax)], 1)
            Z0 = torch.stack([f64.rmatvec(Xv[:, c].contiguous()) for c in range(bmax)], 1)
        finally:
            f64.close()
        for fmt, prec in (("bf16", gk.GKL_PREC_MIXED), ("int8", gk.GKL_PREC_MIXED_INT8)):
            ctx = gk.Context(W.G, n, p, 1, precision=prec, block_width=8, krylov_dim=32)
            try:
                for b in widths:
                    y, ty = timed(lambda: ctx.matmat_mixed(Wv[:, :b]))
                    z, tz = timed(lambda: ctx.rmatmat_mixed(Xv[:, :b]))
                    out["blocked"][f"{fmt}_b{b}"] = {
                        "A W ms": ty * 1e3, "A W GBps": block_bytes(n, p, b) / ty / 1e9,
                        "A^T X ms": tz * 1e3, "A^T X GBps": block_bytes(n, p, b, True) / tz / 1e9,
                        "A W rel err": float(torch.linalg.norm(y - Y0[:, :b]) / torch.linalg.norm(Y0[:, :b])),
                        "A^T X rel err": float(torch.linalg.norm(z - Z0[:, :b]) / torch.linalg.norm(Z0[:, :b]))}
                    log(f"[bench] product bench {fmt} b={b}: {out['blocked'][f'{fmt}_b{b}']}")
            finally:
                ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp64-products", default="auto", choices=["auto", "lut", "limbs", "lut+limbs"],
                    help="product format of the FP64 solves (lookup tables or int8 limbs)")
    ap.add_argument("--certificate-triplets", type=int, default=5,
                    help="leading triplets checked by the CPU oracle (2 products each)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the blocked solves and the FP64 solve at the blocked tolerance")
    ap.add_argument("--widths", default="8,16,32", help="block widths of the blocked solves")
    ap.add_argument("--fp64-block-widths", default="2",
                    help="block widths of the blocked solves with FP64-exact products, at the FP64 "
                         "tolerance ('' for none)")
    ap.add_argument("--formats", default="bf16",
                    help="blocked product formats: bf16 (split BF16), int8 (int8 limbs)")
    ap.add_argument("--blocked-reps", type=int, default=1)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 10,000 x 100,000 workload reported beside the headline")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched solve of the 22 chromosome blocks")
    ap.add_argument("--batched-steps", type=int, default=2)
    ap.add_argument("--c5", action="store_true",
                    help="also solve the 100,000 x 1,000,000 spiked workload (25 GB) by the FP64 "
                         "and both blocked paths (adds a few minutes)")
    ap.add_argument("--no-loco", action="store_true",
                    help="skip the leave-one-chromosome-out solve of the 22-block genome")
    ap.add_argument("--product-bench", default=None, metavar="WIDTHS",
                    help="only time the product kernels (FP64 formats, and block products at "
                         "these comma-separated widths, '' for none) on the workload; prints "
                         "one JSON line")
    ap.add_argument("--product-reps", type=int, default=10)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="after the timed steps, copy BYTES bytes device-to-device 3 times "
                         "(reference dispatch for the HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only; the library has no multi-GPU path, so --gpus "
              "must be 1", file=sys.stderr)
        sys.exit(2)
    FP64_PRODUCTS[:] = [{"auto": 0, "lut": 1, "limbs": 2, "lut+limbs": 3}[args.fp64_products],
                        args.fp64_products]
    args.widths = [int(x) for x in args.widths.split(",") if x]
    args.formats = [x for x in args.formats.split(",") if x]
    args.fp64_block_widths = [int(x) for x in args.fp64_block_widths.split(",") if x]

    import numpy as np
    import torch

    import paper_1808_03374_amd as gk

    stream = torch.cuda.current_stream().cuda_stream
    if args.product_bench is not None:
        widths = [int(x) for x in args.product_bench.split(",") if x]
        res = product_bench(gk, torch, WORKLOADS[args.workload], widths, args.product_reps)
        if args.copy_calibration > 0:
            src = torch.empty(args.copy_calibration, dtype=torch.uint8, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            res["copy_calibration_bytes"] = args.copy_calibration
        print(json.dumps(res), flush=True)
        reap_children()
        return
    wl = WORKLOADS[args.workload]
    W = Workload(gk, torch, wl)
    n, p, k = W.n, W.p, W.k
    rng = np.random.default_rng([7, 0x70726F])
    probe = (torch.from_numpy(rng.standard_normal((p, 4)) / np.sqrt(p)).cuda(),
             torch.from_numpy(rng.standard_normal((n, 4)) / np.sqrt(n)).cuda())
    ref = fp64_solve(gk, torch, W, wl["tol"], args.steps, args.warmup, stream,
                     probe=None if args.no_compare else probe)
    infos = ref["infos"]
    sec_per_step = ref["sec_per_step"]
    nbytes = fp64_bytes(n, p)
    last = infos[-1]
    products = FORMAT_NAMES.get(int(last.fp64_products), "?")
    prod = product_stats(infos, nbytes, products)
    dom = max(prod, key=lambda key: prod[key]["total_ms"])
    other = [key for key in prod if key != dom][0]
    dom_avg = prod[dom]["avg_ms"]
    achieved = nbytes / (dom_avg * 1e-3) / 1e9
    # the read rate this GPU reaches in practice: a plain streaming read of the
    # same packed matrix (the product kernels stream it once per product)
    read_ms = gk.gkl_read_rate(W.G, reps=5, stream=stream)
    read_gbps = W.G.numel() / (read_ms * 1e-3) / 1e9
    log(f"[bench] plain streaming read of the packed matrix: {read_ms:.3f} ms, {read_gbps:.0f} GB/s")
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
                   "reorth": wl["reorth"], "krylov_dim": wl["krylov_dim"], "fp64_products": products,
                   "packed_bytes": int(W.g.nbytes)},
        "solve_s": float(np.mean([i.solve_ms for i in infos])) / 1e3,
        "create_s": float(np.mean([i.create_ms for i in infos])) / 1e3,
        "matvecs": int(last.matvecs),
        "restarts": int(last.restarts),
        "reorth_passes": int(last.reorths),
        "converged": int(last.converged),
        "max_residual_rel": last.max_residual_rel,
        "matvec_GBps": prod[KERNEL_NAMES[products][0]]["GBps"],
        "rmatvec_GBps": prod[KERNEL_NAMES[products][1]]["GBps"],
        "roofline": {
            "kernel": dom,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": measured_traffic(wl["name"], dom),
            "avg_launch_ms": dom_avg,
            "launches": int(prod[dom]["launches"]),
            "timed_one_launch_in": TIMING_STRIDE,
            "algorithmic_bytes_per_launch": int(nbytes),
            "read_ceiling_GBps": read_gbps,
            "frac_of_read_ceiling": achieved / read_gbps,
            "other_kernel": {"kernel": other, "avg_launch_ms": prod[other]["avg_ms"],
                             "achieved_GBps": prod[other]["GBps"],
                             "traffic": measured_traffic(wl["name"], other)},
        },
    }
    if args.copy_calibration > 0:
        src = torch.empty(args.copy_calibration, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        line["copy_calibration_bytes"] = args.copy_calibration
    if not args.no_compare:
        line["compare"] = run_compare(gk, torch, W, ref, args, stream)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle (residual certificate on the full matrix)")
        line["cpu_baseline"], line["certificate"] = cpu_baseline(
            W, ref, int(last.matvecs), min(args.certificate_triplets, k))
        log(f"[bench] certificate: max residual {line['certificate']['max_residual_rel']:.2e} sigma_1")
    W.G = None
    torch.cuda.empty_cache()
    if not args.no_extra and args.workload != "c2":
        line["c2"] = run_extra(gk, torch, "c2", args, stream)
    if not args.no_extra:
        line["paper_model"] = run_paper_model(gk, torch, args, stream)
    if args.c5:
        line["c5"] = run_c5(gk, torch, args, stream)
    if not (args.no_batched and args.no_loco):
        gs = chromosome_blocks()
        if not args.no_batched:
            line["batched"] = run_batched(gk, torch, gs, args)
        if not args.no_loco:
            line["loco"] = run_loco(gk, torch, gs, args)
        del gs
    torch.cuda.synchronize()
    print(json.dumps(line), flush=True)
    reap_children()


def reap_children():
    """End any child process this run left behind (named on stderr), so the
    bench exits with nothing of its own still running."""
    try:
        import psutil
    except ImportError:
        return
    kids = psutil.Process().children(recursive=True)
    for c in kids:
        try:
            log(f"[bench] ending leftover child process {c.pid}: {' '.join(c.cmdline())[:200]}")
            c.terminate()
        except psutil.Error:
            pass
    psutil.wait_procs(kids, timeout=5)


if __name__ == "__main__":
    main()
