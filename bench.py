#!/usr/bin/env python3
"""Throughput of the quaternion pseudoinverse hot path on one MI355X.

Workload of the headline (one "step" = one complete solve, every step of the method on the GPU):
  A = c U diag(s) V^H, 4096 x 4096 quaternion, s geometric from 1 to 1e-3 (condition 1e3), components of unit
  variance, dense structured unitary factors, rounded to FP32 (synthetic, seeded); QHPI19 (Algorithm 3) with every
  product in FP64 (the paper's arithmetic), alpha = 1/sigma_1^2 estimated by 8 power steps, guarded stop rule at
  tol 1e-6.  The input is resident in HBM before timing.  Beside it, on the same input: the BF16 -> FP32 -> FP64
  precision ladder ("mixed"), FP32 iterations with an FP64 finish ("plain"), the ladder from the learned initial
  scaling, QRAPID(5) in each form, and standalone quaternion-product TFLOP/s.  Every result's relative Frobenius
  error is taken against the FP64 oracle's inverse of the same FP32-rounded input.

The LAST stdout line is one compact JSON object (value, roofline of the dominant FP64 product kernel from HIP
events around every product launch, cpu_baseline).  `--sections` adds secondary measurements, each printed as
its own JSON line before the last one.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f32": 157.3, "bf16": 2500.0, "f64": 78.6}  # TFLOP/s, dense MFMA, MI355X datasheet
PEAK["bf16x3"] = PEAK["bf16"] / 3  # three BF16 products per product: the BF16 peak in product flops
METRIC = "pinv solves/s + quaternion GEMM TFLOP/s at rel-err<=1e-6; mixed/learned vs plain"


def hamilton_rows(A, B):
    """Rows of the quaternion product A B in FP64 (A: 4 x r x K planes, B: 4 x K x N); a direct transcription
    of the Hamilton product used only to report the products' sampled error."""
    a, b = [A[i].astype(np.float64) for i in range(4)], [B[i].astype(np.float64) for i in range(4)]
    return np.stack([a[0] @ b[0] - a[1] @ b[1] - a[2] @ b[2] - a[3] @ b[3],
                     a[0] @ b[1] + a[1] @ b[0] + a[2] @ b[3] - a[3] @ b[2],
                     a[0] @ b[2] - a[1] @ b[3] + a[2] @ b[0] + a[3] @ b[1],
                     a[0] @ b[3] + a[1] @ b[2] - a[2] @ b[1] + a[3] @ b[0]])


def qgemm_rate(q, ctx, M, N, K, prec="f32", reps=20, check_rows=16):
    """Median TFLOP/s over `reps` timed launches of C = A B (planes N(0,1), seed 400, tuned tiles) and the
    relative Frobenius error of `check_rows` sampled rows against the FP64 product of the same inputs."""
    import torch

    dt = torch.float64 if prec == "f64" else torch.float32
    g = torch.Generator(device="cuda").manual_seed(400)
    A = torch.randn((4, M, K), device="cuda", dtype=dt, generator=g)
    B = torch.randn((4, K, N), device="cuda", dtype=dt, generator=g)
    C = torch.empty((4, M, N), device="cuda", dtype=dt)
    ctx.set("autotune", 1)
    q.qgemm(ctx, A, B, C, gemm_prec=prec)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record(s)
        q.qgemm(ctx, A, B, C, gemm_prec=prec)
        e1.record(s)
    torch.cuda.synchronize()
    ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
    rows = np.random.default_rng(7).choice(M, min(check_rows, M), replace=False)
    Ah, Bh = A[:, rows, :].double().cpu().numpy(), B.double().cpu().numpy()
    if prec == "bf16":  # the kernel multiplies the BF16-rounded operands
        Ah = A[:, rows, :].bfloat16().double().cpu().numpy()
        Bh = B.bfloat16().double().cpu().numpy()
    ref = hamilton_rows(Ah, Bh)
    got = C[:, rows, :].double().cpu().numpy()
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    del A, B, C
    torch.cuda.empty_cache()
    return {"tflops": 32.0 * M * N * K / (ms * 1e-3) / 1e12, "ms_median": ms, "reps": reps,
            "frac_peak": 32.0 * M * N * K / (ms * 1e-3) / 1e12 / PEAK[prec], "rel_err_sampled_rows": err}


KERNEL_SOURCES = ("common.hpp", "qgemm.hpp", "qgemm_kern.hpp", "qgemm.hip")


def measured_traffic(config_name):
    """HBM bytes per launch of the product kernel `config_name`, from the FETCH_SIZE / WRITE_SIZE counter
    summaries under profiles/ (copy-kernel calibrated).  None unless the product kernel sources still hash to
    the value recorded with the counters, i.e. the kernel has not changed since they were taken."""
    import glob
    import hashlib
    import re

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2605_01464_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    digest = h.hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_hbm_traffic.md"))):
        with open(path) as fh:
            m = re.search(r"```json\n(.*?)\n```", fh.read(), re.S)
        if not m:
            continue
        rec = json.loads(m.group(1))
        if rec.get("config") == config_name and rec.get("kernel_sources_sha256") == digest:
            return rec["traffic_bytes_per_launch"]
    return None


def ladder_breakdown(q, ctx, torch, A, kw):
    """One more (untimed) solve with every product bracketed by HIP events on its stream: product time
    and rate per precision (BF16 including its operand copies); the rest of the solve is norms, power
    steps, stop rules and copies between precisions."""
    ctx.set("gemm_timing", 1)
    q.qpinv_gemm_stats(ctx.handle)  # reset
    torch.cuda.synchronize()
    t = time.perf_counter()
    q.solve(ctx, A, **kw)
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t
    _, rows = q.qpinv_gemm_stats(ctx.handle)
    ctx.set("gemm_timing", 0)
    names = {v: k for k, v in q.GEMM_PREC.items()}
    byp = {}
    for r in rows:
        e = byp.setdefault(names[r["prec"]], {"launches": 0, "ms": 0.0, "flops": 0.0})
        e["launches"] += r["launches"]
        e["ms"] += r["ms"]
        e["flops"] += r["flops"]
    for e in byp.values():
        e["tflops"] = e["flops"] / (e["ms"] * 1e-3) / 1e12 if e["ms"] > 0 else None
    return {"products_by_precision": byp, "one_solve_ms_with_events": 1e3 * t_one,
            "non_product_ms": 1e3 * t_one - sum(e["ms"] for e in byp.values())}


# The paper's own timing workloads (Tables 1-2 and Example 3: MATLAB, FP64, Intel i9-12900K): seconds and
# iteration counts as printed, quoted beside this library's FP64 GPU solves of synthetic stand-ins of the
# same shape (the paper's inputs are unseeded).
PAPER_TABLES = [
    # (workload, m, n, kind, {method: (paper seconds, paper iterations)})
    ("300x300 Gaussian", 300, 300, "gaussian",
     {"qsai": (0.7308, 11), "qrapid": (1.217, 7), "qhpi19": (0.7797, 9), "ns": (2.433, 81)}),
    ("1500x1500 Gaussian", 1500, 1500, "gaussian",
     {"qsai": (37.19, 13), "qrapid": (84.78, 8), "qhpi19": (45.02, 11), "ns": (125.6, 92)}),
    ("1000x500 overdetermined", 1000, 500, "gaussian",
     {"qsai": (4.408, 7), "qrapid": (8.293, 5), "qhpi19": (5.657, 6), "ns": (7.044, 60)}),
    ("500x1000 underdetermined", 500, 1000, "gaussian",
     {"qsai": (1.844, 7), "qrapid": (4.089, 5), "qhpi19": (1.752, 6), "ns": (7.126, 60)}),
    ("1000x1000 rank-deficient (rank 500)", 1000, 1000, "rank500",
     {"qsai": (8.789, 10), "qrapid": (16.78, 6), "qhpi19": (8.570, 8), "ns": (32.73, 73)}),
    ("800x800 Gaussian (Example 3)", 800, 800, "gaussian",
     {"qhpi19": (6.188, 8), "qsai": (6.594, 10), "hpi:19": (13.87, 8), "hpi:10": (11.05, 10)}),
]


def section_paper_tables(q, ctx, torch, reps=3):
    """FP64 solves with the paper's stopping test ||X_{j+1} - X_j||_F < 1e-10 and alpha = 1/||A||_F^2
    (Tables 1-2; Example 3: 1/sigma_1^2 by power iteration, the paper's alpha being 1/sigma_1^2 of its
    own matrix); QRAPID with N = 5.  Inputs: planes iid N(0,1); the rank-deficient matrix is the product
    of 1000 x 500 and 500 x 1000 Gaussian matrices (the paper does not give its construction).  Example 3
    also times the unfactorized order-19 and order-10 iterations ("hpi:19", "hpi:10")."""
    import qsynth

    out = {"settings": "FP64 on the GPU; stop ||X_{j+1}-X_j||_F < 1e-10, max 500 updates; alpha = 1/||A||_F^2 "
                       "(Example 3: 1/sigma_1^2); QRAPID N = 5; the paper's seconds are MATLAB FP64 on an Intel "
                       "i9-12900K (other hardware and software: context only)", "results": {}}
    for wi, (name, m, n, kind, methods) in enumerate(PAPER_TABLES):
        A = qsynth.gaussian(9000 + wi, m, n) if kind == "gaussian" else qsynth.low_rank_gaussian(9000 + wi, m, n, 500)
        Ad = torch.from_numpy(A).cuda()
        scaling = "power" if "Example 3" in name else "frob"
        for key, (t_paper, it_paper) in methods.items():
            # "hpi:p": the unfactorized hyperpower iteration of order p (Horner, p products per update)
            method, order = (key.split(":")[0], int(key.split(":")[1])) if ":" in key else (key, None)
            kw = dict(method=method, order=5 if method == "qrapid" else order, scaling=scaling, tol=1e-10,
                      max_iter=500, stop="dx_abs", precision="f64")
            X, info = q.solve(ctx, Ad, **kw)  # warm-up (and tile tuning)
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t = time.perf_counter()
                X, info = q.solve(ctx, Ad, **kw)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
            dt = float(np.median(ts))
            Ea, Er = q.residuals(ctx, Ad, X)
            out["results"][f"{name}:{key}"] = {
                "ms": 1e3 * dt, "pinv_per_s": 1.0 / dt, "iters": info["iters"], "E1_abs": Ea[0], "E1_rel": Er[0],
                "status": info["status"], "paper_s": t_paper, "paper_iters": it_paper, "speedup_vs_paper": t_paper / dt}
        del Ad
    return out


def section_lorenz(q, ctx, torch):
    import qsynth

    # filter design of Section 5.2 on the delayed noisy Lorenz record [0, 40] (tau = 1, noise std 1):
    # square Toeplitz systems of 401..2001 unknowns, FP64 pseudoinverse + both products on the GPU
    res = {}
    for dt in qsynth.LORENZ_STEPS:
        d = qsynth.lorenz_filter_instance(dt)
        Xd = torch.from_numpy(d["X"]).cuda()
        sd = torch.from_numpy(d["s"]).cuda()
        row = {"n": int(d["p"] + 1)}
        for meth in ("qsai", "qhpi19"):
            q.filter_design(ctx, Xd, sd, method=meth)
            torch.cuda.synchronize()
            times = []
            for _ in range(3):
                t = time.perf_counter()
                h, s_hat, inf_f = q.filter_design(ctx, Xd, sd, method=meth)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t)
            eps = float(torch.linalg.vector_norm(s_hat - sd) / torch.linalg.vector_norm(sd))
            row[meth] = {"ms": 1e3 * float(np.median(times)), "iters": inf_f["iters"], "eps": eps}
        res[f"dt_{dt}"] = row
        del Xd, sd
    return {"workload": "Lorenz (sigma 10, delta 8/3, gamma 28, x0 [1,1,1]) on [0,40], delay 1, imaginary noise "
                        "N(0,1), (p+1)x(p+1) Toeplitz X, h = X^+ s, FP64, guarded stop tol 1e-13", "results": res}


def section_krylov(q, ctx, torch):
    import qsynth

    # Example 4: global quaternion FOM / GMRES on A X = B (n = 238 stand-in operator, m = 3..12 right-hand
    # sides), plain and left-preconditioned by 4 QSAI updates; RR <= 1e-6; preconditioned times include
    # building M
    res = {}
    for m_rhs in (3, 6, 9, 12):
        d = qsynth.krylov_instance(m_rhs)
        Ad = torch.from_numpy(d["A"]).cuda()
        Bd = torch.from_numpy(d["B"]).cuda()
        row = {}
        for name, meth, pre in (("gl_qfom", "fom", False), ("gl_qgmres", "gmres", False),
                                ("pre_gl_qfom", "fom", True), ("pre_gl_qgmres", "gmres", True)):
            for rep in range(2):  # first pass warms the workspaces
                torch.cuda.synchronize()
                t = time.perf_counter()
                Md = None
                if pre:
                    Md, _ = q.solve(ctx, Ad, "qsai", tol=0.0, max_iter=4, stop="dx_abs", precision="f64")
                _, inf_k = q.gl_krylov(ctx, Ad, Bd, method=meth, M=Md, tol=1e-6, max_iter=3000)
                torch.cuda.synchronize()
                dt_s = time.perf_counter() - t
            row[name] = {"iters": inf_k["iters"], "ms": 1e3 * dt_s, "rr": inf_k["true_rr"],
                         "status": inf_k["status"]}
        res[f"m_{m_rhs}"] = row
    return {"workload": "A = A_s (1 - i + 2j + 1.5k), A_s a 238x238 nonsymmetric five-point operator (log-normal "
                        "transmissibilities, skew part), B uniform [0,1), X_0 = 0, RR <= 1e-6, QSAI preconditioner of "
                        "4 updates, FP64", "results": res}




def _r(x, d=4):
    """Round to `d` significant digits for the compact line."""
    if x is None:
        return None
    if isinstance(x, (list, tuple)):
        return [_r(v, d) for v in x]
    x = float(x)
    return float(f"{x:.{d}g}") if np.isfinite(x) else x


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info

        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count()
    return model, cores


def timed_solves(q, ctx, torch, A, kw, steps, warmup, stats=False):
    """`warmup` untimed solves, then `steps` timed ones (synchronised on both sides).  With `stats`, every product
    launch of the timed solves is bracketed by HIP events on the solve's stream (per tile configuration)."""
    for _ in range(warmup):
        q.solve(ctx, A, **kw)
    torch.cuda.synchronize()
    if stats:
        ctx.set("gemm_timing", 1)
        q.qpinv_gemm_stats(ctx.handle)  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, info = q.solve(ctx, A, **kw)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    rows = None
    if stats:
        _, rows = q.qpinv_gemm_stats(ctx.handle)
        ctx.set("gemm_timing", 0)
    return elapsed, info, rows


def section_c2(q, ctx, torch, steps=5, warmup=2):
    """2048 x 1536 of rank 1024 (s geometric 1..1e-4, FP32 input): every method in FP32 with the guarded stop at tol
    1e-6, the FP32 + FP64-finish form, and the finish followed by X <- X A X (Penrose condition 2)."""
    import qsynth

    inst = qsynth.c2_instance()
    A = torch.from_numpy(inst["A"].astype(np.float32)).cuda()
    X = torch.empty((4, A.shape[2], A.shape[1]), dtype=torch.float32, device="cuda")
    res = {}
    for meth in ("qhpi19", "ns", "qsai", "qrapid"):
        kw = dict(method=meth, scaling="power", tol=1e-6, max_iter=200, stop="guarded", precision="f32", X=X)
        el, info, _ = timed_solves(q, ctx, torch, A, kw, steps, warmup)
        _, Er = q.residuals(ctx, A, X)
        res[meth] = {"pinv_per_s": steps / el, "iters": info["iters"], "returned": info["returned"],
                     "reason": info["reason"], "gemm_tflop": info["gemm_flops"] / 1e12, "E_rel_fp64": Er}
    # FP32 QHPI19, FP64 Newton-Schulz finish, then no projection / X A X / (X A)^H X (A X)^H (option penrose_finish)
    X64 = torch.empty((4, A.shape[2], A.shape[1]), dtype=torch.float64, device="cuda")
    for mode, label in ((0, "f32_f64finish"), (1, "f32_f64finish_xax"), (2, "f32_f64finish_projection")):
        ctx.set("penrose_finish", mode)
        kw = dict(method="qhpi19", scaling="power", tol=1e-6, max_iter=200, stop="guarded", precision="f32_f64finish",
                  X=X64)
        el, info, _ = timed_solves(q, ctx, torch, A, kw, steps, warmup)
        _, Er = q.residuals(ctx, A, X64)
        res[label] = {"pinv_per_s": steps / el, "iters_f32": info["iters_f32"], "iters_f64": info["iters_f64"],
                      "E_rel_fp64": Er}
    ctx.set("penrose_finish", 0)
    return {"section": "c2_2048x1536_rank1024", "results": res}


def section_small(q, ctx, torch):
    """64 x 48 FP64 (planes N(0,1), seeds 0..9): latency of one solve to ||AXA - A||_F / ||A||_F <= 1e-12, the
    caller's output X allocated once and the stream passed, as a serving loop would."""
    import qsynth

    res = {}
    smalls = [torch.from_numpy(qsynth.c1_instance(seed)).cuda() for seed in range(10)]
    outs = [torch.empty((4, a.shape[2], a.shape[1]), dtype=a.dtype, device=a.device) for a in smalls]
    stream = torch.cuda.current_stream()
    for meth in ("ns", "qsai", "qhpi19", "qrapid"):
        kw = dict(method=meth, scaling="power", tol=1e-12, max_iter=200, stop="e1_rel", precision="f64",
                  stream=stream)
        for a, x in zip(smalls, outs):
            q.solve(ctx, a, X=x, **kw)
        torch.cuda.synchronize()
        times, its = [], []
        for rep in range(5):
            for a, x in zip(smalls, outs):
                t = time.perf_counter()
                _, inf_s = q.solve(ctx, a, X=x, **kw)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t)
                its.append(inf_s["iters"])
        res[meth] = {"us_median": 1e6 * float(np.median(times)), "iters_mean": float(np.mean(its))}
    return {"section": "small_fp64_64x48", "results": res}


def section_batched(q, ctx, torch, all_configs=False):
    """512 quaternion matrices, rows and cols uniform in [32, 256], planes N(0,1), cond <= 1e3: one persistent
    launch (graph replay) vs a loop of single-matrix solves over the same batch."""
    import qsynth

    sizes = qsynth.c4_sizes()
    As4 = [torch.from_numpy(qsynth.c4_instance(b, sizes).astype(np.float32)).cuda() for b in range(len(sizes))]
    Xs4 = [torch.empty((4, a.shape[2], a.shape[1]), dtype=torch.float32, device="cuda") for a in As4]
    args = q.BatchArgs(As4, Xs4)  # descriptors marshalled once, as a caller solving batch after batch does
    reps = 3
    per_cfg = {}
    if all_configs:
        for cfg in range(q.qpinv_num_batched_configs()):
            ctx.set("batched_cfg", cfg)
            q.solve_batched(ctx, args, "qhpi19", tol=1e-6, stop="guarded")
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                q.solve_batched(ctx, args, "qhpi19", tol=1e-6, stop="guarded")
            torch.cuda.synchronize()
            per_cfg[q.qpinv_batched_config_name(cfg)] = len(As4) * reps / (time.perf_counter() - t)
        ctx.set("batched_cfg", -1)
    q.solve_batched(ctx, args, "qhpi19", tol=1e-6, stop="guarded")
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        _, inf4 = q.solve_batched(ctx, args, "qhpi19", tol=1e-6, stop="guarded")
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t) / reps
    t = time.perf_counter()
    for _ in range(reps):  # the same solves with the tensor lists marshalled on every call
        q.solve_batched(ctx, As4, "qhpi19", tol=1e-6, stop="guarded", Xs=Xs4)
    torch.cuda.synchronize()
    t_lists = (time.perf_counter() - t) / reps
    ctx.set("autotune", 0)
    for a, x in zip(As4[:8], Xs4[:8]):
        q.solve(ctx, a, "qhpi19", tol=1e-6, stop="guarded", precision="f32", X=x)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for a, x in zip(As4, Xs4):
        q.solve(ctx, a, "qhpi19", tol=1e-6, stop="guarded", precision="f32", X=x)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t
    ctx.set("autotune", 1)
    its = [i["iters"] for i in inf4]
    s_ = [min(a.shape[1], a.shape[2]) for a in As4]
    o_ = [max(a.shape[1], a.shape[2]) for a in As4]
    flops = sum(7 * 32.0 * si * si * oi * it for si, oi, it in zip(s_, o_, its))
    return {"section": "batched_512", "persistent_solves_per_s": len(As4) / t_batch, "batch_ms": 1e3 * t_batch,
            "list_args_solves_per_s": len(As4) / t_lists,
            "loop_single_solves_per_s": len(As4) / t_loop, "speedup_vs_loop": t_loop / t_batch,
            "iters_median": float(np.median(its)), "gemm_tflops_effective": flops / t_batch / 1e12,
            "solves_per_s_by_config": per_cfg}


def section_learned(q, ctx, torch, count=256):
    """Learned initial scaling on held-out 1024 x 768 matrices, FP64 QHPI19 to E1_rel <= 1e-10."""
    from paper_2605_01464_amd import learned as L

    meta = L.load(ctx)
    ev = L.build_set(ctx, range(2_000_000, 2_000_000 + count), shape=(1024, 768), keep=True)
    res, _ = L.evaluate(ctx, ev["mats"], ev)
    res["gain_iters_vs_classical"] = res["classical"]["mean_iters"] - res["learned"]["mean_iters"]
    res["headroom_iters_vs_classical"] = res["classical"]["mean_iters"] - res["best"]["mean_iters"]
    res["train_meta"] = meta
    return {"section": "learned_scaling_1024x768", "results": res}


SECTIONS = ("c2", "small", "batched", "batched_all", "learned", "lorenz", "krylov", "paper_tables", "gemm_all")


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--side-steps", type=int, default=2, help="timed solves of each comparison form")
    ap.add_argument("--no-oracle", action="store_true",
                    help="skip the CPU oracle leg (the FP64 reference for the errors and cpu_baseline)")
    ap.add_argument("--no-forms", action="store_true", help="skip the ladder / plain / learned / QRAPID forms")
    ap.add_argument("--no-gemm", action="store_true", help="skip the standalone product rates")
    ap.add_argument("--sections", default="", help="comma list of secondary sections: " + ", ".join(SECTIONS))
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU: the library has no multi-GPU path, so --gpus must be 1 "
                                   "(a batch of independent solves would be dealt across GPUs with no exchange)"}))
        return 2
    sections = [s for s in args.sections.split(",") if s]
    for s in sections:
        if s not in SECTIONS:
            ap.error(f"unknown section {s!r}")

    import torch

    import paper_2605_01464_amd as q
    import qsynth

    t_gen = time.time()
    inst = qsynth.c3_instance()
    t_gen = time.time() - t_gen
    A_host = inst["A"]                                   # FP32-rounded values, held in float64
    A32 = torch.from_numpy(A_host.astype(np.float32)).cuda()
    A64 = A32.double()
    n = A_host.shape[1]
    ctx = q.Context(0)
    # the headline's FP64 products take the library's measured default tiles (no timing-dependent choice)
    ctx.set("autotune", 0)

    # ---------------------------------------------------------------- headline: all-FP64 QHPI19
    X64 = torch.empty((4, n, n), dtype=torch.float64, device="cuda")
    kw = dict(method="qhpi19", scaling="power", tol=1e-6, max_iter=100, stop="guarded", precision="f64", X=X64)
    elapsed, info, rows = timed_solves(q, ctx, torch, A64, kw, args.steps, max(args.warmup, 1), stats=True)
    value = args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    dom = max(rows, key=lambda r: r["ms"])
    prec_name = {0: "f64", 1: "f32", 2: "bf16", 3: "bf16x3"}[dom["prec"]]
    dom_name = q.qpinv_tile_config_name(dom["prec"], dom["cfg"])
    launches = max(dom["launches"], 1)
    achieved = dom["flops"] / (dom["ms"] * 1e-3) / 1e12
    gemm_ms = sum(r["ms"] for r in rows)
    results = {"f64:qhpi19": X64}
    forms = {"f64:qhpi19": {"pinv_per_s": value, "iters": f"{info['iters_f64']}"}}

    # ---------------------------------------------------------------- the other forms on the same input
    ctx.set("autotune", 1)  # tile configurations are timed on each form's own shapes during its warm-up
    if not args.no_forms:
        from paper_2605_01464_amd import learned as L

        L.load(ctx)
        for label, prec, Ain, method, scaling in (("mixed:qhpi19", "mixed", A32, "qhpi19", "power"),
                                                  ("mixed:qrapid", "mixed", A32, "qrapid", "power"),
                                                  ("mixed_learned:qhpi19", "mixed", A32, "qhpi19", "learned"),
                                                  ("plain_f32_f64finish:qhpi19", "f32_f64finish", A32, "qhpi19", "power"),
                                                  ("plain_f32_f64finish:qrapid", "f32_f64finish", A32, "qrapid", "power"),
                                                  ("f64:qrapid", "f64", A64, "qrapid", "power")):
            Xf = torch.empty((4, n, n), dtype=torch.float64, device="cuda")
            fkw = dict(method=method, scaling=scaling, tol=1e-6, max_iter=100, stop="guarded", precision=prec, X=Xf)
            steps_f = 1 if label == "f64:qrapid" else args.side_steps
            el, inf_f, _ = timed_solves(q, ctx, torch, Ain, fkw, steps_f, 1)
            phases = ("iters_f64",) if prec == "f64" else ("iters_bf16", "iters_f32", "iters_f64")
            forms[label] = {"pinv_per_s": steps_f / el,
                            "iters": "+".join(str(inf_f[k]) for k in phases if inf_f[k] or prec == "f64")}
            if scaling == "learned":
                forms[label]["mu"] = inf_f["mu_used"]
            results[label] = Xf
            if label == "mixed:qhpi19":  # where the ladder's time goes, as an earlier line
                rec = ladder_breakdown(q, ctx, torch, Ain, fkw)
                print(json.dumps({"section": "ladder_breakdown_4096", **rec}, default=float), flush=True)

    # ---------------------------------------------------------------- standalone product rates
    gemm = {}
    if not args.no_gemm:
        for nn in (2048, 4096):
            r = qgemm_rate(q, ctx, nn, nn, nn, reps=10)
            gemm[f"f32_n{nn}"] = {"tflops": r["tflops"], "frac": r["frac_peak"], "rel_err": r["rel_err_sampled_rows"]}
        for prec in ("f64", "bf16", "bf16x3"):
            r = qgemm_rate(q, ctx, 4096, 4096, 4096, prec=prec, reps=10)
            gemm[f"{prec}_n4096"] = {"tflops": r["tflops"], "frac": r["frac_peak"],
                                     "rel_err": r["rel_err_sampled_rows"]}

    # ---------------------------------------------------------------- secondary sections (earlier lines)
    for s in sections:
        if s == "c2":
            rec = section_c2(q, ctx, torch)
        elif s == "small":
            rec = section_small(q, ctx, torch)
        elif s in ("batched", "batched_all"):
            rec = section_batched(q, ctx, torch, all_configs=(s == "batched_all"))
        elif s == "learned":
            rec = section_learned(q, ctx, torch)
        elif s == "lorenz":
            rec = dict(section="lorenz_filtering", **section_lorenz(q, ctx, torch))
        elif s == "krylov":
            rec = dict(section="krylov_preconditioning", **section_krylov(q, ctx, torch))
        elif s == "paper_tables":
            rec = dict(section="paper_table_workloads", **section_paper_tables(q, ctx, torch))
        else:
            rec = {"section": "qgemm_rates", "results": {
                f"{p}_{M_}x{N_}x{K_}": qgemm_rate(q, ctx, M_, N_, K_, prec=p, reps=10)
                for p, (M_, N_, K_) in [("f32", (1024,) * 3), ("f32", (8192,) * 3), ("f32", (1536, 1536, 2048)),
                                        ("f32", (1536, 1536, 1536)), ("f32", (1536, 2048, 1536)),
                                        ("bf16", (2048,) * 3), ("f64", (2048,) * 3)]}}
        print(json.dumps(rec), flush=True)

    # ---------------------------------------------------------------- CPU oracle leg
    cpu = None
    if not args.no_oracle:
        from oracle import methods as M
        from oracle import quat as Q

        model, cores = cpu_info()
        t = time.perf_counter()
        Xref = Q.inverse_square(A_host)                 # A^{-1} = A^dagger of the square FP32-rounded input
        t_closed = time.perf_counter() - t
        nref = float(np.linalg.norm(Xref))
        for label, Xd in results.items():
            forms[label]["rel_err"] = float(np.linalg.norm(Xd.cpu().numpy() - Xref) / nref)
        X0 = M.x0(A_host, 1.0 / info["sigma1_sq_est"])
        t = time.perf_counter()
        M.step(A_host, X0, "qhpi19", None, "left")
        t_it = time.perf_counter() - t
        its = max(info["iters"], 1)
        cpu = {"value": 1.0 / (t_it * its), "unit": "pinv/s", "cores": cores, "kind": "oracle",
               "cpu_model": model,
               "sample": f"one FP64 QHPI19 update of the oracle on the same 4096x4096 input ({t_it:.1f} s), scaled by "
                         f"the GPU solve's {its} updates; the oracle's direct inverse (LU of the complex adjoint) "
                         f"took {t_closed:.1f} s"}

    ctx.close()
    for rec in forms.values():
        for k in ("pinv_per_s", "rel_err", "mu"):
            if k in rec:
                rec[k] = _r(rec[k])
    out = {
        "metric": METRIC,
        "value": _r(value, 5),
        "unit": "pinv/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(args.warmup, 1),
        "ms_per_step": _r(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "4096x4096 quaternion pseudoinverse, cond 1e3 (geometric spectrum), unit-variance "
                               "components, FP32-rounded input; QHPI19 all-FP64, power-iteration alpha, guarded stop "
                               "tol 1e-6", "m": n, "n": n, "method": "qhpi19", "precision": "f64"},
        "rel_err_vs_oracle": forms["f64:qhpi19"].get("rel_err"),
        "roofline": {"bound": "mfma", "achieved": _r(achieved), "peak": PEAK[prec_name], "unit": "TFLOP/s",
                     "frac": _r(achieved / PEAK[prec_name]), "traffic": measured_traffic(dom_name),
                     "kernel": dom_name, "launches_per_step": _r(launches / args.steps),
                     "flops_per_launch": _r(dom["flops"] / launches), "avg_launch_ms": _r(dom["ms"] / launches),
                     "product_share_of_step": _r((gemm_ms / args.steps) / ms_per_step)},
        "forms": forms,
        "qgemm": {k: {kk: _r(vv) for kk, vv in v.items()} for k, v in gemm.items()},
        "cpu_baseline": cpu,
        "input_generation_s": _r(t_gen, 3),
    }
    if out["roofline"]["traffic"] is not None:
        out["roofline"]["traffic"] = _r(out["roofline"]["traffic"])
        out["roofline"]["traffic_unit"] = "bytes/launch"
    if cpu is not None:
        cpu["value"] = _r(cpu["value"])
    line = json.dumps(out, separators=(",", ":"))
    print(line, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
