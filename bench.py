#!/usr/bin/env python3
"""Throughput of the quaternion pseudoinverse hot path on one MI355X.

Workload (one "step" = one complete solve, every step of the method on the GPU):
  A = U diag(s) V^H, 2048 x 1536 quaternion of rank 1024, s geometric from 1 to 1e-4, orthonormal
  factors from Gaussian matrices, rounded to FP32 (synthetic, seeded); QHPI19 (Algorithm 3) in FP32
  products with FP32 accumulation, alpha = 1/sigma_1^2 estimated by 8 power steps, guarded stop rule
  at tol 1e-6, residual on the smaller side (1536).  The input is resident in HBM before timing.

Prints one JSON line: solves/s (`value`), the product kernels' TFLOP/s against the FP32 MFMA peak
(`roofline`, from HIP events around every product launch in the timed steps), the FP64 CPU oracle's
rate on a bounded sample (`cpu_baseline`), and standalone square-product TFLOP/s.
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
    names = {q.GEMM_PREC[k]: k for k in ("f64", "f32", "bf16")}
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
    # growth with n (the paper's scalability figure plots CPU time and E1..E4 against n without printing
    # the values): square Gaussian stand-ins, same settings, one timed solve after a warm-up
    sweep = {}
    for n in (500, 1000, 2000, 3000):
        Ad = torch.from_numpy(qsynth.gaussian(9200 + n, n, n)).cuda()
        for method in ("qhpi19", "qsai"):
            kw = dict(method=method, scaling="frob", tol=1e-10, max_iter=500, stop="dx_abs", precision="f64")
            q.solve(ctx, Ad, **kw)
            torch.cuda.synchronize()
            t = time.perf_counter()
            X, info = q.solve(ctx, Ad, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            Ea, Er = q.residuals(ctx, Ad, X)
            flops = 7 * 32.0 * n ** 3 * info["iters"] if method == "qhpi19" else None
            sweep[f"{n}:{method}"] = {"ms": 1e3 * dt, "iters": info["iters"], "E_rel": Er,
                                      "tflops": flops / dt / 1e12 if flops else None}
        del Ad
    out["growth_with_n"] = sweep
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


def section_cur(q, ctx, torch):
    import qsynth

    # CUR image completion of Section 5.1 on a synthetic 512 x 768 colour image (70% of pixels
    # missing, rank-60 factors, 25 impute-reconstruct iterations), every step on the GPU
    def psnr_db(X, ref):  # over the three colour planes, peak 1
        return float(10.0 * np.log10(1.0 / np.mean((X[1:] - ref[1:]) ** 2)))

    d = qsynth.cur_image_instance()
    res = {"masked_psnr_db": psnr_db(d["image"] * d["mask"][None], d["image"])}
    mask_d = torch.from_numpy(d["mask"]).cuda()
    rows_d = torch.from_numpy(d["rows"]).cuda()
    cols_d = torch.from_numpy(d["cols"]).cuda()
    for prec in ("f32", "f64"):
        Md = torch.from_numpy(d["image"]).to(torch.float32 if prec == "f32" else torch.float64).cuda()
        for meth in ("qhpi19", "qsai"):
            kw = dict(iters=25, method=meth, tol=1e-6 if prec == "f32" else 1e-12)
            q.cur_complete(ctx, Md, mask_d, rows_d, cols_d, **kw)
            torch.cuda.synchronize()
            t = time.perf_counter()
            X = q.cur_complete(ctx, Md, mask_d, rows_d, cols_d, **kw)
            torch.cuda.synchronize()
            dt_s = time.perf_counter() - t
            res[f"{meth}_{prec}"] = {"total_ms": 1e3 * dt_s, "ms_per_iteration": 1e3 * dt_s / 25,
                                     "psnr_db": psnr_db(X.double().cpu().numpy(), d["image"])}
    return {"workload": "synthetic 512x768 pure-quaternion colour image (40 smooth separable terms + N(0, 0.02^2) "
                        "texture), 70% of pixels missing, rank-60 row/column sets, 25 impute-reconstruct iterations, "
                        "U = C^+ A R^+", "results": res}


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


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--method", default="qhpi19", choices=["ns", "qsai", "qhpi19", "qrapid"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gemm", action="store_true", help="skip the standalone square-product measurement")
    ap.add_argument("--no-autotune", action="store_true", help="use the heuristic tile choice instead of tuning")
    ap.add_argument("--no-mixed", action="store_true", help="skip the 4096^2 mixed-vs-plain precision comparison")
    ap.add_argument("--mixed-steps", type=int, default=2)
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-matrix batched comparison")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-scaling evaluation")
    ap.add_argument("--learned-count", type=int, default=256)
    ap.add_argument("--no-methods", action="store_true", help="skip the other methods on the 2048x1536 input")
    ap.add_argument("--no-small", action="store_true", help="skip the 64x48 FP64 latency section")
    ap.add_argument("--no-lorenz", action="store_true", help="skip the Lorenz filter-design section")
    ap.add_argument("--no-cur", action="store_true", help="skip the CUR image-completion section")
    ap.add_argument("--no-krylov", action="store_true", help="skip the preconditioned Krylov section")
    ap.add_argument("--no-paper-tables", action="store_true",
                    help="skip the FP64 solves of the paper's own table workloads")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU (the library has no multi-GPU path); --gpus must be 1"}))
        return 2

    import torch

    import paper_2605_01464_amd as q
    import qsynth

    t_gen = time.time()
    inst = qsynth.c2_instance()
    t_gen = time.time() - t_gen
    A_host = inst["A"]
    m, n = A_host.shape[1], A_host.shape[2]
    A = torch.from_numpy(A_host.astype(np.float32)).cuda()
    X = torch.empty((4, n, m), dtype=torch.float32, device="cuda")
    order = {"ns": 2, "qsai": 10, "qhpi19": 19, "qrapid": 5}[args.method]

    ctx = q.Context(0)
    if not args.no_autotune:
        ctx.set("autotune", 1)  # tile configurations are timed on the solve's own shapes during warm-up
    solve_kw = dict(method=args.method, order=order, scaling="power", tol=1e-6, max_iter=100, stop="guarded",
                    precision="f32", X=X)
    for _ in range(max(args.warmup, 1 if not args.no_autotune else 0)):
        q.solve(ctx, A, **solve_kw)
    torch.cuda.synchronize()
    ctx.set("gemm_timing", 1)
    q.qpinv_gemm_stats(ctx.handle)  # reset
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, info = q.solve(ctx, A, **solve_kw)
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    _, rows = q.qpinv_gemm_stats(ctx.handle)
    ctx.set("gemm_timing", 0)
    ms_per_step = 1e3 * elapsed / args.steps
    value = args.steps / elapsed
    # dominant kernel: the (precision, tile configuration) with the most product time
    dom = max(rows, key=lambda r: r["ms"])
    prec_name = {0: "f64", 1: "f32", 2: "bf16"}[dom["prec"]]
    achieved = dom["flops"] / (dom["ms"] * 1e-3) / 1e12
    dom_name = q.qpinv_tile_config_name(dom["prec"], dom["cfg"])
    gemm_ms = sum(r["ms"] for r in rows)
    info = infos[-1]

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pinv/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"rank-1024 quaternion pseudoinverse 2048x1536 (s geometric 1..1e-4, FP32 input), "
                               f"{args.method.upper()} FP32, power-iteration alpha, guarded stop tol 1e-6",
                   "m": m, "n": n, "rank": 1024, "method": args.method, "precision": "f32"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK[prec_name], "unit": "TFLOP/s",
                     "frac": achieved / PEAK[prec_name], "traffic": measured_traffic(dom_name),
                     "traffic_unit": "bytes/launch",
                     "kernel": f"qgemm_kernel {dom_name}",
                     "launches_per_step": dom["launches"] / args.steps,
                     "flops_per_launch": dom["flops"] / max(dom["launches"], 1),
                     "avg_launch_ms": dom["ms"] / max(dom["launches"], 1),
                     "all_kernels": [{"kernel": q.qpinv_tile_config_name(r["prec"], r["cfg"]),
                                      "launches_per_step": r["launches"] / args.steps,
                                      "avg_launch_ms": r["ms"] / r["launches"],
                                      "tflops": r["flops"] / (r["ms"] * 1e-3) / 1e12} for r in rows]},
        "solve": {"iters": info["iters"], "returned": info["returned"], "reason": info["reason"],
                  "side": info["side"], "alpha": info["alpha_used"], "gemm_flops": info["gemm_flops"],
                  "gemm_ms_share": (gemm_ms / args.steps) / ms_per_step},
        "input_generation_s": t_gen,
    }

    XL = None
    if not args.no_learned:
        # the learned initial scaling on the same workload, reported beside the plain method's value
        from paper_2605_01464_amd import learned as L

        L.load(ctx)
        XL = torch.empty_like(X)
        lkw = dict(solve_kw, scaling="learned", X=XL)
        q.solve(ctx, A, **lkw)  # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            _, linfo = q.solve(ctx, A, **lkw)
        torch.cuda.synchronize()
        dtl = (time.perf_counter() - t) / args.steps
        _, er_plain = q.residuals(ctx, A, X)
        _, er_learned = q.residuals(ctx, A, XL)
        out["learned_alpha_same_workload"] = {
            "pinv_per_s": 1.0 / dtl, "iters": linfo["iters"], "mu": linfo["mu_used"],
            "fallback_used": linfo["fallback_used"], "plain_pinv_per_s": value, "plain_iters": info["iters"],
            "E_rel_plain": er_plain, "E_rel_learned": er_learned}

    if not args.no_gemm:
        # standalone quaternion products: square sizes and the solver's own shapes, per precision
        out["qgemm_square"] = {}
        for nn in (1024, 2048, 4096, 8192):
            out["qgemm_square"][f"f32_n{nn}"] = qgemm_rate(q, ctx, nn, nn, nn, reps=10 if nn == 8192 else 20)
        for prec in ("f64", "bf16"):
            out["qgemm_square"][f"{prec}_n4096"] = qgemm_rate(q, ctx, 4096, 4096, 4096, prec=prec, reps=10)
        out["qgemm_solver_shapes"] = {
            f"f32_{M_}x{N_}x{K_}": qgemm_rate(q, ctx, M_, N_, K_)
            for M_, N_, K_ in ((1536, 1536, 2048), (1536, 1536, 1536), (1536, 2048, 1536))}
        ctx.set("autotune", 0 if args.no_autotune else 1)

    if not args.no_methods:
        # the same 2048 x 1536 workload with the other methods (FP32, guarded stop), and the factorized
        # order-19 update against the plain hyperpower polynomial of order 19 at equal update counts
        res = {}
        Xm = torch.empty_like(X)  # the headline solve's result in X stays untouched
        for meth in ("ns", "qsai", "qrapid", "qhpi19"):
            kw = dict(method=meth, scaling="power", tol=1e-6, max_iter=200, stop="guarded", precision="f32", X=Xm)
            q.solve(ctx, A, **kw)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, inf_m = q.solve(ctx, A, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            res[meth] = {"pinv_per_s": 1.0 / dt, "ms": 1e3 * dt, "iters": inf_m["iters"], "returned": inf_m["returned"],
                         "reason": inf_m["reason"], "gemm_tflop": inf_m["gemm_flops"] / 1e12}
        fixed = {}
        for key_, meth, order_ in (("qhpi19", "qhpi19", 19), ("hpi19", "hpi", 19)):
            kw = dict(method=meth, order=order_, scaling="power", tol=0.0, max_iter=4, stop="dx_abs",
                      precision="f32", X=Xm, check=False)
            q.solve(ctx, A, **kw)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, inf_m = q.solve(ctx, A, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            fixed[key_] = {"ms_per_4_updates": 1e3 * dt, "gemm_tflop": inf_m["gemm_flops"] / 1e12}
        fixed["time_ratio_unfactorized_over_factorized"] = (fixed["hpi19"]["ms_per_4_updates"] /
                                                            fixed["qhpi19"]["ms_per_4_updates"])
        out["methods_2048x1536"] = {"guarded_tol_1e-6": res, "order19_factorized_vs_horner_4_updates": fixed}

    if not args.no_small:
        # 64 x 48 FP64 (planes N(0,1), seeds 0..9): latency of one solve to ||AXA - A||_F / ||A||_F <= 1e-12
        res = {}
        smalls = [torch.from_numpy(qsynth.c1_instance(seed)).cuda() for seed in range(10)]
        for meth in ("ns", "qsai", "qhpi19", "qrapid"):
            kw = dict(method=meth, scaling="power", tol=1e-12, max_iter=200, stop="e1_rel", precision="f64")
            for a in smalls:
                q.solve(ctx, a, **kw)
            torch.cuda.synchronize()
            times, its = [], []
            for rep in range(5):
                for a in smalls:
                    t = time.perf_counter()
                    _, inf_s = q.solve(ctx, a, **kw)
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t)
                    its.append(inf_s["iters"])
            res[meth] = {"us_median": 1e6 * float(np.median(times)), "pinv_per_s": 1.0 / float(np.median(times)),
                         "iters_mean": float(np.mean(its))}
        out["small_fp64_64x48"] = res

    mixed_inst = None
    if not args.no_mixed:
        # 4096 x 4096, condition 1e3, geometric spectrum, components of unit variance: solves/s of
        # the precision ladder vs the plain forms, each reaching relative error <= 1e-6 (FP64 finish)
        t_g = time.time()
        mixed_inst = qsynth.c3_instance()
        t_g = time.time() - t_g
        A3 = torch.from_numpy(mixed_inst["A"].astype(np.float32)).cuda()
        A3d = A3.double()
        X3 = torch.empty((4, A3.shape[2], A3.shape[1]), dtype=torch.float64, device="cuda")
        res = {}
        # default FP64 finish: Newton-Schulz updates with FP64 residual and sum around an FP32 product;
        # "allfp64": every finish product in FP64; "samefinish": the solve's own method, all in FP64
        # (the default ladder runs last, so X3 holds its QHPI19 result for the sampled-row check below)
        for label, prec, Ain, refined, finish in (("plain_f32_f64finish", "f32_f64finish", A3, 1, 0),
                                                  ("plain_f64", "f64", A3d, 1, 0),
                                                  ("mixed_bf16_f32_f64allfp64", "mixed", A3, 0, 0),
                                                  ("mixed_bf16_f32_f64samefinish", "mixed", A3, 0, -1),
                                                  ("mixed_bf16_f32_f64", "mixed", A3, 1, 0)):
            ctx.set("f64_refined", refined)
            ctx.set("finish_method", finish)
            for method in (("qhpi19",) if label.endswith(("allfp64", "samefinish")) else ("qrapid", "qhpi19")):
                kw = dict(method=method, order=None, scaling="power", tol=1e-6, max_iter=100, stop="guarded",
                          precision=prec, X=X3)
                q.solve(ctx, Ain, **kw)  # warm-up (and tile tuning)
                torch.cuda.synchronize()
                t = time.perf_counter()
                for _ in range(args.mixed_steps):
                    _, inf3 = q.solve(ctx, Ain, **kw)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t) / args.mixed_steps
                Ea, Er = q.residuals(ctx, A3, X3)
                res[f"{label}:{method}"] = {"pinv_per_s": 1.0 / dt, "ms": 1e3 * dt, "iters_bf16": inf3["iters_bf16"],
                                            "iters_f32": inf3["iters_f32"], "iters_f64": inf3["iters_f64"],
                                            "E_rel_fp64": Er}
                if label.startswith("mixed"):
                    res[f"{label}:{method}"].update(ladder_breakdown(q, ctx, torch, Ain, kw))
        ctx.set("f64_refined", 1)
        ctx.set("finish_method", 0)
        if XL is not None:
            # the ladder started from the learned scaling (the network was loaded with the headline's comparison)
            X3L = torch.empty_like(X3)
            kw = dict(method="qhpi19", order=None, scaling="learned", tol=1e-6, max_iter=100, stop="guarded",
                      precision="mixed", X=X3L)
            q.solve(ctx, A3, **kw)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.mixed_steps):
                _, inf3 = q.solve(ctx, A3, **kw)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / args.mixed_steps
            Ea, Er = q.residuals(ctx, A3, X3L)
            res["mixed_bf16_f32_f64_learned:qhpi19"] = {
                "pinv_per_s": 1.0 / dt, "ms": 1e3 * dt, "iters_bf16": inf3["iters_bf16"], "iters_f32": inf3["iters_f32"],
                "iters_f64": inf3["iters_f64"], "mu": inf3["mu_used"], "E_rel_fp64": Er}
            del X3L
        out["mixed_vs_plain"] = {"workload": "4096x4096 quaternion, cond 1e3, geometric spectrum, unit-variance "
                                             "components (FP32 input), guarded stop tol 1e-6",
                                 "input_generation_s": t_g, "results": res}

    if not args.no_batched:
        # 512 quaternion matrices, rows and cols uniform in [32, 256], planes N(0,1), cond <= 1e3:
        # one persistent launch (graph replay) vs a loop of single-matrix solves over the same batch
        t_g = time.time()
        sizes = qsynth.c4_sizes()
        As4 = [torch.from_numpy(qsynth.c4_instance(b, sizes).astype(np.float32)).cuda() for b in range(len(sizes))]
        t_g = time.time() - t_g
        Xs4 = [torch.empty((4, a.shape[2], a.shape[1]), dtype=torch.float32, device="cuda") for a in As4]
        reps = 3
        per_cfg = {}
        for cfg in range(q.qpinv_num_batched_configs()):  # every kernel form and tile shape
            ctx.set("batched_cfg", cfg)
            q.solve_batched(ctx, As4, "qhpi19", tol=1e-6, stop="guarded", Xs=Xs4)  # graph build
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                q.solve_batched(ctx, As4, "qhpi19", tol=1e-6, stop="guarded", Xs=Xs4)
            torch.cuda.synchronize()
            per_cfg[q.qpinv_batched_config_name(cfg)] = len(As4) * reps / (time.perf_counter() - t)
        ctx.set("batched_cfg", -1)
        q.solve_batched(ctx, As4, "qhpi19", tol=1e-6, stop="guarded", Xs=Xs4)  # autotuned choice + graph build
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            _, inf4 = q.solve_batched(ctx, As4, "qhpi19", tol=1e-6, stop="guarded", Xs=Xs4)
        torch.cuda.synchronize()
        t_batch = (time.perf_counter() - t) / reps
        # the loop uses the heuristic tile choice (tuning each of the 512 shapes would be timed otherwise)
        ctx.set("autotune", 0)
        for a, x in zip(As4[:8], Xs4[:8]):  # warm-up
            q.solve(ctx, a, "qhpi19", tol=1e-6, stop="guarded", precision="f32", X=x)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for a, x in zip(As4, Xs4):
            q.solve(ctx, a, "qhpi19", tol=1e-6, stop="guarded", precision="f32", X=x)
        torch.cuda.synchronize()
        t_loop = time.perf_counter() - t
        ctx.set("autotune", 0 if args.no_autotune else 1)
        its = [i["iters"] for i in inf4]
        s_ = [min(a.shape[1], a.shape[2]) for a in As4]
        o_ = [max(a.shape[1], a.shape[2]) for a in As4]
        flops = sum(7 * 32.0 * si * si * oi * it for si, oi, it in zip(s_, o_, its))
        out["batched"] = {"workload": "512 quaternion matrices, rows/cols uniform in [32,256], N(0,1) planes, "
                                      "cond <= 1e3, QHPI19 FP32, guarded stop tol 1e-6",
                          "persistent_solves_per_s": len(As4) / t_batch, "batch_ms": 1e3 * t_batch,
                          "loop_single_solves_per_s": len(As4) / t_loop, "loop_ms": 1e3 * t_loop,
                          "speedup_vs_loop": t_loop / t_batch, "iters_median": float(np.median(its)),
                          "gemm_tflops_effective": flops / t_batch / 1e12, "input_generation_s": t_g,
                          "solves_per_s_by_config": per_cfg}

    if not args.no_learned:
        # learned initial scaling (network trained on the GPU by this library on 20k matrices 64..512):
        # FP64 QHPI19 to ||AXA - A||_F / ||A||_F <= 1e-10 on held-out 1024 x 768 matrices
        from paper_2605_01464_amd import learned as L

        meta = L.load(ctx)
        t_g = time.time()
        ev = L.build_set(ctx, range(2_000_000, 2_000_000 + args.learned_count), shape=(1024, 768), keep=True)
        t_g = time.time() - t_g
        res, _ = L.evaluate(ctx, ev["mats"], ev)
        res["workload"] = (f"{args.learned_count} held-out 1024x768 quaternion matrices (geometric / clustered / "
                           "low-rank+noise spectra), QHPI19 FP64, tol 1e-10 on E1_rel")
        res["gain_iters_vs_classical"] = res["classical"]["mean_iters"] - res["learned"]["mean_iters"]
        res["headroom_iters_vs_classical"] = res["classical"]["mean_iters"] - res["best"]["mean_iters"]
        res["train_meta"] = meta
        res["input_and_feature_s"] = t_g
        out["learned_scaling"] = res
        del ev

    if not args.no_lorenz:
        out["lorenz_filtering"] = section_lorenz(q, ctx, torch)
    if not args.no_cur:
        out["cur_completion"] = section_cur(q, ctx, torch)
    if not args.no_krylov:
        out["krylov_preconditioning"] = section_krylov(q, ctx, torch)
    if not args.no_paper_tables:
        out["paper_table_workloads"] = section_paper_tables(q, ctx, torch)

    if not args.no_cpu_baseline:
        # FP64 oracle on the host: one iteration of the same method on the same input (left side),
        # scaled by the GPU solve's iteration count -> solves/s.  Bounded sample of the workload.
        from oracle import methods as M
        from oracle import quat as Q

        try:
            from threadpoolctl import threadpool_info

            cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
        except Exception:
            cores = os.cpu_count()
        X0 = M.x0(A_host, 1.0 / max(info["sigma1_sq_est"], 1e-300))
        t = time.perf_counter()
        M.step(A_host, X0, args.method, order, "left")
        t_it = time.perf_counter() - t
        its = max(info["iters"], 1)
        out["cpu_baseline"] = {"value": 1.0 / (t_it * its), "unit": "pinv/s", "cores": cores, "kind": "oracle",
                               "sample": f"one FP64 {args.method.upper()} iteration (left side) of the oracle on the "
                                         f"same 2048x1536 input ({t_it:.2f} s), scaled by the GPU solve's "
                                         f"{its} iterations"}
        Xd = X.detach().cpu().double().numpy()
        Xc = Q.pinv_from_factors(inst["U"], inst["s"], inst["V"])
        out["rel_err_vs_rank1024_pinv"] = float(np.linalg.norm(Xd - Xc) / np.linalg.norm(Xc))
        if XL is not None:
            XLd = XL.detach().cpu().double().numpy()
            out["learned_alpha_same_workload"]["rel_err_vs_rank1024_pinv"] = float(
                np.linalg.norm(XLd - Xc) / np.linalg.norm(Xc))
        if mixed_inst is not None:
            # sampled rows of the default ladder's QHPI19 result (the mixed section's last) vs the exact inverse of
            # the FP32 input: relative residual of rows of A X - I, times the condition number
            A3h = mixed_inst["A"]
            X3h = X3.detach().cpu().numpy()
            rows = np.random.default_rng(5).choice(A3h.shape[1], 8, replace=False)
            AXr = Q.qmul(A3h[:, rows, :], X3h)
            AXr[0, np.arange(8), rows] -= 1.0
            out["mixed_vs_plain"]["row_residual_bound_last"] = float(
                np.linalg.norm(AXr) / np.sqrt(8) * mixed_inst["s"][0] / mixed_inst["s"][-1])

    ctx.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
