"""Learned initial scaling: build a labelled set, train the scaling network, save/load it, evaluate it.

Orchestration only.  Matrices come from the seeded generator (qsynth); their scaling features, the
labels (iteration-count-minimising alpha from each matrix's spectrum), the network's forward and
backward passes, Adam and inference all run in libqpinv's kernels.

    python -m paper_2605_01464_amd.learned train --count 20000 --out paper_2605_01464_amd/scaling_net.json
    python -m paper_2605_01464_amd.learned eval --net paper_2605_01464_amd/scaling_net.json --count 256

Label definition: for method M and tolerance tol, J(alpha) is the number of updates until
||A X A - A||_F <= tol ||A||_F in exact arithmetic (evaluated from the spectrum); the label is the
point nearest mu = 1.8 of the longest run of a 64-point geometric grid mu in [0.05, 1.95]
(alpha = mu/s_1^2) that attains min J, expressed relative to the power-iteration estimate:
target = log(alpha* s1sq_est).  (For the order-19 method the runs reach the top of the admissible
interval; their midpoints would bias the regression below the narrow runs' lower ends.)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_NET = os.path.join(HERE, "scaling_net.json")
GRID = dict(ngrid=64, mu_lo=0.05, mu_hi=1.95, mu_target=1.8)


def _pool_init():
    import qsynth

    qsynth.DCT_WORKERS = 1


def _gen(args):
    import qsynth

    seed, size_range, shape = args
    d = qsynth.c5_sample(seed, size_range=size_range, shape=shape)
    return d["A"], d["s"], d["family"]


def generate(seeds, size_range=(64, 512), shape=None, workers=None):
    """Matrices for `seeds` (CPU, in a process pool); yields (A, s, family)."""
    workers = workers or min(16, os.cpu_count() or 1)
    jobs = [(int(sd), size_range, shape) for sd in seeds]
    if workers <= 1 or len(jobs) < 4:
        for j in jobs:
            yield _gen(j)
        return
    with ProcessPoolExecutor(max_workers=workers, initializer=_pool_init) as ex:
        for out in ex.map(_gen, jobs, chunksize=8):
            yield out


def build_set(ctx, seeds, method="qhpi19", order=None, tol=1e-10, size_range=(64, 512), shape=None, keep=False,
              workers=None):
    """Features (GPU), spectra and labels (GPU) for the matrices of `seeds`."""
    import torch

    import paper_2605_01464_amd as q

    raw, spectra, offsets, fams, mats = [], [], [0], [], []
    for A, s, fam in generate(seeds, size_range, shape, workers):
        Ad = torch.from_numpy(A).cuda()
        f = q.features(ctx, Ad)
        raw.append(q.raw_features(f))
        spectra.append(s)
        offsets.append(offsets[-1] + len(s))
        fams.append(fam)
        if keep:
            mats.append(Ad)
    dev = "cuda"
    raw_d = torch.tensor(raw, dtype=torch.float64, device=dev)
    spec_d = torch.from_numpy(np.concatenate(spectra)).to(dev)
    off_d = torch.tensor(offsets, dtype=torch.int32, device=dev)
    s1 = raw_d[:, 0].contiguous()
    n = len(raw)
    mu = torch.empty(n, dtype=torch.float64, device=dev)
    jb = torch.empty(n, dtype=torch.int32, device=dev)
    jc = torch.empty(n, dtype=torch.int32, device=dev)
    meth = q.METHOD[method]
    st = q.qpinv_spectral_labels(ctx.handle, meth, q._order(method, order), spec_d, off_d, s1, tol, 64, GRID["ngrid"],
                                 GRID["mu_lo"], GRID["mu_hi"], GRID["mu_target"], mu, jb, jc)
    q._err(st, "qpinv_spectral_labels")
    return {"raw": raw_d, "target": torch.log(mu), "mu": mu, "j_best": jb, "j_classical": jc, "family": fams,
            "spectra": spectra, "mats": mats}


def train(ctx, data, epochs=60, batch=256, lr=2e-3, seed=1, verbose=False):
    """Fit the normalisation, then Adam over shuffled minibatches (GPU kernels).  Returns per-epoch loss."""
    import torch

    import paper_2605_01464_amd as q

    q._err(q.qpinv_mlp_init(ctx.handle, seed), "qpinv_mlp_init")
    q._err(q.qpinv_mlp_fit_normalization(ctx.handle, data["raw"]), "qpinv_mlp_fit_normalization")
    n = data["raw"].shape[0]
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n).astype(np.int32)).cuda()
        lr_ep = lr * 0.5 * (1 + math.cos(math.pi * ep / epochs))  # cosine schedule
        tot, cnt = 0.0, 0
        for b0 in range(0, n, batch):
            idx = perm[b0:b0 + batch]
            st, loss = q.qpinv_mlp_train_step(ctx.handle, data["raw"], data["target"], idx, idx.shape[0], lr_ep)
            q._err(st, "qpinv_mlp_train_step")
            tot += loss * idx.shape[0]
            cnt += idx.shape[0]
        hist.append(tot / cnt)
        if verbose:
            print(f"epoch {ep} loss {hist[-1]:.4e}", flush=True)
    return hist


def predict_mu(ctx, raw):
    import torch

    import paper_2605_01464_amd as q

    mu = torch.empty(raw.shape[0], dtype=torch.float64, device=raw.device)
    q._err(q.qpinv_mlp_predict(ctx.handle, raw, mu), "qpinv_mlp_predict")
    return mu


def save(ctx, path, meta=None):
    import paper_2605_01464_amd as q

    st, vals = q.qpinv_mlp_get_params(ctx.handle)
    q._err(st, "qpinv_mlp_get_params")
    arr = np.asarray(vals, dtype=np.float32)
    doc = {"format": "qpinv-scaling-net-1", "layers": [10, 64, 64, 1], "activation": "tanh",
           "output": "log(alpha * sigma1_est^2)", "values": [float(v) for v in arr],
           "sha256": hashlib.sha256(arr.tobytes()).hexdigest(), "meta": meta or {}}
    with open(path, "w") as f:
        json.dump(doc, f)


def load(ctx, path=DEFAULT_NET):
    import paper_2605_01464_amd as q

    with open(path) as f:
        doc = json.load(f)
    arr = np.asarray(doc["values"], dtype=np.float32)
    if hashlib.sha256(arr.tobytes()).hexdigest() != doc["sha256"]:
        raise ValueError(f"{path}: checksum mismatch")
    q._err(q.qpinv_mlp_set_params(ctx.handle, list(arr)), "qpinv_mlp_set_params")
    return doc.get("meta", {})


def evaluate(ctx, mats, data, method="qhpi19", tol=1e-10, max_iter=60, reps=2):
    """FP64 solves of every matrix with the learned, classical (1/sigma1_est^2), Frobenius (1/||A||_F^2)
    and spectrum-best alpha, arms interleaved per matrix; iteration counts and times per arm (each time the
    fastest of `reps` solves, so that a host stall in one solve does not weigh on its arm's mean)."""
    import torch

    import paper_2605_01464_amd as q

    arms = {"learned": [], "classical": [], "frobenius": [], "best": []}
    times = {k: [] for k in arms}
    fallback = 0
    s1 = data["raw"][:, 0].cpu().numpy()
    mu_best = data["mu"].cpu().numpy()
    for i, A in enumerate(mats):
        for arm in arms:
            if arm == "learned":
                kw = dict(scaling="learned")
            elif arm == "classical":
                kw = dict(scaling="power")
            elif arm == "frobenius":
                kw = dict(scaling="frob")
            else:
                kw = dict(scaling="given", alpha=float(mu_best[i] / s1[i]))
            best_t = None
            for _ in range(reps):
                torch.cuda.synchronize()
                t = time.perf_counter()
                _, info = q.solve(ctx, A, method, scaling=kw["scaling"], alpha=kw.get("alpha", 0.0), tol=tol,
                                  max_iter=max_iter, stop="e1_rel", precision="f64", check=False)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t
                best_t = dt if best_t is None else min(best_t, dt)
            times[arm].append(best_t)
            arms[arm].append(info["iters"])
            if arm == "learned":
                fallback += info["fallback_used"]
    out = {k: {"mean_iters": float(np.mean(v)), "median_iters": float(np.median(v)),
               "mean_ms": 1e3 * float(np.mean(times[k]))} for k, v in arms.items()}
    out["learned_fallbacks"] = int(fallback)
    out["count"] = len(mats)
    return out, arms


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--count", type=int, default=20000)
    t.add_argument("--seed0", type=int, default=1_000_000)
    t.add_argument("--epochs", type=int, default=60)
    t.add_argument("--out", default=DEFAULT_NET)
    e = sub.add_parser("eval")
    e.add_argument("--net", default=DEFAULT_NET)
    e.add_argument("--count", type=int, default=256)
    e.add_argument("--seed0", type=int, default=2_000_000)
    args = ap.parse_args(argv)

    sys.path.insert(0, os.path.dirname(HERE))
    import paper_2605_01464_amd as q

    with q.Context(0) as ctx:
        if args.cmd == "train":
            t0 = time.time()
            data = build_set(ctx, range(args.seed0, args.seed0 + args.count))
            t1 = time.time()
            hist = train(ctx, data, epochs=args.epochs, verbose=True)
            t2 = time.time()
            jb = data["j_best"].cpu().numpy()
            jc = data["j_classical"].cpu().numpy()
            meta = {"count": args.count, "seed0": args.seed0, "epochs": args.epochs, "final_loss": hist[-1],
                    "data_s": t1 - t0, "train_s": t2 - t1, "label_mean_best_iters": float(jb.mean()),
                    "label_mean_classical_iters": float(jc.mean())}
            save(ctx, args.out, meta)
            print(json.dumps(meta))
        else:
            meta = load(ctx, args.net)
            data = build_set(ctx, range(args.seed0, args.seed0 + args.count), shape=(1024, 768), keep=True)
            res, _ = evaluate(ctx, data["mats"], data)
            res["train_meta"] = meta
            print(json.dumps(res))


if __name__ == "__main__":
    main()
