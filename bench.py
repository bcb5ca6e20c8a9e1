"""Benchmark: the whole IHS-BIN ridge path on one MI355X.

A step is one pass of the hot path over one synthetic problem: sketch, sketched
Gram, per-interval Cholesky and inverse factors, step-size estimate, basis
recursion, and evaluation of x(lam) at all T lambdas (the path is freed after).
The inputs are resident in HBM before the timed region starts.

Default workload: dense A, n = 131072, d = 2048, FP32 storage, singular values
exp(-i/300), b = A x* + 0.05 noise, SRHT sketch with initial m = 1024, T = 200
lambdas log-spaced in [1e-4, 1e1].

Prints one JSON line.  ``value`` = lambda-solves per second (T per step).
Outside the timed region the result is checked on sampled lambdas against the
FP64 CPU oracle, which is also timed on the host as ``cpu_baseline``.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_MFMA_PEAK = 78.6e12   # MI355X dense FP64 matrix, flop/s
HBM_PEAK = 8.0e12          # bytes/s

# HBM bytes per launch of the A^T A product GEMMs on the default workload come
# from rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled by a 1 GiB copy
# calibration, recorded in the profile summary below together with the sha256
# of the GEMM source they were measured on.  When that source has changed
# since (or for another workload) the figure is stale and reported as null.
TRAFFIC_WORKLOAD = "dense_exp300_131072x2048"
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "gemm_ata_traffic_dense_131072x2048.md")
GEMM_SOURCE = os.path.join(ROOT, "paper_2210_12212_amd", "csrc", "gemm.hip")


def recorded_traffic(kernel):
    """Measured HBM bytes per launch of `kernel`, or None when stale/absent."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_PROFILE).read()
        src = hashlib.sha256(open(GEMM_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"gemm\.hip sha256: ([0-9a-f]{64})", text)
    if not m or m.group(1) != src:
        return None
    m = re.search(r"bytes per launch %s: ([0-9.eE+]+)" % re.escape(kernel), text)
    return float(m.group(1)) if m else None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def ata_sweep(args, torch, W, Context):
    """Time W = A^T A U through the C ABI at the widths the basis steps use."""
    p = W.make(args.workload, n=args.n)
    dev = torch.device("cuda", 0)
    A = torch.from_numpy(p.A).to(dev)
    ctx = Context(0)
    g = torch.Generator(device=dev).manual_seed(7)
    print(f"# W = A^T A U on {p.name} (n={p.n}, d={p.d}, {p.A.dtype}); flops 4 n d w per call")
    print("| w | ms per call | TFLOP/s |\n|---:|---:|---:|")
    for w in (16, 23, 32, 46, 48, 64, 69, 80, 92, 96, 115, 128, 138, 161, 184, 207, 230, 253, 256):
        ldu = 16 if w <= 16 else 32 if w <= 32 else (w + 63) // 64 * 64
        U = torch.randn((p.d, ldu), generator=g, device=dev, dtype=torch.float64)[:, :w]
        ctx.ata_apply(A, U)
        torch.cuda.synchronize()
        reps = 5
        t = time.perf_counter()
        for _ in range(reps):
            ctx.ata_apply(A, U)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / reps
        print(f"| {w} | {ms:.3f} | {4.0 * p.n * p.d * w / ms / 1e9:.1f} |", flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="dense_exp300_131072x2048")
    ap.add_argument("--n", type=int, default=None, help="override n (smaller runs)")
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--rate-target", type=float, default=0.5)
    ap.add_argument("--lanczos-steps", type=int, default=6)
    ap.add_argument("--gram-prec", choices=("f64", "bf16x3"), default="f64",
                    help="sketched Gram precision (the factor and the recursion stay FP64)")
    ap.add_argument("--m-policy", choices=("spectral", "alg4", "fixed"), default="spectral",
                    help="sketch size: spectral probe (default), Algorithm 4 at lam_min, or m0")
    ap.add_argument("--oracle-lambdas", type=int, default=12,
                    help="lambdas of the sample solved by the CPU oracle")
    ap.add_argument("--no-oracle", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (counter calibration)")
    ap.add_argument("--ata-sweep", action="store_true",
                    help="only time the A^T A product (ihsbin_ata_apply) at basis-step widths")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the path is built and "
              "measured on a single MI355X", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        # a plain copy of known size: HBM counters read for it calibrate the
        # FETCH_SIZE / WRITE_SIZE figures of the solver kernels
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.calibrate_copy} MiB three times")
        return
    import workloads as W
    from paper_2210_12212_amd import Context

    if args.ata_sweep:
        ata_sweep(args, torch, W, Context)
        return

    t0 = time.time()
    p = W.make(args.workload, n=args.n)
    log(f"[bench] workload {p.name}: n={p.n} d={p.d} K={p.B.shape[1]} T={len(p.lambdas)} "
        f"sketch={p.sketch} m0={p.m} (generated in {time.time() - t0:.1f}s)")
    dev = torch.device("cuda", 0)
    A = torch.from_numpy(p.A).to(dev)
    B = torch.from_numpy(p.B).to(dev)
    torch.cuda.synchronize()
    ctx = Context(0)
    opts = dict(sketch=p.sketch, m=p.m, seed=p.sketch_seed, tol=args.tol,
                rate_target=args.rate_target, lanczos_steps=args.lanczos_steps, timing=1,
                gram_prec={"f64": 0, "bf16x3": 1}[args.gram_prec],
                adaptive_m={"fixed": 0, "spectral": 1, "alg4": 2}[args.m_policy])
    X = torch.empty((len(p.lambdas), p.d, p.B.shape[1]), dtype=torch.float64, device=dev)

    def step():
        path, rep = ctx.path_build(A, B, p.lam_min, p.lam_max, **opts)
        path.eval(p.lambdas, out=X)
        path.free()
        return rep

    for w in range(args.warmup):
        rep = step()
        log(f"[bench] warmup {w}: {rep['ms_total']:.1f} ms  m_used={rep['m_used']} "
            f"k_max={rep['k_max_used']} k_sum={rep['k_sum']} status={rep['status']}")
    lat = []
    reps = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        ts = time.perf_counter()
        reps.append(step())
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - ts) * 1e3)
        log(f"[bench] step {s}: {lat[-1]:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    T = len(p.lambdas)
    value = T * args.steps / elapsed
    rep = reps[-1]

    # dominant kernel: the two FP64 MFMA GEMMs of A^T A U (each 2*n*d*w flops)
    launches = max(1, rep["ata_launches"])
    half_flops = rep["ata_flops"] / 2.0
    dom = "gemm_y_AU" if rep["ata_ms_y"] >= rep["ata_ms_w"] else "gemm_w_AtY"
    dom_ms = max(rep["ata_ms_y"], rep["ata_ms_w"])
    achieved = (half_flops / launches) / (dom_ms / launches * 1e-3) / 1e12 if dom_ms > 0 else 0.0
    traffic = recorded_traffic(dom) if p.name == TRAFFIC_WORKLOAD and args.n is None else None
    roofline = {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 3),
                "peak": FP64_MFMA_PEAK / 1e12, "unit": "TFLOP/s",
                "frac": round(achieved * 1e12 / FP64_MFMA_PEAK, 4), "traffic": traffic,
                "launches": rep["ata_launches"],
                "flops_per_launch": half_flops / launches,
                "avg_launch_ms": dom_ms / launches,
                "ata_ms_y": rep["ata_ms_y"], "ata_ms_w": rep["ata_ms_w"]}

    # marginal cost of a lambda on a resident basis (outside the timed region):
    # evaluation only, for the workload's T and for a dense grid of 100000 lambdas
    path, _ = ctx.path_build(A, B, p.lam_min, p.lam_max, **opts)
    eval_only = {}
    n_dense = int(min(100000, 4e9 // (8 * p.d * p.B.shape[1])))  # output kept <= 4 GB
    for name, lams in (("T", p.lambdas),
                       (f"dense_{n_dense}", W.lambda_grid(p.lam_min, p.lam_max, n_dense))):
        out = torch.empty((len(lams), p.d, p.B.shape[1]), dtype=torch.float64, device=dev)
        path.eval(lams, out=out)
        torch.cuda.synchronize()
        reps = 20 if len(lams) < 10000 else 3
        te = time.perf_counter()
        for _ in range(reps):
            path.eval(lams, out=out)
        torch.cuda.synchronize()
        eval_only[name] = round(len(lams) * reps / (time.perf_counter() - te), 1)
        del out
    path.free()
    log(f"[bench] eval only: {eval_only} lambda-solves/s")

    # accuracy on sampled lambdas, and the oracle timed on the host (outside the timed region)
    Xh = X.cpu().numpy()
    cpu = None
    max_err = None
    if not args.no_oracle:
        from oracle import direct
        cores = len(os.sched_getaffinity(0))
        idx = np.unique(np.linspace(0, T - 1, min(T, args.oracle_lambdas)).round().astype(int))
        wide = p.n < p.d  # the oracle takes the n x n dual form (Section 5.2)
        tg = time.perf_counter()
        if wide:
            G = direct.dual_gram(p.A)
        else:
            G = direct.gram(p.A)
            C = direct.atb(p.A, p.B)
        t_gram = time.perf_counter() - tg
        ts = time.perf_counter()
        if wide:
            Xo = direct.solve_dual_from_gram(G, p.A, p.B, p.lambdas[idx])
        else:
            Xo = direct.solve_from_gram(G, C, p.lambdas[idx])
        t_solve = (time.perf_counter() - ts) / len(idx)
        err = direct.rel_err(Xh[idx], Xo)
        max_err = float(err.max())
        t_full = t_gram + T * t_solve
        cpu = {"value": round(T / t_full, 3), "unit": "lambda-solves/s", "cores": cores,
               "kind": "oracle",
               "sample": f"{'A A^T (dual form)' if wide else 'G=A^T A and A^T b'} over the full "
                         f"matrix ({t_gram:.1f}s) plus {len(idx)} of "
                         f"{T} per-lambda Cholesky solves ({t_solve * 1e3:.1f} ms each); the full "
                         f"path time is t_G + T*t_solve = {t_full:.1f}s"}
        log(f"[bench] oracle: gram {t_gram:.1f}s, solve {t_solve * 1e3:.1f} ms/lambda, "
            f"max rel err on {len(idx)} lambdas = {max_err:.3e}")

    out = {
        "metric": "ridge-path lambda-solves/s at <=1e-6 rel err vs FP64",
        "value": round(value, 3),
        "unit": "lambda-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": p.name, "n": p.n, "d": p.d, "K": int(p.B.shape[1]), "T": T,
                   "storage": str(p.A.dtype), "sketch": p.sketch, "m0": p.m,
                   "m_used": rep["m_used"], "L": rep["L"], "k_max": rep["k_max_used"],
                   "k_sum": rep["k_sum"], "lam": [p.lam_min, p.lam_max], "tol": args.tol,
                   "rate_target": args.rate_target, "lanczos_steps": args.lanczos_steps,
                   "gram_prec": args.gram_prec, "m_policy": args.m_policy},
        "max_rel_err": max_err,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "phase_ms": {k: rep[k] for k in ("ms_sketch", "ms_factor", "ms_spectrum", "ms_basis",
                                         "ms_total")},
        "eval_only_lambda_solves_per_s": eval_only,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
