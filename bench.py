"""Benchmark: the whole IHS-BIN ridge path on one MI355X.

A step is one pass of the hot path over one synthetic problem: sketch, sketched
Gram, per-interval Cholesky and inverse factors, step-size estimate, basis
recursion, and evaluation of x(lam) at all T lambdas (the path is freed after).
The inputs are resident in HBM before the timed region starts.

Default workload: the matrix-valued problem (Section 5.3), dense A with
n = 262144, d = 4096, FP32 storage, singular values i^-0.5, B = A X* + 0.05
noise with K = 64 right-hand sides, Gaussian sketch with initial m = 2048 on
the BF16 matrix cores, T = 100 lambdas log-spaced in [1e-4, 1e1]; the basis
products run in FP64 until the increments they refine are below 1e-2 of x,
then on the FP32 matrix cores (--basis-prec, --f32-switch).

Prints one JSON line.  ``value`` = lambda-solves per second (T per step).
Outside the timed region every lambda of the last step is checked against the
FP64 CPU oracle (the eigendecomposition form of Section 2.1); ``value`` is
null unless every error is
<= 1e-6 and every build returned IHSBIN_OK.  The oracle's per-lambda Cholesky
form is also timed on the host on a sample of lambdas as ``cpu_baseline``.
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
FP32_MFMA_PEAK = 157.3e12  # MI355X dense FP32 matrix, flop/s
HBM_PEAK = 8.0e12          # bytes/s

# HBM bytes per launch of the A^T A product GEMMs on the default workload come
# from rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled by a 1 GiB copy
# calibration, recorded in the profile summary below together with the sha256
# of the GEMM source they were measured on.  When that source has changed
# since (or for another workload) the figure is stale and reported as null.
TRAFFIC_PROFILES = {
    "dense_invsqrt_262144x4096_k64": os.path.join(ROOT, "profiles",
                                                  "gemm_ata_traffic_dense_262144x4096_k64.md"),
    "csr_zipf_1048576x8192": os.path.join(ROOT, "profiles",
                                          "csr_products_traffic_csr_1048576x8192.md"),
}
DEFAULT_WORKLOAD = "dense_invsqrt_262144x4096_k64"
# the arithmetic of the Gaussian sketch product per workload when not given:
# the matrix-valued workload is specified with its sketch on the BF16 matrix cores
SKETCH_PREC_DEFAULT = {"dense_invsqrt_262144x4096_k64": "bf16"}
# the sketched Gram on the BF16 matrix cores per workload when not given (none
# by default: the CSR workload's CountSketch keeps SA sparse and forms its
# Gram from the entries in FP64, which gram_prec does not change)
GRAM_PREC_DEFAULT = {}
# the spectral policy's rate target per workload when not given (0.5
# otherwise): with the BF16 sketch, doubling m to 131072 costs the
# 262144 x 4096 workload ~0.38 s of sketch and saves ~0.57 s of basis steps
# (k 17 -> 13; bench.py --m-sweep --sweep-m-min 65536 --sweep-rates 0.35)
RATE_TARGET_DEFAULT = {"dense_invsqrt_262144x4096_k64": 0.35}
CSRC = os.path.join(ROOT, "paper_2210_12212_amd", "csrc")


def recorded_traffic(workload, kernel):
    """Measured HBM bytes per launch of `kernel`, or None when stale/absent.

    The profile names the kernel sources it was measured on with their sha256
    ("<file>.hip sha256: <hash>"); a changed source makes the figure stale."""
    import hashlib
    import re
    if workload not in TRAFFIC_PROFILES:
        return None
    try:
        text = open(TRAFFIC_PROFILES[workload]).read()
    except OSError:
        return None
    pinned = re.findall(r"(\w+\.hip) sha256: ([0-9a-f]{64})", text)
    if not pinned:
        return None
    for fname, digest in pinned:
        try:
            src = hashlib.sha256(open(os.path.join(CSRC, fname), "rb").read()).hexdigest()
        except OSError:
            return None
        if src != digest:
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


def m_sweep(args, torch, W, Context):
    """Sketch-size policies on one workload: the spectral probe, Algorithm 4,
    and fixed m from m0 doubling up to the cap; one build + evaluation each
    (after one untimed warm-up build), with k, phase times and the error
    at every lambda against the oracle's eigendecomposition form."""
    from oracle import direct
    p = W.make(args.workload, n=args.n)
    dev = torch.device("cuda", 0)
    csr = hasattr(p.A, "row_ptr")
    if csr:
        from paper_2210_12212_amd import CsrInput
        A = CsrInput(torch.from_numpy(p.A.row_ptr).to(dev), torch.from_numpy(p.A.col_idx).to(dev),
                     torch.from_numpy(p.A.vals).to(dev), p.A.n, p.A.d)
    else:
        A = torch.from_numpy(p.A).to(dev)
    B = torch.from_numpy(p.B).to(dev)
    sp = args.sketch_prec or SKETCH_PREC_DEFAULT.get(p.name, "f64")
    gp = args.gram_prec or GRAM_PREC_DEFAULT.get(p.name, "f64")
    base = dict(sketch=p.sketch, seed=p.sketch_seed, tol=args.tol, rate_target=args.rate_target,
                lanczos_steps=args.lanczos_steps, sketch_prec={"f64": 0, "bf16": 1, "fp8": 2}[sp], k_max=96,
                gram_prec={"f64": 0, "bf16x3": 1}[gp],
                basis_prec={"f64": 0, "f32": 1, "mixed": 2}[args.basis_prec],
                f32_switch=args.f32_switch)
    ev, V = direct.eig_of_gram(direct.gram(p.A))
    ref = direct.solve_from_eig(ev, V, direct.atb(p.A, p.B), p.lambdas)
    log(f"[sweep] {p.name}: oracle ready")
    cap = args.sweep_m_max or min(p.n, 32 * p.d)
    runs = [("spectral", dict(m=p.m, adaptive_m=1))]
    if p.sketch == "gaussian":
        runs.append(("spectral_exact", dict(m=p.m, adaptive_m=3)))
    for r in args.sweep_rates:
        runs.append((f"spectral_rate{r:g}", dict(m=p.m, adaptive_m=1, rate_target=r)))
    if not args.sweep_no_alg4:
        runs.append(("alg4", dict(m=p.m, adaptive_m=2)))
    m = p.m
    while m <= cap:
        if m >= args.sweep_m_min:
            runs.append((f"fixed_{m}", dict(m=m, adaptive_m=0)))
        m *= 2
    ctx = Context(0)
    for name, extra in runs:
        opts = dict(base, **extra)
        try:
            ctx.solve_path(A, B, p.lambdas[:1], **opts)
            torch.cuda.synchronize()
            t = time.perf_counter()
            X, rep = ctx.solve_path(A, B, p.lambdas, **opts)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t) * 1e3
            err = float(direct.rel_err(X.cpu().numpy(), ref).max())
            row = {"policy": name, "m_used": rep["m_used"], "k_max": rep["k_max_used"],
                   "k_sum": rep["k_sum"], "status": rep["status"], "ms_path": round(ms, 2),
                   "ms_sketch": round(rep["ms_sketch"], 2), "ms_factor": round(rep["ms_factor"], 2),
                   "ms_spectrum": round(rep["ms_spectrum"], 2),
                   "ms_basis": round(rep["ms_basis"], 2), "max_rel_err": err,
                   "lambda_solves_per_s": round(len(p.lambdas) / ms * 1e3, 2)}
        except Exception as e:  # noqa: BLE001 - report and go on with the next policy
            row = {"policy": name, "error": str(e)[:200]}
        print(json.dumps(row), flush=True)
    ctx.close()


def batch_small(args, torch, W, Context):
    """Many small problems through ihsbin_path_build_batch: the requests of
    --serve-small (dense 2048 x 256, FP32, K = 1, T = 100 in [1e-4, 1e1],
    Gaussian sketch) built --batch-size at a time; paths/s and lambda-solves/s
    over the whole set, each path evaluated at its T lambdas; sampled
    problems checked against the oracle."""
    from oracle import direct
    dev = torch.device("cuda", 0)
    reqs = [dict(index=i, arrival=0.0, n=2048, d=256, dense=True, K=1, seed=9000 + i)
            for i in range(args.serve_requests)]
    data = [_serving_inputs(torch, r, dev) for r in reqs]
    A = torch.stack([a for a, _ in data])
    B = torch.stack([b for _, b in data])
    del data
    T = 100
    lams = W.lambda_grid(1e-4, 1e1, T)
    opts = dict(sketch="gaussian", seed=77, adaptive_m=1, tol=args.tol,
                rate_target=args.rate_target, lanczos_steps=args.lanczos_steps,
                graph_steps=args.graph_steps)
    ctx = Context(0)
    P = len(reqs)
    bs = min(args.batch_size, P)
    X = torch.empty((P, T, 256, 1), dtype=torch.float64, device=dev)

    def run():
        reps = []
        for p0 in range(0, P, bs):
            paths, rep = ctx.path_build_batch(A[p0:p0 + bs], B[p0:p0 + bs], lams[0], lams[-1],
                                              **opts)
            for j, path in enumerate(paths):
                path.eval(lams, out=X[p0 + j])
                path.free()
            reps.append(rep)
        return reps

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        reps = run()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t) / args.steps
    Xh = X.cpu().numpy()
    errs = []
    for i in np.linspace(0, P - 1, min(P, 8)).round().astype(int):
        Ah = A[i].cpu().numpy()
        Bh = B[i].cpu().numpy()
        errs.append(float(direct.rel_err(Xh[i], direct.ridge_path(Ah, Bh, lams)).max()))
    res = {"metric": "paths/s (many small problems, one batched build)",
           "value": round(P / el, 2), "unit": "paths/s",
           "lambda_solves_per_s": round(P * T / el, 1), "problems": P, "batch_size": bs,
           "ms_per_batch": round(el * 1e3 / len(reps), 2), "steps": args.steps,
           "warmup": args.warmup, "m_used": reps[-1]["m_used"], "k": reps[-1]["k_max_used"],
           "statuses": sorted({int(r["status"]) for r in reps}),
           "phase_ms_last_batch": {k: round(reps[-1][k], 2) for k in
                                   ("ms_sketch", "ms_factor", "ms_spectrum", "ms_basis",
                                    "ms_total")},
           "max_rel_err_sampled": max(errs),
           "config": {"workload": "small_2048x256_burst", "T": T, "lam": [1e-4, 1e1],
                      "tol": args.tol, "graph_steps": args.graph_steps}}
    print(json.dumps(res), flush=True)
    ctx.close()


def _serving_inputs(torch, req, dev):
    """Request data drawn on the device from (seed, shape): dense A with columns
    scaled by (j+1)^-0.7 and B = A x* + 0.05 noise, or CSR A with 16 entries
    per row (uniform columns; repeats are summed) and B ~ N(0, 1); FP32."""
    g = torch.Generator(device=dev)
    g.manual_seed(req["seed"])
    n, d, K = req["n"], req["d"], req["K"]
    if req["dense"]:
        scale = (torch.arange(d, device=dev, dtype=torch.float32) + 1.0) ** -0.7
        A = torch.randn((n, d), generator=g, device=dev, dtype=torch.float32) * scale
        xs = torch.randn((d, K), generator=g, device=dev, dtype=torch.float32)
        B = A @ xs + 0.05 * torch.randn((n, K), generator=g, device=dev, dtype=torch.float32)
        return A, B.contiguous()
    from paper_2210_12212_amd import CsrInput
    per = 16
    cols = torch.randint(0, d, (n, per), generator=g, device=dev, dtype=torch.int64)
    cols = torch.sort(cols, dim=1).values.to(torch.int32).reshape(-1).contiguous()
    vals = torch.randn(n * per, generator=g, device=dev, dtype=torch.float32)
    rp = torch.arange(0, n * per + 1, per, device=dev, dtype=torch.int32)
    B = torch.randn((n, K), generator=g, device=dev, dtype=torch.float32)
    return CsrInput(rp, cols, vals, n, d), B


def serve(args, torch, W):
    """Replay of the serving workload through the request server."""
    from paper_2210_12212_amd import Server
    dev = torch.device("cuda", 0)
    reqs = _serve_requests(args, W)
    lams = W.lambda_grid(1e-4, 1e1, 100)
    srv = Server(0, workers=args.serve_workers)
    log(f"[serve] {len(reqs)} requests, {args.serve_rate}/s, {args.serve_workers} workers, "
        f"at most {args.serve_outstanding} outstanding")
    # warm-up (one small dense and one CSR request, not counted)
    for wreq in (dict(seed=1, n=4096, d=128, K=1, dense=True),
                 dict(seed=2, n=4096, d=128, K=1, dense=False)):
        A, B = _serving_inputs(torch, wreq, dev)
        path, _ = srv.wait(srv.submit(A, B, lams[0], lams[-1], **_serve_opts(wreq, args)))
        path.free()
    torch.cuda.synchronize()
    out = {}
    done = []
    i = 0
    t0 = time.perf_counter()
    last = t0
    while i < len(reqs) or out:
        now = time.perf_counter() - t0
        progressed = False
        while i < len(reqs) and reqs[i]["arrival"] <= now and len(out) < args.serve_outstanding:
            A, B = _serving_inputs(torch, reqs[i], dev)
            ts = time.perf_counter() - t0
            rid = srv.submit(A, B, lams[0], lams[-1], **_serve_opts(reqs[i], args))
            out[rid] = (reqs[i], A, B, ts)
            i += 1
            progressed = True
        for rid in list(out):
            path, info = srv.wait(rid, timeout_ms=0)
            if path is None:
                continue
            req, A, B, ts = out.pop(rid)
            X = path.eval(lams)
            path.free()
            te = time.perf_counter() - t0
            done.append(dict(index=req["index"], arrival=req["arrival"], submit=ts, end=te,
                             ms_build=info["ms_build"], ms_queue=info["ms_queue"],
                             status=info["status"], m_used=info["report"]["m_used"],
                             k_max=info["report"]["k_max_used"], n=req["n"], d=req["d"],
                             K=req["K"], dense=req["dense"]))
            if req["index"] in args._check:
                args._check[req["index"]] = (A, B, X.cpu().numpy())
            del X
            progressed = True
        if time.perf_counter() - last > 5.0:
            last = time.perf_counter()
            log(f"[serve] t={now:.1f}s submitted {i} done {len(done)} outstanding {len(out)}")
        if not progressed:
            time.sleep(0.0005)
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    return reqs, done, wall, st, lams


def _serve_requests(args, W):
    if args.serve_small:
        # many small problems at once: 2048 x 256 dense requests, all arriving at t = 0
        return [dict(index=i, arrival=0.0, n=2048, d=256, dense=True, K=1, seed=9000 + i)
                for i in range(args.serve_requests)]
    return W.serving_mix(args.serve_requests, rate=args.serve_rate)


def _serve_opts(req, args):
    return dict(sketch="gaussian" if req["dense"] else "countsketch", seed=req["seed"],
                adaptive_m={"spectral": 1, "alg4": 2, "spectral-exact": 3}[args.serve_m_policy], tol=args.tol,
                sketch_prec={"f64": 0, "bf16": 1, "fp8": 2}[args.serve_sketch_prec],
                rate_target=args.rate_target,
                lanczos_steps=args.lanczos_steps)


def serve_main(args, torch, W):
    from oracle import direct
    # requests checked against the oracle: the three smallest dense and CSR ones
    reqs = _serve_requests(args, W)
    small = sorted(reqs, key=lambda r: r["n"] * r["d"])
    pick = [r["index"] for r in small if r["dense"]][:2] + \
           [r["index"] for r in small if not r["dense"]][:1]
    args._check = {k: None for k in pick}
    reqs, done, wall, st, lams = serve(args, torch, W)
    lat = np.array([d["end"] - d["arrival"] for d in done]) * 1e3
    lat_submit = np.array([d["end"] - d["submit"] for d in done]) * 1e3
    T = len(lams)
    errs = {}
    cpu_t = 0.0
    cores = len(os.sched_getaffinity(0))
    idx = np.unique(np.linspace(0, T - 1, 5).round().astype(int))
    for k, v in args._check.items():
        if v is None:
            continue
        A, B, X = v
        if hasattr(A, "row_ptr"):
            Ah = W.CsrMatrix(A.n, A.d, A.row_ptr.cpu().numpy(), A.col_idx.cpu().numpy(),
                             A.vals.cpu().numpy())
        else:
            Ah = A.cpu().numpy()
        Bh = B.cpu().numpy()
        tc = time.perf_counter()
        ref = direct.ridge_path(Ah, Bh, lams[idx])
        cpu_t += (time.perf_counter() - tc) / len(idx) * T
        errs[k] = float(direct.rel_err(X[idx], ref).max())
    solves = T * len(done)
    res = {
        "metric": "served ridge paths: lambda-solves/s, latency p50/p99",
        "value": round(solves / wall, 3),
        "unit": "lambda-solves/s",
        "n_gpus": 1,
        "requests": len(done),
        "requests_per_s": round(len(done) / wall, 3),
        "wall_s": round(wall, 3),
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "latency_from_submit_ms": {"p50": float(np.percentile(lat_submit, 50)),
                                   "p99": float(np.percentile(lat_submit, 99))},
        "build_ms": {"p50": float(np.percentile([d["ms_build"] for d in done], 50)),
                     "p99": float(np.percentile([d["ms_build"] for d in done], 99))},
        "statuses": sorted({d["status"] for d in done}),
        "server": st,
        "max_rel_err_sampled": errs,
        "higher_is_better": True,
        "dtype": "+".join(["f64"] + ([args.serve_sketch_prec] if args.serve_sketch_prec != "f64"
                                      else []) +
                          (["bf16"] if (args.gram_prec or "f64") == "bf16x3" and
                           args.serve_sketch_prec != "bf16" else [])),
        "data": "synthetic",
        "config": {"workload": "small_2048x256_burst" if args.serve_small else "serving_mix",
                   "rate_per_s": None if args.serve_small else args.serve_rate,
                   "workers": args.serve_workers, "outstanding_cap": args.serve_outstanding,
                   "T": T, "lam": [1e-4, 1e1], "m_policy": args.serve_m_policy,
                   "sketch_prec": args.serve_sketch_prec,
                   "tol": args.tol},
        "cpu_baseline": {"value": round(T * len(errs) / cpu_t, 3) if cpu_t else None,
                         "unit": "lambda-solves/s", "cores": cores, "kind": "oracle",
                         "sample": f"direct per-lambda solves of {len(errs)} sampled requests "
                                   f"({len(idx)} lambdas each, scaled to T)"},
    }
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--n", type=int, default=None, help="override n (smaller runs)")
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--rate-target", type=float, default=None,
                    help="spectral policy's rate target (default: per workload, else 0.5)")
    ap.add_argument("--lanczos-steps", type=int, default=4)
    ap.add_argument("--gram-prec", choices=("f64", "bf16x3"), default=None,
                    help="sketched Gram precision (the factor and the recursion stay FP64); "
                         "default bf16x3 for the CSR workload, else f64")
    ap.add_argument("--sketch-prec", choices=("f64", "bf16", "fp8"), default=None,
                    help="arithmetic of the Gaussian sketch product (other sketches ignore it); "
                         "default bf16 for the matrix-valued workload, else f64")
    ap.add_argument("--basis-prec", choices=("f64", "f32", "mixed"), default="mixed",
                    help="arithmetic of the basis steps' A^T A products (dense FP32 A; other "
                         "inputs always FP64): FP64, FP32 matrix cores, or FP64 until the "
                         "increments are small, then FP32 (default)")
    ap.add_argument("--f32-switch", type=float, default=3e-2,
                    help="relative increment below which --basis-prec mixed uses FP32 "
                         "(3e-2: on the 262144 x 4096 workload 1e-2 gives 8.3e-8 at every "
                         "lambda, 2e-2 to 5e-2 switch one step earlier at 8.6e-8, 1e-1 "
                         "gives 2.3e-7)")
    ap.add_argument("--m-policy", choices=("spectral", "alg4", "fixed", "spectral-exact"),
                    default="spectral",
                    help="sketch size: spectral probe (default), Algorithm 4 at lam_min, m0, "
                         "or the spectral probe with S = I once a Gaussian sketch would cost "
                         "more than A^T A")
    ap.add_argument("--oracle-lambdas", type=int, default=12,
                    help="lambdas of the sample the CPU oracle's Cholesky form is timed on")
    ap.add_argument("--no-oracle", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (counter calibration)")
    ap.add_argument("--serve", action="store_true",
                    help="replay the serving workload (Poisson arrivals) through the server")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-small", action="store_true",
                    help="serve many 2048 x 256 dense problems submitted at once instead")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--serve-m-policy", choices=("spectral", "alg4", "spectral-exact"),
                    default="spectral",
                    help="sketch size of served builds")
    ap.add_argument("--serve-sketch-prec", choices=("f64", "bf16", "fp8"), default="bf16",
                    help="arithmetic of the Gaussian sketch product of served dense requests")
    ap.add_argument("--serve-outstanding", type=int, default=32,
                    help="client-side cap on submitted, unfinished requests")
    ap.add_argument("--batch-small", action="store_true",
                    help="build the --serve-small problems with batched builds (--batch-size "
                         "problems per build) instead of serving them one by one")
    ap.add_argument("--batch-size", type=int, default=256)
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="batched builds: basis steps captured per HIP graph (0: none)")
    ap.add_argument("--sweep-rates", type=lambda v: [float(x) for x in v.split(",") if x],
                    default=[], help="--m-sweep: also the spectral policy at these rate targets")
    ap.add_argument("--sweep-m-min", type=int, default=0,
                    help="--m-sweep: fixed sketch sizes from this one up")
    ap.add_argument("--sweep-m-max", type=int, default=0,
                    help="--m-sweep: fixed sketch sizes up to this one (default: the cap 32 d)")
    ap.add_argument("--sweep-no-alg4", action="store_true")
    ap.add_argument("--m-sweep", action="store_true",
                    help="only compare sketch-size policies (spectral, Algorithm 4, fixed m)")
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

    if args.rate_target is None:
        single = not (args.serve or args.batch_small)
        args.rate_target = RATE_TARGET_DEFAULT.get(args.workload, 0.5) if single else 0.5
    if args.ata_sweep:
        ata_sweep(args, torch, W, Context)
        return
    if args.m_sweep:
        m_sweep(args, torch, W, Context)
        return
    if args.batch_small:
        batch_small(args, torch, W, Context)
        return
    if args.serve:
        serve_main(args, torch, W)
        return

    if args.sketch_prec is None:
        args.sketch_prec = SKETCH_PREC_DEFAULT.get(args.workload, "f64")
    if args.gram_prec is None:
        args.gram_prec = GRAM_PREC_DEFAULT.get(args.workload, "f64")
    t0 = time.time()
    p = W.make(args.workload, n=args.n)
    log(f"[bench] workload {p.name}: n={p.n} d={p.d} K={p.B.shape[1]} T={len(p.lambdas)} "
        f"sketch={p.sketch} m0={p.m} (generated in {time.time() - t0:.1f}s)")
    dev = torch.device("cuda", 0)
    csr = hasattr(p.A, "row_ptr")
    # CountSketch / SJLT of a CSR matrix with d <= 8192: the library keeps SA
    # sparse (its Gram from the entries, FP64)
    sparse_gram = csr and p.sketch in ("countsketch", "sjlt") and p.d <= 8192
    if csr:
        from paper_2210_12212_amd import CsrInput
        A = CsrInput(torch.from_numpy(p.A.row_ptr).to(dev), torch.from_numpy(p.A.col_idx).to(dev),
                     torch.from_numpy(p.A.vals).to(dev), p.A.n, p.A.d)
    else:
        A = torch.from_numpy(p.A).to(dev)
    B = torch.from_numpy(p.B).to(dev)
    torch.cuda.synchronize()
    ctx = Context(0)
    opts = dict(sketch=p.sketch, m=p.m, seed=p.sketch_seed, tol=args.tol,
                rate_target=args.rate_target, lanczos_steps=args.lanczos_steps, timing=1,
                gram_prec={"f64": 0, "bf16x3": 1}[args.gram_prec],
                adaptive_m={"fixed": 0, "spectral": 1, "alg4": 2, "spectral-exact": 3}[args.m_policy],
                sketch_prec={"f64": 0, "bf16": 1, "fp8": 2}[args.sketch_prec],
                basis_prec={"f64": 0, "f32": 1, "mixed": 2}[args.basis_prec],
                f32_switch=args.f32_switch)
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
    step_reps = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        ts = time.perf_counter()
        step_reps.append(step())
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - ts) * 1e3)
        log(f"[bench] step {s}: {lat[-1]:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    T = len(p.lambdas)
    value = T * args.steps / elapsed
    rep = step_reps[-1]

    # dominant kernel: the two products of A^T A U (dense: MFMA GEMMs of
    # 2*n*d*w flops each, on the FP64 matrix cores, and with basis_prec on the
    # FP32 ones for the later steps; the one with more summed time is reported)
    def _gemm_roofline(ms_y, ms_w, flops, launches, peak, tag):
        launches = max(1, launches)
        half = flops / 2.0
        dms = max(ms_y, ms_w)
        kern = ("gemm_y_AU" if ms_y >= ms_w else "gemm_w_AtY") + tag
        ach = (half / launches) / (dms / launches * 1e-3) / 1e12 if dms > 0 else 0.0
        return {"bound": "mfma", "kernel": kern, "achieved": round(ach, 3), "peak": peak / 1e12,
                "unit": "TFLOP/s", "frac": round(ach * 1e12 / peak, 4),
                "launches": launches, "flops_per_launch": half / launches,
                "avg_launch_ms": dms / launches, "ata_ms_y": ms_y, "ata_ms_w": ms_w}, dms

    if csr:
        # CSR products: 2 nnz w multiply-adds each, bound by their loads.
        # Algorithmic bytes of a launch of width w: Y = A U reads A (column
        # index and value, 8 B per entry, plus the row pointers) and U once and
        # writes Y once (8 n w + 8 d w); W = A^T Y reads the column-major copy
        # (row index and value, 8 B per entry, plus the column pointers) and Y
        # once and writes W once.  The summed width follows from the launches'
        # flop count (4 nnz w each).
        launches = max(1, rep["ata_launches"])
        nnz = int(p.A.col_idx.size)
        sum_w = rep["ata_flops"] / (4.0 * nnz) if nnz else 0.0
        vec = 8.0 * (p.n + p.d) * sum_w / launches
        by = 8.0 * nnz + 4.0 * (p.n + 1) + vec
        bw = 8.0 * nnz + 4.0 * (p.d + 1) + vec
        if rep["ata_ms_y"] >= rep["ata_ms_w"]:
            dom, dom_ms, abytes = "csr_Y_AU", rep["ata_ms_y"], by
        else:
            dom, dom_ms, abytes = "csc_gather_W_AtY", rep["ata_ms_w"], bw
        achieved = abytes / (dom_ms / launches * 1e-3) / 1e9 if dom_ms > 0 else 0.0
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 3),
                    "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                    "frac": round(achieved * 1e9 / HBM_PEAK, 4),
                    "traffic": recorded_traffic(p.name, dom) if args.n is None else None,
                    "bytes_per_launch": abytes, "mean_width": sum_w / launches,
                    "launches": rep["ata_launches"], "avg_launch_ms": dom_ms / launches,
                    "ata_ms_y": rep["ata_ms_y"], "ata_ms_w": rep["ata_ms_w"]}
    else:
        r64, t64 = _gemm_roofline(rep["ata_ms_y"], rep["ata_ms_w"], rep["ata_flops"],
                                  rep["ata_launches"], FP64_MFMA_PEAK, "")
        r32, t32 = _gemm_roofline(rep["ata_f32_ms_y"], rep["ata_f32_ms_w"], rep["ata_f32_flops"],
                                  rep["ata_f32_launches"], FP32_MFMA_PEAK, "_f32")
        roofline = r32 if rep["ata_f32_launches"] and t32 > t64 else r64
        roofline["traffic"] = (recorded_traffic(p.name, roofline["kernel"])
                               if args.n is None else None)
        if rep["ata_f32_launches"] and rep["ata_launches"]:
            roofline["other_precision"] = r64 if roofline is r32 else r32

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

    # accuracy at every lambda, and the oracle timed on the host (outside the
    # timed region)
    Xh = X.cpu().numpy()
    cpu = None
    max_err = None
    n_checked = 0
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
        err_s = direct.rel_err(Xh[idx], Xo)
        t_full = t_gram + T * t_solve
        cpu = {"value": round(T / t_full, 3), "unit": "lambda-solves/s", "cores": cores,
               "kind": "oracle",
               "sample": f"{'A A^T (dual form)' if wide else 'G=A^T A and A^T b'} over the full "
                         f"matrix ({t_gram:.1f}s) plus {len(idx)} of "
                         f"{T} per-lambda Cholesky solves ({t_solve * 1e3:.1f} ms each); the full "
                         f"path time is t_G + T*t_solve = {t_full:.1f}s"}
        log(f"[bench] oracle: gram {t_gram:.1f}s, solve {t_solve * 1e3:.1f} ms/lambda, "
            f"max rel err on the {len(idx)} timed lambdas = {err_s.max():.3e}")
        # every lambda: the eigendecomposition form (one eigh of the d x d
        # Gram, then O(d^2 K) per lambda; the dual form for n < d)
        te = time.perf_counter()
        if wide:
            # z(lam) = (A A^T + lam I)^-1 B through one eigendecomposition of
            # A A^T, then x = A^T z (the dual map of Section 5.2)
            ev, V = direct.eig_of_gram(G)
            log(f"[bench] oracle: eigendecomposition of the {G.shape[0]} x {G.shape[0]} dual Gram "
                f"in {time.perf_counter() - te:.1f}s")
            Z = direct.solve_from_eig(ev, V, p.B, p.lambdas)
            A64 = np.asarray(p.A, dtype=np.float64)
            Xall = np.stack([A64.T @ Z[t] for t in range(len(p.lambdas))])
            del A64
        else:
            ev, V = direct.eig_of_gram(G)
            Xall = direct.solve_from_eig(ev, V, C, p.lambdas)
        err = direct.rel_err(Xh, Xall)
        max_err = float(max(err.max(), err_s.max()))
        n_checked = T
        log(f"[bench] oracle: every lambda checked in {time.perf_counter() - te:.1f}s, "
            f"max rel err {max_err:.3e}")
    statuses = sorted({int(r_["status"]) for r_ in step_reps})
    valid = (max_err is not None and max_err <= 1e-6 and statuses == [0])
    invalid_reason = None
    if max_err is None:
        invalid_reason = "accuracy not checked (--no-oracle)"
    elif max_err > 1e-6:
        invalid_reason = f"max rel err {max_err:.3e} > 1e-6"
    elif statuses != [0]:
        invalid_reason = f"build status {statuses}"

    out = {
        "metric": "ridge-path lambda-solves/s at <=1e-6 rel err vs FP64",
        "value": round(value, 3) if valid else None,
        "unit": "lambda-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # arithmetic types the build ran: FP32 products only for dense FP32 A
        # after the switch, BF16 only where a dense sketch or Gram used it (a
        # CountSketch of a CSR matrix keeps SA sparse, its Gram in FP64)
        "dtype": "+".join(["f64"] + (["f32"] if rep.get("ata_f32_launches") else []) +
                          (["bf16"] if args.sketch_prec == "bf16" or
                           (args.gram_prec == "bf16x3" and not sparse_gram) else []) +
                          (["fp8"] if args.sketch_prec == "fp8" else [])),
        "data": "synthetic",
        "config": {"workload": p.name, "n": p.n, "d": p.d, "K": int(p.B.shape[1]), "T": T,
                   "storage": str(p.A.dtype), "sketch": p.sketch, "m0": p.m,
                   "m_used": rep["m_used"], "L": rep["L"], "k_max": rep["k_max_used"],
                   "k_sum": rep["k_sum"], "lam": [p.lam_min, p.lam_max], "tol": args.tol,
                   "rate_target": args.rate_target, "lanczos_steps": args.lanczos_steps,
                   "gram_prec": args.gram_prec, "m_policy": args.m_policy,
                   "basis_prec": args.basis_prec, "f32_switch": args.f32_switch,
                   "sketch_prec": args.sketch_prec},
        "max_rel_err": max_err,
        "lambdas_checked": n_checked,
        "invalid_reason": invalid_reason,
        "measured_value": round(value, 3),
        "est_rel_err": rep["est_rel_err"],
        "bytes_moved_per_step": rep["bytes_moved"],
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
