#!/usr/bin/env python3
"""Benchmark of mixed-precision block-Jacobi PCG on one MI355X.

Workload: 3D 7-point variable-coefficient diffusion on a 128^3 grid
(n = 2,097,152, nnz = 14,581,760), point coefficients 10**U(-2,2), contiguous
row blocks of 32, RHS U[-1,1] (seed 0), x0 = 0, stop at ||r||/||b|| <= 1e-10.
One step = block-Jacobi setup (extract, FP64 invert, features, round + pack)
plus the PCG solve to 1e-10, with A and b already resident in HBM.

The headline value is the time to solution with the block inverses stored in
FP16 (fMP); the same steps with FP64 storage are timed beside it. A profile
pass times each kernel with HIP events on the stream it runs on and reports
the dominant kernel against the 8 TB/s HBM roofline. The CPU oracle is timed
on a bounded sample on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def spmv_bytes(n, nnz):
    """Algorithmic bytes of one SpMV launch with the folded p update: CSR values
    and column indices, row pointers, z and p_old read once, p_new and q written."""
    return 12 * nnz + 4 * (n + 1) + 32 * n


def apply_bytes(n, nb, ntiles, stored_bytes):
    """Algorithmic bytes of one fused update + apply launch: the stored block
    inverses, per-block metadata (offset 8, scale 8, tag 1, row start 4), the
    tile list, and x, r read+written, p, q read, z written."""
    return stored_bytes + 21 * nb + 4 * (ntiles + 1) + 56 * n


def cpu_baseline(p, iters_hint, budget_iters=8):
    """The oracle as it stands on the host: full FP64 setup of every block and
    FP16 storage, then a few PCG iterations; scaled to a full solve with the
    GPU's iteration count. BLAS limited to one thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import blocks as OB
    from oracle import pcg as OP
    from oracle import precision as OPr
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        nb = len(p.block_ptr) - 1
        M = OP.BJAC(p.A, p.block_ptr, np.full(nb, OPr.FP16, np.uint8))
        t1 = time.perf_counter()
        S = p.A.to_scipy()
        res = OP.pcg(lambda v: S @ v, p.b, M.low, 0.0, budget_iters)
        t2 = time.perf_counter()
    per_iter = (t2 - t1) / max(1, res.iters)
    total_ms = 1e3 * ((t1 - t0) + per_iter * iters_hint)
    return {"value": total_ms, "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": f"oracle setup of all {nb} blocks (Cholesky inverse, FP16 storage) "
                      f"{(t1 - t0):.1f} s + {res.iters} PCG iterations at {per_iter * 1e3:.0f} ms each, "
                      f"scaled to {iters_hint} iterations"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run one 1 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the design for sharding is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2407_15973_amd import binding as mb
    from paper_2407_15973_amd import gen

    dev = "cuda:0"
    log("building the workload")
    p = gen.config2(seed=0, N=args.N, b=32)
    n, nnz, nb = p.A.n, p.A.nnz, len(p.block_ptr) - 1
    A = mb.DeviceCSR(p.A, dev)
    b = torch.as_tensor(p.b, device=dev)
    solver = mb.Solver(n, dev)
    tol, maxit = p.tol, p.maxit
    pol16 = mb.Policy(mode=mb.FIXED, low=mb.FP16)
    pol64 = mb.Policy(mode=mb.UNIFORM)

    def step(policy, profile=False):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        M = mb.BlockJacobi(A, p.block_ptr, policy)
        e1.record()
        res = solver.solve(A, M, b, tol=tol, maxit=maxit, profile=profile)
        e2.record()
        return M, res, (e0, e1, e2)

    def timed(policy, k):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        runs = [step(policy) for _ in range(k)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        setup = [r[2][0].elapsed_time(r[2][1]) for r in runs]
        solve = [r[2][1].elapsed_time(r[2][2]) for r in runs]
        return (t1 - t0) * 1e3 / k, float(np.median(setup)), float(np.median(solve)), runs[-1]

    if args.calibrate:
        src = torch.empty(2 ** 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy: 1 GiB read, 1 GiB written")
    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step(pol16)
    step(pol64)
    log(f"timing {args.steps} steps, FP16 block storage")
    ms16, setup16, solve16, (M16, r16, _) = timed(pol16, args.steps)
    log(f"fp16: {ms16:.2f} ms/step ({r16.iters} iterations)")
    log(f"timing {args.steps} steps, FP64 block storage")
    ms64, setup64, solve64, (M64, r64, _) = timed(pol64, args.steps)
    log(f"fp64: {ms64:.2f} ms/step ({r64.iters} iterations)")

    # FP64 check of the returned solutions
    S = p.A.to_scipy()
    bn = float(np.linalg.norm(p.b))
    true16 = float(np.linalg.norm(p.b - S @ r16.x.cpu().numpy()) / bn)
    true64 = float(np.linalg.norm(p.b - S @ r64.x.cpu().numpy()) / bn)

    # profile pass: per-kernel event timing of the same solve
    log("profile pass")
    _, rp16, _ = step(pol16, profile=True)
    info16 = M16.info()
    ntiles = info16["ntiles"]
    kb = {"spmv": spmv_bytes(n, nnz), "apply": apply_bytes(n, nb, ntiles, info16["low_bytes"])}
    kern = {}
    for name in ("spmv", "apply"):
        tot, cnt = rp16.kernel_ms[name]
        avg_ms = tot / max(1, cnt)
        kern[name] = {"launches": cnt, "avg_us": avg_ms * 1e3, "bytes": kb[name],
                      "gbs": kb[name] / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None}
    dom = max(kern, key=lambda k: kern[k]["avg_us"] * kern[k]["launches"])
    dk = kern[dom]
    iter_bytes = kb["spmv"] + kb["apply"]
    iter_us16 = solve16 * 1e3 / max(1, r16.iters)
    roofline = {"bound": "hbm", "achieved": dk["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dk["gbs"] / HBM_PEAK_GBS, "traffic": None, "kernel": f"{dom}_kernel",
                "bytes_per_launch": dk["bytes"], "avg_launch_us": dk["avg_us"]}
    pair_gbs = iter_bytes / ((kern["spmv"]["avg_us"] + kern["apply"]["avg_us"]) * 1e-6) / 1e9

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")
        cpu = cpu_baseline(p, r16.iters)

    line = {
        "metric": "PCG time-to-1e-10 residual + BJAC-apply HBM GB/s, mixed/learned vs FP64",
        "value": ms16, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms16, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "apply_arith": "fp16-stored block inverses, f32 accumulation", "data": "synthetic",
        "config": {"workload": f"diff3d_loguniform_{args.N}^3_b32", "n": n, "nnz": nnz, "blocks": nb,
                   "block_rows": 32, "precision_map": "fp16 fixed (fMP)", "tol": tol, "seed": 0},
        "iters": r16.iters, "iters_fp64": r64.iters, "delay_iters": r16.iters - r64.iters,
        "setup_ms": setup16, "solve_ms": solve16, "fp64_ms_per_step": ms64, "fp64_setup_ms": setup64,
        "fp64_solve_ms": solve64, "speedup_vs_fp64": ms64 / ms16,
        "true_relres": true16, "true_relres_fp64": true64,
        "us_per_iter": iter_us16, "bytes_per_iter": iter_bytes,
        "iter_gbs": iter_bytes / (iter_us16 * 1e-6) / 1e9,
        "apply_spmv_gbs": pair_gbs, "apply_spmv_frac": pair_gbs / HBM_PEAK_GBS,
        "kernels": kern, "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
