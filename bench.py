#!/usr/bin/env python3
"""Benchmark of mixed-precision block-Jacobi PCG on one MI355X.

Default workload (the largest single system): 3D anisotropic diffusion on a
192^3 grid (n = 7,077,888, nnz = 49,324,032), K = diag(1e3, 1, 1) times a
coefficient of 1e4 on 16 random subcubes and 1 elsewhere, contiguous row
blocks of 48, RHS U[-1,1] (held-out seed 100), x0 = 0, stop at
||r||/||b|| <= 1e-10 with an FP64 check of the true residual. One step =
block-Jacobi setup (extract, FP64 invert, features, precision map, round +
pack) plus the PCG solve, with A and b already resident in HBM.

The headline value is the time to solution with the precision map the
learned selector picks (the network is trained first, untimed, on labels the
solver generates on the 2D Poisson and 3D log-uniform diffusion families);
the per-block rule, fixed FP16 and FP64 maps are timed beside it over fewer
steps. Every map stores each block's upper 16 x 16 quarters (the inverse is
symmetric). Iteration counts are reported against the oracle's, stored by
tests/golden/make_oracle_iters.py. A profile pass times each kernel with HIP
events on the stream it runs on and reports the dominant kernel against the
8 TB/s HBM roofline. The CPU oracle is timed on the host's cores. The 128^3
log-uniform workload (blocks of 32) is timed as extra keys.

Other workloads (each prints its own line of the same form):
  --workload diff3d    128^3 log-uniform diffusion (10^U(-2,2)), blocks of
                       32: FP16 vs FP64 maps, symmetric storage
  --workload batched   256 independent 7-point systems, edges U{32..96},
                       1-8 right-hand sides each, blocks from {16,32,48,64};
                       FP16 block storage vs FP64 (and FP16 band storage),
                       autotuned launch shape
  --workload aniso     160^3 anisotropic (1e3) diffusion with 1e4 jumps on
                       16 random subcubes, blocks of 48: per-block rule vs
                       FP16 and FP64 storage; --axis yz puts the strong axes
                       across the row blocks (the paper's Ani(s) orientation)
  --workload rhd       synthetic radiation-diffusion-like systems at 128^3:
                       coupled 3T (eq. 4-3, 6.3M rows) and 1T, stored
                       inverses and paper mode, and a P_diag sweep (Sec. 4.5.2)
  --workload band      128^3 log-uniform diffusion, blocks of 32: full vs
                       band-truncated storage of the inverses (diagonals
                       kept down to the format's unit roundoff), FP64 /
                       FP32 / FP16, and symmetric storage (three of the
                       four 16 x 16 quarters), FP64 / FP16
  --workload paper     the paper's own setting (Sec. 4.2, Table 4.2): 128^3
                       Diff3D-Const / Dis(1000) / Ani(s), f = 1, 32 slabs,
                       BJAC(k=2, t=2) uniform FP64 vs fMP FP32 vs aMP(hl/lh)

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload W]
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


def index_bytes(A, codes=True):
    """Bytes per column index the PCG SpMV reads: 1 when the matrix has at
    most 256 distinct offsets col - row (the solver's 8-bit dictionary codes;
    codes=False for the batched SpMV, which has none), else 2 when every entry
    lies within 32767 rows of its row (16-bit offsets), else 4 (the CSR's own
    indices)."""
    import numpy as np
    rows = np.repeat(np.arange(A.n, dtype=np.int64), np.diff(A.row_ptr.astype(np.int64)))
    d = A.col_idx.astype(np.int64) - rows
    if codes and A.nnz and len(np.unique(d)) <= 256:
        return 1
    far = np.max(np.abs(d)) if A.nnz else 0
    return 2 if far <= 32767 else 4


def value_bytes(A, ib):
    """Bytes per matrix value the PCG SpMV reads: 1 when the column offsets are
    8-bit coded (ib == 1) and the matrix holds at most 256 distinct values
    (bitwise; none equal to the dictionary's empty key), the solver's 8-bit
    value codes, else 8."""
    import numpy as np
    if ib != 1 or not A.nnz:
        return 8
    bits = np.ascontiguousarray(A.val, dtype=np.float64).view(np.uint64)
    u = np.unique(bits)
    return 1 if len(u) <= 256 and not np.any(u == np.uint64(0x7FF4DEADBEEF0001)) else 8


def spmv_bytes(n, nnz, ib=4, vb=8):
    """Algorithmic bytes of one SpMV launch with the folded p update: CSR values
    (vb bytes each; 2 KiB of dictionary with 8-bit value codes) and column
    indices (ib bytes each; 1 KiB of dictionary with 8-bit codes), row
    pointers, z and p_old read once, p_new and q written."""
    return ((vb + ib) * nnz + 4 * (n + 1) + 32 * n + (1024 if ib == 1 else 0)
            + (2048 if vb == 1 else 0))


def apply_bytes(n, nb, ntiles, stored_bytes, band=False):
    """Algorithmic bytes of one fused update + apply launch: the stored block
    inverses, per-block metadata (offset 8, scale 8, tag 1, row start 4, and
    the half-bandwidth 1 for band storage), the tile list, and x, r
    read+written, p, q read, z written."""
    return stored_bytes + (22 if band else 21) * nb + 4 * (ntiles + 1) + 56 * n


METRIC = "PCG time-to-1e-10 residual + BJAC-apply HBM GB/s, mixed/learned vs FP64"
# every timed solve checks ||b - A x|| / ||b|| <= tol in FP64 on the device and
# restarts from the true residual (at most this many times) when it is above
VERIFY = 3

# HBM bytes per launch of the per-iteration kernels, from rocprofv3
# FETCH_SIZE / WRITE_SIZE runs (profiles/, scaled by a 1 GiB copy), keyed by
# workload and kernel. Valid only for the kernel sources they were measured
# on: reported when the digest of those sources matches, null otherwise.
TRAFFIC = {
    "heldout_192:apply": ("54bc83f21c0e63765b996224c9206b9d97d045b6fd4c2f506a7dd90b3d44f951", 885363386),
    "heldout_192:spmv": ("54bc83f21c0e63765b996224c9206b9d97d045b6fd4c2f506a7dd90b3d44f951", 539915313),
}
TRAFFIC_SOURCES = ("solve.hip", "device_util.hpp", "internal.hpp")


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2407_15973_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(key):
    e = TRAFFIC.get(key)
    return e[1] if e is not None and e[0] == sources_digest() else None


def calibration_copy():
    """One device-to-device copy of 1 GiB (read 1 GiB, write 1 GiB): the
    reference dispatch that scales rocprofv3's FETCH_SIZE / WRITE_SIZE."""
    import torch
    src = torch.empty(2 ** 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()
    log("calibration copy: 1 GiB read, 1 GiB written")


def stream_ceilings(dev, mib=512):
    """Achievable streaming rates of this GPU for the read:write mixes of the
    hot kernels, measured with the library's streaming probe
    (bjac_stream_probe) on eight or fewer `mib`-MiB FP64 streams (several GiB
    in all, far beyond the 256 MiB Infinity Cache): read only, write only,
    copy (1:1), 4 reads : 1 write (the fused update + application reads about
    four bytes per byte written) and 6:1 (the SpMV). Each mix takes the best
    of a few launch shapes (grid of 1024 to 8192 workgroups, 1 to 4 accesses
    per lane and stream in flight), each timed as the median of 3 launches;
    bytes = streams x stream size."""
    import torch

    from paper_2407_15973_amd import binding as mb
    n = mib * (2 ** 20) // 8
    bufs = [torch.ones(n, dtype=torch.float64, device=dev) for _ in range(8)]
    sink = torch.empty(8192 * 256, dtype=torch.float64, device=dev)
    out, shape = {}, {}
    for name, ni, no in (("read", 8, 0), ("write", 0, 2), ("copy", 1, 1), ("r4w1", 4, 1), ("r6w1", 6, 1)):
        ins, outs = bufs[:ni], bufs[ni:ni + no] if ni else bufs[:no]
        best = 0.0
        for grid in (1024, 2048, 4096, 8192):
            for unroll in (1, 2, 4):
                mb.stream_probe(ins, outs, grid=grid, unroll=unroll, sink=sink)
                ts = []
                for _ in range(3):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    mb.stream_probe(ins, outs, grid=grid, unroll=unroll, sink=sink)
                    e1.record()
                    e1.synchronize()
                    ts.append(e0.elapsed_time(e1) * 1e-3)
                ts.sort()
                rate = (ni + no) * n * 8 / ts[1] / 1e9
                if rate > best:
                    best, shape[name] = rate, (grid, unroll)
        out[name] = best
    del bufs, sink
    torch.cuda.empty_cache()
    out["shapes"] = shape
    return out


def bench_diff3d(args):
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
    # both maps store each block's H00, H01 and H11 (the inverse is symmetric)
    pol16 = mb.Policy(mode=mb.FIXED, low=mb.FP16, storage=mb.STORE_SYM)
    pol64 = mb.Policy(mode=mb.UNIFORM, storage=mb.STORE_SYM)

    def step(policy, profile=False):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        M = mb.BlockJacobi(A, p.block_ptr, policy)
        e1.record()
        res = solver.solve(A, M, b, tol=tol, maxit=maxit, profile=profile, verify=0 if profile else VERIFY)
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
    ib = index_bytes(p.A)
    kb = {"spmv": spmv_bytes(n, nnz, ib, value_bytes(p.A, ib)), "apply": apply_bytes(n, nb, ntiles, info16["low_bytes"])}
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
                "frac": dk["gbs"] / HBM_PEAK_GBS,
                "traffic": measured_traffic(f"diff3d_128:{dom}") if args.N == 128 else None, "kernel": f"{dom}_kernel",
                "bytes_per_launch": dk["bytes"], "avg_launch_us": dk["avg_us"]}
    pair_gbs = iter_bytes / ((kern["spmv"]["avg_us"] + kern["apply"]["avg_us"]) * 1e-6) / 1e9

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")
        cpu = cpu_baseline_full(p, r16.iters)
    ceil = stream_ceilings(dev)
    mix = ceil["r6w1"] if dom == "spmv" else ceil["r4w1"]
    roofline["mix_ceiling_gbs"] = mix
    roofline["frac_of_mix_ceiling"] = dk["gbs"] / mix

    line = {
        "metric": METRIC,
        "value": ms16, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms16, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "apply_arith": "fp16-stored block inverses, f32 accumulation", "data": "synthetic",
        "config": {"workload": f"diff3d_loguniform_{args.N}^3_b32", "n": n, "nnz": nnz, "blocks": nb,
                   "block_rows": 32, "precision_map": "fp16 fixed (fMP)",
                   "storage": "symmetric (H00, H01, H11 of each block)", "tol": tol, "seed": 0},
        "iters": r16.iters, "iters_fp64": r64.iters, "delay_iters": r16.iters - r64.iters,
        "restarts": r16.restarts, "restarts_fp64": r64.restarts, "true_relres_device": r16.true_relres,
        "setup_ms": setup16, "solve_ms": solve16, "fp64_ms_per_step": ms64, "fp64_setup_ms": setup64,
        "fp64_solve_ms": solve64, "speedup_vs_fp64": ms64 / ms16,
        "true_relres": true16, "true_relres_fp64": true64,
        "us_per_iter": iter_us16, "bytes_per_iter": iter_bytes,
        "iter_gbs": iter_bytes / (iter_us16 * 1e-6) / 1e9,
        "apply_spmv_gbs": pair_gbs, "apply_spmv_frac": pair_gbs / HBM_PEAK_GBS,
        "kernels": kern, "roofline": roofline, "cpu_baseline": cpu, "stream_ceilings_gbs": ceil,
    }
    return line



# ------------------------------------------------------------- batched solves
def batched_spmv_bytes(n, nnz, veclen, ib=4):
    """One batched SpMV launch: CSR once (ib bytes per column index), and per
    (row, column) z and p_old read, p_new and q written."""
    return (8 + ib) * nnz + 4 * (n + 1) + 32 * veclen


def batched_apply_bytes(nb, stored_bytes, veclen):
    """One batched update + apply launch: stored inverses and block metadata
    once, and per (row, column) x, r read and written, p, q read, z written."""
    return stored_bytes + 21 * nb + 56 * veclen


def cpu_baseline_batched(st, col_iters, nsample=2, budget_iters=8):
    """Oracle on the first ``nsample`` systems, thread pools set to the host's
    core count: block setup (FP16 storage) and a few PCG iterations of every
    column; scaled by rows (setup) and by rows x iterations summed over every
    column of the batch (solve). `cores` is the oracle's CPU time over its
    wall time."""
    import resource

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import pcg as OP
    from oracle import precision as OPr
    from paper_2407_15973_amd import gen
    rows_s = np.diff(st.sys_row).astype(np.int64)
    t_setup = t_iter = 0.0
    row_sample = row_iter_sample = 0
    ncores, model = host_cores()
    ru0 = resource.getrusage(resource.RUSAGE_SELF)
    w0 = time.perf_counter()
    with threadpool_limits(limits=ncores):
        for s in range(nsample):
            r0, r1 = int(st.sys_row[s]), int(st.sys_row[s + 1])
            k0, k1 = (int(np.searchsorted(st.block_ptr, v)) for v in (r0, r1))
            bp = (st.block_ptr[k0:k1 + 1] - r0).astype(np.int32)
            a, b = int(st.A.row_ptr[r0]), int(st.A.row_ptr[r1])
            sub = gen.CSR(r1 - r0, (st.A.row_ptr[r0:r1 + 1] - a).astype(np.int32),
                          (st.A.col_idx[a:b] - r0).astype(np.int32), st.A.val[a:b])
            t0 = time.perf_counter()
            M = OP.BJAC(sub, bp, np.full(len(bp) - 1, OPr.FP16, np.uint8))
            t1 = time.perf_counter()
            S = sub.to_scipy()
            m = int(st.sys_m[s])
            B = st.b[st.system_slice(s)].reshape(r1 - r0, m)
            its = 0
            for c in range(m):
                its += OP.pcg(lambda v: S @ v, B[:, c], M.low, 0.0, budget_iters).iters
            t2 = time.perf_counter()
            t_setup += t1 - t0
            t_iter += t2 - t1
            row_sample += r1 - r0
            row_iter_sample += (r1 - r0) * its
    col_rows = np.repeat(rows_s, st.sys_m)
    total_row_iters = float(np.sum(col_rows * np.asarray(col_iters, dtype=np.int64)))
    est = t_setup / row_sample * rows_s.sum() + t_iter / row_iter_sample * total_row_iters
    ru1 = resource.getrusage(resource.RUSAGE_SELF)
    used = (ru1.ru_utime + ru1.ru_stime - ru0.ru_utime - ru0.ru_stime) / max(1e-9, time.perf_counter() - w0)
    return {"value": est * 1e3, "unit": "ms", "cores": max(1, round(used)), "kind": "oracle",
            "host_cores": ncores, "host_cpu": model, "threads_allowed": ncores,
            "sample": f"oracle setup + {budget_iters} PCG iterations per column on the first {nsample} systems "
                      f"({row_sample} rows, {t_setup + t_iter:.1f} s), scaled by rows (setup) and by "
                      f"rows x iterations of every column (solve)"}


def bench_batched(args):
    import numpy as np
    import torch

    from paper_2407_15973_amd import autotune
    from paper_2407_15973_amd import binding as mb
    from paper_2407_15973_amd import gen

    dev = "cuda:0"
    log(f"building the batch ({args.nsys} systems)")
    st = gen.stack_batch(gen.config4(seed=0, nsys=args.nsys))
    n, nnz, nb = st.A.n, st.A.nnz, len(st.block_ptr) - 1
    veclen = int(st.b.size)
    log(f"n = {n}, nnz = {nnz}, blocks = {nb}, columns = {int(st.sys_m.sum())}, vector entries = {veclen}")
    A = mb.DeviceCSR(st.A, dev)
    b = torch.as_tensor(st.b, device=dev)
    tol, maxit = 1e-10, 5000
    pol16 = mb.Policy(mode=mb.FIXED, low=mb.FP16)
    pol64 = mb.Policy(mode=mb.UNIFORM)
    M0 = mb.BlockJacobi(A, st.block_ptr, pol16)
    bs = mb.BatchSolver(A, M0, st.sys_row, st.sys_m)
    log("autotuning the launch shape")
    cfg, entry = autotune.tuned_cfg(bs, b)
    log(f"tuned (spmv_grab, wg_per_cu, spmv_wg_per_cu, apply_rows) = {cfg}: {entry['ms_per_iter']}")
    del M0

    def step(policy, profile=False):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        M = mb.BlockJacobi(A, st.block_ptr, policy)
        e1.record()
        bs.M = M
        res = bs.solve(b, tol=tol, maxit=maxit, cfg=cfg, profile=profile)
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

    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step(pol16)
    log(f"timing {args.steps} steps, FP16 block storage")
    ms16, setup16, solve16, (M16, r16, _) = timed(pol16, args.steps)
    log(f"fp16: {ms16:.1f} ms/step (max {r16.iters} iterations)")
    log(f"timing {args.steps} steps, FP64 block storage")
    ms64, setup64, solve64, (M64, r64, _) = timed(pol64, args.steps)
    log(f"fp64: {ms64:.1f} ms/step (max {r64.iters} iterations)")
    polb = mb.Policy(mode=mb.FIXED, low=mb.FP16, storage=mb.STORE_BAND)
    log(f"timing {args.steps} steps, FP16 band storage")
    msb, setupb, solveb, (Mb, rb, _) = timed(polb, args.steps)
    log(f"fp16 band: {msb:.1f} ms/step (max {rb.iters} iterations)")

    # FP64 check of the returned solutions on a sample of systems
    x16 = r16.x.cpu().numpy()
    worst = 0.0
    for s in range(0, len(st.sys_m), max(1, len(st.sys_m) // 16)):
        r0, r1 = int(st.sys_row[s]), int(st.sys_row[s + 1])
        a, bb = int(st.A.row_ptr[r0]), int(st.A.row_ptr[r1])
        sub = gen.CSR(r1 - r0, (st.A.row_ptr[r0:r1 + 1] - a).astype(np.int32),
                      (st.A.col_idx[a:bb] - r0).astype(np.int32), st.A.val[a:bb]).to_scipy()
        m = int(st.sys_m[s])
        X = x16[st.system_slice(s)].reshape(r1 - r0, m)
        B = st.b[st.system_slice(s)].reshape(r1 - r0, m)
        worst = max(worst, float(np.max(np.linalg.norm(B - sub @ X, axis=0) / np.linalg.norm(B, axis=0))))

    log("profile pass")
    _, rp16, _ = step(pol16, profile=True)
    info16 = M16.info()
    kb = {"spmv": batched_spmv_bytes(n, nnz, veclen, index_bytes(st.A, codes=False)), "apply": batched_apply_bytes(nb, info16["low_bytes"], veclen)}
    kern = {}
    for name in ("spmv", "apply"):
        tot, cnt = rp16.kernel_ms[name]
        avg_ms = tot / max(1, cnt)
        kern[name] = {"launches": cnt, "avg_us": avg_ms * 1e3, "bytes": kb[name],
                      "gbs": kb[name] / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None}
    tot, cnt = rp16.kernel_ms["reduce"]
    kern["reduce"] = {"launches": cnt, "avg_us": tot / max(1, cnt) * 1e3}
    dom = max(("spmv", "apply"), key=lambda k: kern[k]["avg_us"])
    dk = kern[dom]
    roofline = {"bound": "hbm", "achieved": dk["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dk["gbs"] / HBM_PEAK_GBS, "traffic": None,
                "kernel": "bspmv_kernel" if dom == "spmv" else "bapply_kernel",
                "bytes_per_launch": dk["bytes"], "avg_launch_us": dk["avg_us"]}
    iter_bytes = kb["spmv"] + kb["apply"]
    pair_gbs = iter_bytes / ((kern["spmv"]["avg_us"] + kern["apply"]["avg_us"]) * 1e-6) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")
        cpu = cpu_baseline_batched(st, r16.col_iters)
    return {
        "metric": METRIC, "value": ms16, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms16, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "apply_arith": "fp16-stored block inverses, f32 matrix-core products", "data": "synthetic",
        "config": {"workload": f"batched_{len(st.sys_m)}sys_diff3d_edges32-96_rhs1-8", "n": n, "nnz": nnz,
                   "blocks": nb, "columns": int(st.sys_m.sum()), "vector_entries": veclen,
                   "block_rows": "U{16,32,48,64}", "precision_map": "fp16 fixed", "tol": tol, "seed": 0,
                   "tuned": dict(zip(("spmv_grab", "wg_per_cu", "spmv_wg_per_cu", "apply_rows"), cfg))},
        "iters_max": r16.iters, "iters_mean": float(np.mean(r16.col_iters)),
        "iters_fp64_max": r64.iters, "iters_fp64_mean": float(np.mean(r64.col_iters)),
        "status": r16.status, "status_fp64": r64.status,
        "setup_ms": setup16, "solve_ms": solve16, "fp64_ms_per_step": ms64, "fp64_setup_ms": setup64,
        "fp64_solve_ms": solve64, "speedup_vs_fp64": ms64 / ms16, "true_relres_sampled_max": worst,
        "fp16_band_ms_per_step": msb, "fp16_band_setup_ms": setupb, "fp16_band_solve_ms": solveb,
        "fp16_band_iters_max": rb.iters, "fp16_band_status": rb.status,
        "fp16_band_stored_bytes": Mb.info()["low_bytes"], "fp16_stored_bytes": M16.info()["low_bytes"],
        "bytes_per_iter": iter_bytes, "apply_spmv_gbs": pair_gbs, "apply_spmv_frac": pair_gbs / HBM_PEAK_GBS,
        "kernels": kern, "roofline": roofline, "cpu_baseline": cpu,
        "autotune_ms_per_iter": entry["ms_per_iter"],
    }


# ------------------------------------------- per-block rule / learned selector
def train_selector(dev):
    """Selector trained on labels the solver generates on the 2D Poisson and
    3D diffusion families (selector.training_problems: seeds 0-1, 32^3 grids
    at coefficient contrasts 10^0 to 10^5)."""
    import numpy as np

    from paper_2407_15973_amd import binding as mb
    from paper_2407_15973_amd import selector as sel
    F, Y = [], []
    for p in sel.training_problems():
        ls = sel.make_labels(mb.DeviceCSR(p.A, dev), p.block_ptr, p.b, tol=p.tol, maxit=p.maxit)
        F.append(ls.features)
        Y.append(ls.labels)
    return sel.train(np.concatenate(F), np.concatenate(Y), steps=400, lr=3e-3)


def oracle_golden(workload, pmap):
    """The oracle's iteration count and sampled solution at a benchmark size,
    as stored by tests/golden/make_oracle_iters.py (which calls only oracle/);
    None when not stored."""
    path = os.path.join(ROOT, "tests", "golden", f"oracle_iters_{workload}_{pmap}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def x_err_vs_oracle(g, x):
    """||x - x_oracle|| / ||x_oracle|| on the stored oracle run's sample rows
    (None when no run is stored)."""
    import numpy as np
    if g is None:
        return None
    rows = np.asarray(g["sample_rows"], dtype=np.int64)
    xo = np.asarray(g["x_sample"])
    return float(np.linalg.norm(x[rows] - xo) / np.linalg.norm(xo))


def host_cores():
    """Physical cores of the host (lscpu: cores per socket x sockets), else
    the logical CPU count."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        kv = {}
        for line in out.splitlines():
            k, _, v = line.partition(":")
            kv[k.strip()] = v.strip()
        return int(kv["Core(s) per socket"]) * int(kv["Socket(s)"]), kv.get("Model name", "")
    except Exception:
        return os.cpu_count() or 1, ""


def cpu_baseline_full(p, iters_total, reps=3, iters_sample=3):
    """The oracle as it stands, on the host with its thread pools set to the
    host's core count: the FP64 setup of every block with FP16 storage, timed
    once, then `reps` runs of `iters_sample` PCG iterations of the same
    problem; the solve is the median time per iteration times the full
    solve's iteration count. `cores` is the CPU time the oracle used over its
    wall time (its NumPy/SciPy work is mostly single-threaded)."""
    import resource

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import pcg as OP
    from oracle import precision as OPr
    ncores, model = host_cores()

    def cpu_s():
        r = resource.getrusage(resource.RUSAGE_SELF)
        return r.ru_utime + r.ru_stime

    with threadpool_limits(limits=ncores):
        c0, t0 = cpu_s(), time.perf_counter()
        nb = len(p.block_ptr) - 1
        M = OP.BJAC(p.A, p.block_ptr, np.full(nb, OPr.FP16, np.uint8))
        S = p.A.to_scipy()
        t1 = time.perf_counter()
        per = []
        for _ in range(reps):
            ta = time.perf_counter()
            res = OP.pcg(lambda v: S @ v, p.b, M.low, 0.0, iters_sample)
            per.append((time.perf_counter() - ta) / max(1, res.iters))
        c1, t2 = cpu_s(), time.perf_counter()
    setup_s, iter_s = t1 - t0, float(np.median(per))
    used = (c1 - c0) / max(1e-9, t2 - t0)
    return {"value": 1e3 * (setup_s + iter_s * iters_total), "unit": "ms", "cores": max(1, round(used)),
            "kind": "oracle", "host_cores": ncores, "host_cpu": model, "threads_allowed": ncores,
            "setup_ms": 1e3 * setup_s, "solve_ms": 1e3 * iter_s * iters_total, "ms_per_iter": 1e3 * iter_s,
            "sample": f"oracle setup of all {nb} blocks (Cholesky inverse, FP16 storage) timed once "
                      f"({setup_s:.1f} s); PCG iterations timed in {reps} runs of {iters_sample} "
                      f"(median {1e3 * iter_s:.0f} ms per iteration) and multiplied by the full solve's "
                      f"{iters_total} iterations; CPU time / wall time {used:.2f}"}


def bench_policies(args):
    """Precision maps on one large anisotropic jump-coefficient problem, every
    map with symmetric storage of the block inverses. ``selector`` (the
    default workload): the held-out 192^3 problem, the learned selector
    (trained first, untimed, on labels from the solver's own runs) timed over
    the requested steps, the per-block rule, fixed FP16 and FP64 beside it over
    fewer steps; ``aniso``: the 160^3 problem, the rule as the headline."""
    import numpy as np
    import torch

    from paper_2407_15973_amd import binding as mb
    from paper_2407_15973_amd import gen

    dev = "cuda:0"
    selector_mode = args.workload == "selector"
    gkey = "heldout_192" if selector_mode else "aniso_160"
    log("building the workload")
    p = (gen.config5_eval(seed=100, N=args.N) if selector_mode else
         gen.aniso_jump_problem(seed=0, N=args.N, name="diff3d_aniso1e3yz_jump1e4", ratio=1e3, strong="yz")
         if args.axis == "yz" else gen.config3(seed=0, N=args.N))
    if args.axis == "yz":
        gkey = None
    n, nnz, nb = p.A.n, p.A.nnz, len(p.block_ptr) - 1
    A = mb.DeviceCSR(p.A, dev)
    b = torch.as_tensor(p.b, device=dev)
    solver = mb.Solver(n, dev)
    sym = dict(storage=mb.STORE_SYM)
    pols = {"fp64": mb.Policy(mode=mb.UNIFORM, **sym), "fp16": mb.Policy(mode=mb.FIXED, low=mb.FP16, **sym),
            "rule": mb.Policy(mode=mb.RULE, **sym)}
    head = "rule"
    if selector_mode:
        log("training the selector (untimed)")
        t0 = time.perf_counter()
        sel = train_selector(dev)
        log(f"trained in {time.perf_counter() - t0:.1f} s")
        pols = {"learned": mb.Policy(mode=mb.LEARNED, mlp_blob=sel.blob, **sym), **pols}
        head = "learned"
    else:
        pols = {"rule": pols["rule"], "fp16": pols["fp16"], "fp64": pols["fp64"]}
    cmp_steps = min(args.steps, args.cmp_steps)
    if cmp_steps < 1:   # profiling runs: the headline map only
        pols = {head: pols[head]}

    def step(policy, profile=False):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        M = mb.BlockJacobi(A, p.block_ptr, policy)
        e1.record()
        res = solver.solve(A, M, b, tol=p.tol, maxit=p.maxit, profile=profile, verify=0 if profile else VERIFY)
        e2.record()
        return M, res, (e0, e1, e2)

    S = p.A.to_scipy()
    bn = float(np.linalg.norm(p.b))
    g64 = oracle_golden(gkey, "fp64") if gkey else None
    rows = {}
    for name, pol in pols.items():
        k = args.steps if name == head else cmp_steps
        for _ in range(args.warmup if name == head else 1):
            step(pol)
        log(f"timing {k} steps, {name}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        runs = [step(pol) for _ in range(k)]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / k
        M, res, ev = runs[-1]
        info = M.info()
        x = res.x.cpu().numpy()
        g = oracle_golden(gkey, name) if (gkey and name != "learned") else None
        if gkey and name == "learned":
            # a learned map that equals a fixed map (every block in one
            # format) is compared with the oracle's count for that map
            fixed = {(0, 0, 0, 1): "fp16", (0, 1, 0, 0): "fp32", (1, 0, 0, 0): "fp64"}
            hist = tuple(int(v > 0) for v in info["blocks_per_prec"])
            g = oracle_golden(gkey, fixed[hist]) if hist in fixed else None
        rows[name] = {"ms_per_step": ms, "steps": k, "iters": res.iters, "status": res.status,
                      "restarts": res.restarts, "true_relres_device": res.true_relres,
                      "true_relres": float(np.linalg.norm(p.b - S @ x) / bn),
                      "setup_ms": float(np.median([r[2][0].elapsed_time(r[2][1]) for r in runs])),
                      "solve_ms": float(np.median([r[2][1].elapsed_time(r[2][2]) for r in runs])),
                      "blocks_per_prec": info["blocks_per_prec"], "stored_bytes": info["low_bytes"],
                      "iters_oracle_same_map": g["iters"] if g else None,
                      "delay_vs_oracle_fp64": res.iters - g64["iters"] if g64 else None,
                      "x_rel_err_vs_oracle_fp64": x_err_vs_oracle(g64, x)}
        log(f"{name}: {ms:.1f} ms/step, {res.iters} iterations (oracle FP64 "
            f"{g64['iters'] if g64 else '-'}), map {info['blocks_per_prec']}")
        del runs, M

    log("profile pass")
    M, rp, _ = step(pols[head], profile=True)
    info = M.info()
    ib = index_bytes(p.A)
    kb = {"spmv": spmv_bytes(n, nnz, ib, value_bytes(p.A, ib)), "apply": apply_bytes(n, nb, info["ntiles"], info["low_bytes"])}
    kern = {}
    for name in ("spmv", "apply"):
        tot, cnt = rp.kernel_ms[name]
        avg_ms = tot / max(1, cnt)
        kern[name] = {"launches": cnt, "avg_us": avg_ms * 1e3, "bytes": kb[name],
                      "gbs": kb[name] / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None}
    dom = max(kern, key=lambda k: kern[k]["avg_us"] * kern[k]["launches"])
    dk = kern[dom]
    iter_bytes = kb["spmv"] + kb["apply"]
    pair_gbs = iter_bytes / ((kern["spmv"]["avg_us"] + kern["apply"]["avg_us"]) * 1e-6) / 1e9
    traffic = measured_traffic(f"{gkey}:{dom}") if gkey else None
    roofline = {"bound": "hbm", "achieved": dk["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dk["gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                "traffic_source": ("rocprofv3 FETCH_SIZE and WRITE_SIZE runs of the same kernel sources "
                                   f"(profiles/hbm_traffic_heldout_192_b48.md), not measured in this run")
                if traffic else None,
                "kernel": f"{dom}_kernel", "bytes_per_launch": dk["bytes"], "avg_launch_us": dk["avg_us"]}
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on the host cores)")
        cpu = cpu_baseline_full(p, rows[head]["iters"])
    hv = rows[head]
    del M, A, b, solver
    torch.cuda.empty_cache()
    extra = bench_config2_keys(args) if (selector_mode and not args.no_config2) else None
    small = bench_config1_keys() if (selector_mode and not args.no_config2) else None
    ceil = stream_ceilings(dev)
    mix = ceil["r6w1"] if dom == "spmv" else ceil["r4w1"]
    roofline["mix_ceiling_gbs"] = mix
    roofline["frac_of_mix_ceiling"] = dk["gbs"] / mix
    return {
        "metric": METRIC, "value": hv["ms_per_step"], "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": hv["ms_per_step"], "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "apply_arith": "per-block FP64/FP32/FP16-stored block inverses (symmetric storage), "
                       "f32 accumulation for reduced blocks",
        "config": {"workload": p.name, "n": n, "nnz": nnz, "blocks": nb, "block_rows": 48,
                   "precision_map": head, "storage": "symmetric (upper 16x16 quarters of each block)",
                   "tol": p.tol, "seed": 100 if selector_mode else 0},
        "iters": hv["iters"], "iters_oracle_fp64": g64["iters"] if g64 else None,
        "delay_vs_oracle_fp64": hv["delay_vs_oracle_fp64"],
        "true_relres": hv["true_relres"], "setup_ms": hv["setup_ms"], "solve_ms": hv["solve_ms"],
        "speedup_vs_fp64": rows["fp64"]["ms_per_step"] / hv["ms_per_step"] if "fp64" in rows else None,
        "speedup_vs_rule": rows["rule"]["ms_per_step"] / hv["ms_per_step"] if "rule" in rows else None,
        "speedup_vs_fp16": rows["fp16"]["ms_per_step"] / hv["ms_per_step"] if "fp16" in rows else None,
        "policies": rows, "comparison_steps": cmp_steps,
        "us_per_iter": hv["solve_ms"] * 1e3 / max(1, hv["iters"]), "bytes_per_iter": iter_bytes,
        "apply_spmv_gbs": pair_gbs, "apply_spmv_frac": pair_gbs / HBM_PEAK_GBS,
        "kernels": kern, "roofline": roofline, "cpu_baseline": cpu, "stream_ceilings_gbs": ceil,
        "diff3d_128": extra, "poisson_64": small,
    }


def bench_config1_keys():
    """The 2D Poisson 64x64 workload (4,096 rows, blocks of 64, tol 1e-8) as
    extra keys of the default line: latency-bound (a 2.7 MB working set), so
    microseconds per iteration and per solve, FP64 map, against the oracle's
    iteration count."""
    import numpy as np
    import torch

    from paper_2407_15973_amd import binding as mb
    from paper_2407_15973_amd import gen

    dev = "cuda:0"
    p = gen.config1(seed=0)
    A = mb.DeviceCSR(p.A, dev)
    b = torch.as_tensor(p.b, device=dev)
    solver = mb.Solver(p.A.n, dev)
    M = mb.BlockJacobi(A, p.block_ptr, mb.Policy(mode=mb.UNIFORM))
    for _ in range(3):
        solver.solve(A, M, b, tol=p.tol, maxit=p.maxit)
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        res = solver.solve(A, M, b, tol=p.tol, maxit=p.maxit)
    torch.cuda.synchronize()
    us = (time.perf_counter() - t0) * 1e6 / reps
    ts = time.perf_counter()
    for _ in range(reps):
        Ms = mb.BlockJacobi(A, p.block_ptr, mb.Policy(mode=mb.UNIFORM))
        rs = solver.solve(A, Ms, b, tol=p.tol, maxit=p.maxit)
    torch.cuda.synchronize()
    us_step = (time.perf_counter() - ts) * 1e6 / reps
    S = p.A.to_scipy()
    g = oracle_golden("poisson_64", "fp64")
    log(f"64x64 Poisson: {us:.0f} us per solve, {res.iters} iterations")
    return {"workload": p.name, "n": p.A.n, "nnz": p.A.nnz, "tol": p.tol, "map": "fp64",
            "iters": res.iters, "iters_oracle": g["iters"] if g else None,
            "us_per_solve": us, "us_per_iter": us / max(1, res.iters), "us_per_step_with_setup": us_step,
            "true_relres": float(np.linalg.norm(p.b - S @ res.x.cpu().numpy()) / np.linalg.norm(p.b)),
            "x_rel_err_vs_oracle": x_err_vs_oracle(g, res.x.cpu().numpy())}


def bench_config2_keys(args):
    """The 128^3 log-uniform workload (blocks of 32) as extra keys of the
    default line: FP16 and FP64 maps in symmetric storage, a few steps each,
    iterations against the oracle's."""
    import numpy as np
    import torch

    from paper_2407_15973_amd import binding as mb
    from paper_2407_15973_amd import gen

    dev = "cuda:0"
    log("128^3 log-uniform workload (extra keys)")
    p = gen.config2(seed=0, N=128, b=32)
    A = mb.DeviceCSR(p.A, dev)
    b = torch.as_tensor(p.b, device=dev)
    solver = mb.Solver(p.A.n, dev)
    out = {"workload": p.name, "n": p.A.n, "nnz": p.A.nnz, "blocks": len(p.block_ptr) - 1}
    S = p.A.to_scipy()
    for name, pol in (("fp16", mb.Policy(mode=mb.FIXED, low=mb.FP16, storage=mb.STORE_SYM)),
                      ("fp64", mb.Policy(mode=mb.UNIFORM, storage=mb.STORE_SYM))):
        def one():
            M = mb.BlockJacobi(A, p.block_ptr, pol)
            return solver.solve(A, M, b, tol=p.tol, maxit=p.maxit, verify=VERIFY)
        one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            res = one()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / 5
        x = res.x.cpu().numpy()
        g = oracle_golden("diff3d_128", name)
        out[name] = {"ms_per_step": ms, "steps": 5, "iters": res.iters,
                     "true_relres": float(np.linalg.norm(p.b - S @ x) / np.linalg.norm(p.b)),
                     "iters_oracle_same_map": g["iters"] if g else None,
                     "x_rel_err_vs_oracle_same_map": x_err_vs_oracle(g, x)}
        log(f"128^3 {name}: {ms:.1f} ms/step, {res.iters} iterations")
    out["speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / out["fp16"]["ms_per_step"]
    return out


# ------------------------------------------------ band-truncated storage
def bench_band(args):
    import numpy as np
    import torch

    from paper_2407_15973_amd import binding as mb
    from paper_2407_15973_amd import gen

    dev = "cuda:0"
    N = args.N or 128
    log("building the workload")
    p = gen.config2(seed=0, N=N, b=32)
    n, nnz, nb = p.A.n, p.A.nnz, len(p.block_ptr) - 1
    A = mb.DeviceCSR(p.A, dev)
    b = torch.as_tensor(p.b, device=dev)
    solver = mb.Solver(n, dev)
    band = dict(storage=mb.STORE_BAND)
    pols = {"fp64_full": mb.Policy(mode=mb.UNIFORM), "fp16_full": mb.Policy(mode=mb.FIXED, low=mb.FP16),
            "fp64_band": mb.Policy(mode=mb.UNIFORM, **band), "fp32_band": mb.Policy(mode=mb.FIXED, low=mb.FP32, **band),
            "fp16_band": mb.Policy(mode=mb.FIXED, low=mb.FP16, **band),
            "fp64_sym": mb.Policy(mode=mb.UNIFORM, storage=mb.STORE_SYM),
            "fp16_sym": mb.Policy(mode=mb.FIXED, low=mb.FP16, storage=mb.STORE_SYM)}
    head = "fp16_band"

    def step(policy, profile=False):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        M = mb.BlockJacobi(A, p.block_ptr, policy)
        e1.record()
        res = solver.solve(A, M, b, tol=p.tol, maxit=p.maxit, profile=profile, verify=0 if profile else VERIFY)
        e2.record()
        return M, res, (e0, e1, e2)

    S = p.A.to_scipy()
    bn = float(np.linalg.norm(p.b))
    ib = index_bytes(p.A)
    vb = value_bytes(p.A, ib)
    rows, kern_all = {}, {}
    for name, pol in pols.items():
        for _ in range(args.warmup):
            step(pol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        runs = [step(pol) for _ in range(args.steps)]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        M, res, ev = runs[-1]
        info = M.info()
        is_band = pol.storage == mb.STORE_BAND
        w = M.band_widths() if is_band else None
        rows[name] = {"ms_per_step": ms, "iters": res.iters, "status": res.status, "restarts": res.restarts,
                      "true_relres": float(np.linalg.norm(p.b - S @ res.x.cpu().numpy()) / bn),
                      "setup_ms": float(np.median([r[2][0].elapsed_time(r[2][1]) for r in runs])),
                      "solve_ms": float(np.median([r[2][1].elapsed_time(r[2][2]) for r in runs])),
                      "stored_bytes": info["low_bytes"],
                      "mean_width": float(w.mean()) if is_band else None,
                      "max_width": int(w.max()) if is_band else None}
        # per-kernel event timing of the same solve
        _, rp, _ = step(pol, profile=True)
        kb = {"spmv": spmv_bytes(n, nnz, ib, vb),
              "apply": apply_bytes(n, nb, info["ntiles"], info["low_bytes"], band=is_band)}
        kern = {}
        for kname in ("spmv", "apply"):
            tot, cnt = rp.kernel_ms[kname]
            avg_ms = tot / max(1, cnt)
            kern[kname] = {"launches": cnt, "avg_us": avg_ms * 1e3, "bytes": kb[kname],
                           "gbs": kb[kname] / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None}
        kern_all[name] = kern
        rows[name]["apply_us"] = kern["apply"]["avg_us"]
        rows[name]["apply_gbs"] = kern["apply"]["gbs"]
        log(f"{name}: {ms:.1f} ms/step, {res.iters} iterations, stored {info['low_bytes'] / 1e6:.1f} MB, "
            f"apply {kern['apply']['avg_us']:.1f} us ({kern['apply']['gbs']:.0f} GB/s)")
        del M, runs
    kern = kern_all[head]
    dom = max(kern, key=lambda k: kern[k]["avg_us"] * kern[k]["launches"])
    dk = kern[dom]
    # the SpMV is the same kernel as in the default workload: its measured traffic applies
    traffic = measured_traffic("diff3d_128:spmv") if (N == 128 and dom == "spmv") else None
    roofline = {"bound": "hbm", "achieved": dk["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dk["gbs"] / HBM_PEAK_GBS, "traffic": traffic, "kernel": f"{dom}_kernel",
                "bytes_per_launch": dk["bytes"], "avg_launch_us": dk["avg_us"]}
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")
        cpu = cpu_baseline_full(p, rows[head]["iters"])
    hv = rows[head]
    return {
        "metric": METRIC, "value": hv["ms_per_step"], "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": hv["ms_per_step"], "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "apply_arith": "band-truncated fp16-stored block inverses, f32 accumulation",
        "config": {"workload": f"diff3d_loguniform_{N}^3_b32_band", "n": n, "nnz": nnz, "blocks": nb,
                   "block_rows": 32, "precision_map": "fp16 fixed, band storage", "tol": p.tol, "seed": 0},
        "policies": rows, "speedup_vs_fp64_full": rows["fp64_full"]["ms_per_step"] / hv["ms_per_step"],
        "speedup_vs_fp16_full": rows["fp16_full"]["ms_per_step"] / hv["ms_per_step"],
        "delay_iters": hv["iters"] - rows["fp64_full"]["iters"],
        "kernels": kern_all, "roofline": roofline, "cpu_baseline": cpu,
    }


# ------------------------------------------------- the paper's own setting
# Iteration counts printed by the paper (Table 4.2; Sec. 4.5.1 for Ani(s)),
# BJAC k = t = 2 on 32 blocks, tol 1e-10, fp32 low precision, Diff3D 128^3.
PAPER_TABLE_4_2 = {
    "Const": {"uniform": 148, "fMP": 165, "hl@10": 165, "hl@5": 148, "hl@1": 148, "hl@0.1": 148,
              "lh@1e-05": 165, "lh@10": 165},
    "Dis(1000)": {"uniform": 185, "fMP": 211, "hl@10": 205, "hl@5": 201, "hl@1": 185, "hl@0.1": 185,
                  "lh@1e-05": 211, "lh@10": 201},
}
PAPER_ANI = {1000: (327, 327), 100: (321, 321), 10: (205, 205), 4: (179, 179), 2: (159, 177), 1: (148, 165)}


def poly_apply_bytes(n, nnz, k, t, tb):
    """Algorithmic bytes of one paper-mode application BJAC(k, t) with values
    of tb bytes: the first sweep from y = 0 (r, 1/a_ii read; v, y written),
    t - 1 block sweeps per outer step (row pointers, block ranges, the CSR
    entries, v, y, 1/a_ii read and y written; the last sweep of a later step
    also reads the step's start), k - 1 residuals A z (CSR, v, z, 1/a_ii read;
    w, y written), and the widening of z with (r, z)."""
    csr = 4 * (n + 1) + (4 + tb) * nnz
    first = (8 + 3 * tb) * n
    sweep = csr + 8 * n + 4 * tb * n
    resid = csr + 5 * tb * n + (tb * n if t == 1 else 0)
    finish = (16 + tb) * n
    sweeps = (t - 1) * k
    adds = (k - 1) if t > 1 else 0
    return first + sweeps * sweep + adds * tb * n + (k - 1) * resid + finish


def bench_paper(args):
    import numpy as np
    import torch

    from paper_2407_15973_amd import binding as mb
    from paper_2407_15973_amd import gen

    dev = "cuda:0"
    N = args.N or 128
    runs = {}

    def solve(A, Ad, bp, b, S, low, temporal=mb.TEMPORAL_NONE, adp=math.inf):
        M = mb.PaperBJAC(Ad, bp, k=2, t=2, low=low, temporal=temporal, adp_tol=adp)
        for _ in range(args.warmup):
            S.solve(Ad, M, b, tol=1e-10, maxit=2000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res = S.solve(Ad, M, b, tol=1e-10, maxit=2000)
        torch.cuda.synchronize()
        return res, (time.perf_counter() - t0) * 1e3 / args.steps

    problems = [("Const", gen.kappa_const(N), (1.0, 1.0, 1.0)), ("Dis(1000)", gen.kappa_dis(N, 1000.0), (1.0, 1.0, 1.0))]
    for s_ in PAPER_ANI:
        problems.append((f"Ani({s_})", gen.kappa_const(N), (1.0, float(s_), float(s_))))
    head_ms = None
    for name, kap, an in problems:
        log(f"paper mode {name}")
        A = gen.diffusion3d(kap, aniso=an)
        Ad = mb.DeviceCSR(A, dev)
        bp = gen.uniform_blocks(A.n, A.n // 32)
        b = torch.ones(A.n, dtype=torch.float64, device=dev)
        S = mb.Solver(A.n, dev)
        pols = [("uniform", False, mb.TEMPORAL_NONE, math.inf), ("fMP", True, mb.TEMPORAL_NONE, math.inf)]
        if not name.startswith("Ani"):
            pols += [(f"hl@{a:g}", True, mb.TEMPORAL_HL, a) for a in (10.0, 5.0, 1.0, 0.1)]
            pols += [(f"lh@{a:g}", True, mb.TEMPORAL_LH, a) for a in (1e-5, 10.0)]
        row = {}
        for pname, low, temporal, adp in pols:
            res, ms = solve(A, Ad, bp, b, S, low, temporal, adp)
            if name.startswith("Ani"):
                paper = PAPER_ANI[int(name[4:-1])][0 if pname == "uniform" else 1]
            else:
                paper = PAPER_TABLE_4_2[name][pname]
            row[pname] = {"iters": res.iters, "paper_iters": paper, "ms": ms, "status": res.status,
                          "high_applications": res.high_applications}
            log(f"  {pname}: {res.iters} iterations (paper {paper}), {ms:.1f} ms")
        runs[name] = row
        if name == "Const":
            head_ms = row["fMP"]["ms"]
            speed = row["uniform"]["ms"] / row["fMP"]["ms"]
            # per-kernel event timing of the same solves
            kern = {}
            for pname, low in (("fMP", True), ("uniform", False)):
                M = mb.PaperBJAC(Ad, bp, k=2, t=2, low=low)
                rp = S.solve(Ad, M, b, tol=1e-10, maxit=2000, profile=True)
                kb = {"spmv": spmv_bytes(A.n, A.nnz, index_bytes(A), value_bytes(A, index_bytes(A))), "apply": poly_apply_bytes(A.n, A.nnz, 2, 2, 4 if low else 8),
                      "update": 48 * A.n}
                for kname in ("spmv", "apply", "update"):
                    tot, cnt = rp.kernel_ms[kname]
                    avg_ms = tot / max(1, cnt)
                    kern[f"{pname}_{kname}"] = {"launches": cnt, "avg_us": avg_ms * 1e3, "bytes": kb[kname],
                                                "gbs": kb[kname] / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None}
                log(f"  profile {pname}: " + ", ".join(f"{kn} {kern[pname + '_' + kn]['avg_us']:.1f} us"
                                                       for kn in ("spmv", "apply", "update")))
        del Ad, S
        torch.cuda.empty_cache()
    # the application (five kernels: first sweep, block sweep, residual, block
    # sweep, widening) dominates; its bytes over its event-timed duration
    dk = kern["fMP_apply"]
    roofline = {"bound": "hbm", "achieved": dk["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dk["gbs"] / HBM_PEAK_GBS, "traffic": None, "kernel": "paper-mode application (FP32)",
                "bytes_per_launch": dk["bytes"], "avg_launch_us": dk["avg_us"]}
    return {
        "metric": METRIC, "value": head_ms, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head_ms, "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "apply_arith": "paper-mode BJAC(2, 2): FP32 (fMP) or FP64 application", "data": "synthetic",
        "config": {"workload": f"paper_mode_diff3d_{N}^3_32slabs_k2t2_f1", "tol": 1e-10},
        "speedup_vs_fp64": speed, "runs": runs, "kernels": kern, "roofline": roofline, "cpu_baseline": None,
    }


# ----------------------------------------- radiation-diffusion-like systems
# Sec. 4.5.2 (RHD3D-1T): ratio of fp32-fMP to uniform iterations at P_diag
# 1, 2, 8 as the paper states them.
PAPER_PDIAG_ITER_O = {1.0: 1.36, 2.0: 1.24, 8.0: 1.20}


def bench_rhd(args):
    import numpy as np
    import torch

    from paper_2407_15973_amd import binding as mb
    from paper_2407_15973_amd import gen

    dev = "cuda:0"
    N = args.N or 128
    out = {}

    def timed(Ad, M, b, S, tol):
        for _ in range(args.warmup):
            S.solve(Ad, M, b, tol=tol, maxit=5000, raise_on_error=False, verify=VERIFY)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r = S.solve(Ad, M, b, tol=tol, maxit=5000, raise_on_error=False, verify=VERIFY)
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t0) * 1e3 / args.steps

    for kind, tol in (("3T", 1e-10), ("1T", 1e-12)):
        log(f"rhd {kind} {N}^3")
        A = gen.rhd3t_like(N) if kind == "3T" else gen.rhd1t_like(N)
        Ad = mb.DeviceCSR(A, dev)
        b = torch.ones(A.n, dtype=torch.float64, device=dev)
        S = mb.Solver(A.n, dev)
        bp48 = gen.uniform_blocks(A.n, 48)
        slabs = gen.uniform_blocks(A.n, A.n // 32)
        row = {}
        for name, mk in (("fp64", lambda: mb.BlockJacobi(Ad, bp48, mb.Policy())),
                         ("fp32", lambda: mb.BlockJacobi(Ad, bp48, mb.Policy(mode=mb.FIXED, low=mb.FP32))),
                         ("fp16", lambda: mb.BlockJacobi(Ad, bp48, mb.Policy(mode=mb.FIXED, low=mb.FP16))),
                         ("rule", lambda: mb.BlockJacobi(Ad, bp48, mb.Policy(mode=mb.RULE))),
                         ("paper_fp64", lambda: mb.PaperBJAC(Ad, slabs, 2, 2, low=False)),
                         ("paper_fp32", lambda: mb.PaperBJAC(Ad, slabs, 2, 2, low=True))):
            M = mk()
            r, ms = timed(Ad, M, b, S, tol)
            row[name] = {"iters": r.iters, "status": r.status, "true_relres_device": r.true_relres,
                         "restarts": r.restarts, "ms": ms, "blocks_per_prec": M.info()["blocks_per_prec"]}
            log(f"  {name}: {r.iters} iterations, status {r.status}, true relres {r.true_relres:.2e}, {ms:.1f} ms")
            del M
        out[kind] = {"n": A.n, "nnz": A.nnz, "tol": tol, "runs": row}
        del Ad, S
        torch.cuda.empty_cache()
    log("P_diag sweep (1T, paper mode)")
    sweep = {}
    A0 = gen.rhd1t_like(N)
    for p in (0.0, 1.0, 2.0, 4.0, 8.0):
        A = gen.with_pdiag(A0, p)
        Ad = mb.DeviceCSR(A, dev)
        b = torch.ones(A.n, dtype=torch.float64, device=dev)
        S = mb.Solver(A.n, dev)
        slabs = gen.uniform_blocks(A.n, A.n // 32)
        it = {}
        for low in (False, True):
            r = S.solve(Ad, mb.PaperBJAC(Ad, slabs, 2, 2, low=low), b, tol=1e-12, maxit=5000, raise_on_error=False)
            it[low] = r.iters
        sweep[p] = {"uniform": it[False], "fMP": it[True], "iter_o": it[True] / max(1, it[False]),
                    "paper_iter_o": PAPER_PDIAG_ITER_O.get(p)}
        log(f"  P_diag {p:g}: uniform {it[False]}, fMP {it[True]}")
        del Ad, S
    head = out["3T"]["runs"]["rule"]
    return {
        "metric": METRIC, "value": head["ms"], "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "apply_arith": "stored inverses (rule map) / paper-mode BJAC(2, 2)", "data": "synthetic",
        "config": {"workload": f"rhd3t_like_{N}^3_interlaced_b48", "tol": out["3T"]["tol"]},
        "speedup_vs_fp64": out["3T"]["runs"]["fp64"]["ms"] / head["ms"], "rhd": out, "pdiag_sweep": sweep,
    }

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=None, help="grid edge (diff3d 128, aniso 160, selector 192)")
    ap.add_argument("--workload", default="selector",
                    choices=("diff3d", "batched", "aniso", "selector", "paper", "rhd", "band"))
    ap.add_argument("--axis", default="x", choices=("x", "yz"),
                    help="aniso: strong axis along x (inside the row blocks) or y and z (the paper's Ani(s))")
    ap.add_argument("--cmp-steps", type=int, default=3,
                    help="selector / aniso: timed steps of each comparison map (the headline map takes --steps)")
    ap.add_argument("--no-config2", action="store_true", help="selector: skip the 128^3 extra keys")
    ap.add_argument("--nsys", type=int, default=256, help="batched: number of systems")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run one 1 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path, so --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)
    if args.calibrate:
        calibration_copy()
    if args.workload == "diff3d":
        args.N = args.N or 128
        line = bench_diff3d(args)
    elif args.workload == "batched":
        line = bench_batched(args)
    elif args.workload == "paper":
        line = bench_paper(args)
    elif args.workload == "rhd":
        line = bench_rhd(args)
    elif args.workload == "band":
        line = bench_band(args)
    else:
        args.N = args.N or (160 if args.workload == "aniso" else 192)
        line = bench_policies(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
