#!/usr/bin/env python3
"""Writes the oracle's PCG iteration counts at the benchmark sizes.

Calls only the CPU oracle (``oracle/``) and the seeded input generator; no
value here comes from the GPU library. One invocation solves one (workload,
precision map) pair and writes ``oracle_iters_<workload>_<map>.json`` beside
this script:

  poisson_64   2D 5-point Poisson 64x64, blocks of 64 (grid lines), seed 0,
               relative residual 1e-8 (the latency-bound small workload)
  diff3d_128   3D 7-point diffusion 128^3, coefficients 10^U(-2,2), blocks
               of 32, seed 0 (the fixed-precision benchmark workload)
  aniso_160    anisotropic (1e3) diffusion with 1e4 jumps on 16 subcubes,
               160^3, blocks of 48, seed 0 (the per-block rule workload)
  heldout_192  the same generator at 192^3, held-out seed 100 (the learned
               selector's evaluation workload)

Maps: fp64 (uniform BJAC), fp32 / fp16 (fixed, Algorithm 3.1), rule (the
per-block condition / dominance rule on the oracle's own features). Each
file records the iteration count of textbook PCG from x0 = 0 to the recursive
relative residual 1e-10 (Sec. 4.2), the status, the final recursive and true
relative residuals, the map's histogram, the solution's 2-norm and its values
at 1024 seeded sample rows (for the ||x - x_oracle|| / ||x_oracle|| report).

Perturbations (a third argument; the file name gains _<perturbation>): the
same solve after a change of the inputs at the level of FP64 rounding, to
measure how far the iteration count of a long CG moves under rounding alone:
  b1ulp   every b_i times (1 + s_i 2^-52), s_i = +-1 from a fixed seed
  b1ulpK  the same with the signs from seed 4242 + K (K = 1, 2, ...): more
          samples of the spread
  upper   every block inverse replaced by its upper triangle mirrored (the
          symmetric storage of the GPU path keeps only that triangle)

Usage: python tests/golden/make_oracle_iters.py <workload> <map> [perturbation]
Runtime (one core): minutes at 128^3, about half an hour per map at 160^3 and
an hour at 192^3.
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import blocks as OB  # noqa: E402
from oracle import pcg as OP  # noqa: E402
from oracle import precision as OPr  # noqa: E402
from paper_2407_15973_amd import gen  # noqa: E402

WORKLOADS = {
    "poisson_64": lambda: gen.config1(seed=0),
    "diff3d_128": lambda: gen.config2(seed=0, N=128, b=32),
    "aniso_160": lambda: gen.config3(seed=0, N=160, b=48),
    "heldout_192": lambda: gen.config5_eval(seed=100, N=192, b=48),
}
MAPS = ("fp64", "fp32", "fp16", "rule")
NSAMPLE = 1024


def sample_rows(n: int) -> np.ndarray:
    """1024 distinct rows drawn with a fixed seed (independent of the workload's own)."""
    return np.sort(np.random.default_rng(12345).choice(n, size=min(n, NSAMPLE), replace=False))


def perturbation_seed(perturb: str | None):
    """Sign seed of a b1ulp[K] perturbation, None for any other."""
    if perturb == "b1ulp":
        return 4242
    if perturb and perturb.startswith("b1ulp") and perturb[5:].isdigit():
        return 4242 + int(perturb[5:])
    return None


def main(workload: str, pmap: str, perturb: str | None = None) -> None:
    t0 = time.perf_counter()
    p = WORKLOADS[workload]()
    if perturbation_seed(perturb) is not None:
        sgn = np.random.default_rng(perturbation_seed(perturb)).choice([-1.0, 1.0], size=p.b.size)
        p.b = p.b * (1.0 + sgn * 2.0 ** -52)
    nb = len(p.block_ptr) - 1
    print(f"[golden] {workload} {pmap}: n = {p.A.n}, nnz = {p.A.nnz}, blocks = {nb}", flush=True)
    H = OB.invert_blocks(p.A, p.block_ptr)
    if perturb == "upper":
        H = [np.triu(h) + np.triu(h, 1).T for h in H]
    if pmap == "fp64":
        tags = np.full(nb, OPr.FP64, np.uint8)
    elif pmap == "fp32":
        tags = np.full(nb, OPr.FP32, np.uint8)
    elif pmap == "fp16":
        tags = np.full(nb, OPr.FP16, np.uint8)
    else:
        _, raw = OB.block_features(p.A, p.block_ptr, H)
        tags = OB.select_rule(raw)
    store = OB.store_blocks(H, tags)
    del H
    S = p.A.to_scipy()
    t1 = time.perf_counter()
    print(f"[golden] setup {t1 - t0:.1f} s; solving", flush=True)
    count = [0]

    def precond(r):
        count[0] += 1
        if count[0] % 100 == 0:
            print(f"[golden] {workload} {pmap}: application {count[0]} "
                  f"({time.perf_counter() - t1:.0f} s)", flush=True)
        return OB.apply(store, p.block_ptr, r)

    res = OP.pcg(lambda v: S @ v, p.b, precond, p.tol, p.maxit)
    t2 = time.perf_counter()
    rows = sample_rows(p.A.n)
    out = {
        "source": "oracle/ (textbook PCG, x0 = 0, recursive relres stopping test of Sec. 4.2) "
                  "written by tests/golden/make_oracle_iters.py",
        "workload": p.name, "seed_workload": workload, "map": pmap, "perturbation": perturb,
        "n": int(p.A.n), "nnz": int(p.A.nnz), "blocks": nb, "tol": p.tol, "maxit": p.maxit,
        "iters": int(res.iters), "status": int(res.status), "relres": float(res.relres),
        "true_relres": OP.true_relres(p.A, res.x, p.b),
        "blocks_per_prec": [int(np.count_nonzero(tags == t)) for t in range(4)],
        "x_norm": float(np.linalg.norm(res.x)),
        "sample_rows": [int(v) for v in rows], "x_sample": [float(v) for v in res.x[rows]],
        "setup_s": t1 - t0, "solve_s": t2 - t1,
    }
    suffix = f"_{perturb}" if perturb else ""
    path = os.path.join(HERE, f"oracle_iters_{workload}_{pmap}{suffix}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"[golden] {workload} {pmap}: {res.iters} iterations, status {res.status}, "
          f"true relres {out['true_relres']:.3e}, {t2 - t1:.0f} s -> {path}", flush=True)


if __name__ == "__main__":
    if (len(sys.argv) not in (3, 4) or sys.argv[1] not in WORKLOADS or sys.argv[2] not in MAPS
            or (len(sys.argv) == 4 and sys.argv[3] != "upper" and perturbation_seed(sys.argv[3]) is None)):
        sys.exit(f"usage: {sys.argv[0]} {{{','.join(WORKLOADS)}}} {{{','.join(MAPS)}}} [upper|b1ulp|b1ulpK]")
    main(sys.argv[1], sys.argv[2], sys.argv[3] if len(sys.argv) == 4 else None)
