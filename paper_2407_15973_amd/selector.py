"""Learned per-block precision selector: labels from the solver's own runs,
training with the library's MLP kernels, evaluation against the per-block rule
and FP64.

Labels (for one training matrix): solve with the all-FP64 map to get the
reference iteration count it64; then, for a descending grid of tolerances eta,
give each block the lowest precision p in {FP16, FP32} with
kappa_1(A_ii) * u_p <= eta (FP64 otherwise), solve with that explicit map, and
keep the first map (the largest eta) whose iteration count stays within
(1 + delay) * it64. The block's label is its precision in that map. The paper
relates the convergence delay of low-precision block-Jacobi to block features
(Sec. 4.5: multiscale strength, eq. 4-5, and diagonal dominance); the network
learns that relation from the 16 block features the setup computes.

Every solve runs on the GPU through the C ABI; training calls the library's
forward / backward / Adam kernels.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import binding as mb

U = {mb.FP16: 2.0 ** -11, mb.FP32: 2.0 ** -24}
CLASS_OF_TAG = {mb.FP64: 0, mb.FP32: 1, mb.FP16: 2}
TAG_OF_CLASS = np.array([mb.FP64, mb.FP32, mb.FP16], dtype=np.uint8)
ETAS = (math.inf, 1e3, 1e2, 1e1, 1e0, 1e-1, 1e-2, 1e-3, 0.0)


def tags_for_eta(kappa1: np.ndarray, eta: float) -> np.ndarray:
    tags = np.full(kappa1.shape, mb.FP64, dtype=np.uint8)
    tags[kappa1 * U[mb.FP32] <= eta] = mb.FP32
    tags[kappa1 * U[mb.FP16] <= eta] = mb.FP16
    return tags


@dataclass
class LabelSet:
    features: np.ndarray          # (nb, 16) float32
    labels: np.ndarray            # (nb,) int32 classes 0 FP64, 1 FP32, 2 FP16
    eta: float
    it64: int
    iters: int
    runs: list = field(default_factory=list)


TRAIN_CONTRASTS = (0.0, 2.0, 3.0, 4.0, 5.0)


def training_problems(seeds=(0, 1), N=32):
    """The training family: config 1 (2D Poisson) and config 2's 3D
    diffusion generator at point-coefficient contrasts 10^+-c. Up to c = 3
    every block tolerates FP16; at c = 4, 5 the all-FP16 map breaks down and
    the labels become mostly FP32 with FP16 for the best-conditioned blocks."""
    from . import gen
    probs = [gen.config1(s) for s in seeds]
    probs += [gen.config2(seed=s, N=N, contrast=c) for c in TRAIN_CONTRASTS for s in seeds]
    return probs


def make_labels(A: mb.DeviceCSR, block_ptr, b, tol=1e-10, maxit=5000, delay=0.05, solver=None,
                etas=ETAS) -> LabelSet:
    import torch
    solver = solver or mb.Solver(A.n, A.val.device)
    bt = torch.as_tensor(np.ascontiguousarray(b), device=A.val.device)
    M64 = mb.BlockJacobi(A, block_ptr, mb.Policy(mode=mb.UNIFORM))
    feat = M64.features()
    r64 = solver.solve(A, M64, bt, tol=tol, maxit=maxit, raise_on_error=False)
    if r64.status != mb.OK:
        raise ValueError("the FP64 reference solve did not converge: no delay to measure against")
    it64 = r64.iters
    kappa1 = 10.0 ** feat[:, 13].astype(np.float64)
    runs, seen = [], {}
    chosen = None
    for eta in etas:
        tags = tags_for_eta(kappa1, eta)
        key = tags.tobytes()
        if key in seen:
            it = seen[key]
        else:
            M = mb.BlockJacobi(A, block_ptr, mb.Policy(mode=mb.EXPLICIT, explicit_tags=tags))
            r = solver.solve(A, M, bt, tol=tol, maxit=maxit, raise_on_error=False)
            it = r.iters if r.status == mb.OK else maxit + 1
            seen[key] = it
        runs.append((eta, it, np.bincount(tags, minlength=4).tolist()))
        if it <= (1.0 + delay) * it64:
            chosen = (eta, tags, it)
            break
    if chosen is None:
        chosen = (0.0, np.full(len(kappa1), mb.FP64, np.uint8), it64)
    eta, tags, it = chosen
    labels = np.array([CLASS_OF_TAG[int(t)] for t in tags], dtype=np.int32)
    return LabelSet(feat, labels, eta, it64, it, runs)


@dataclass
class Selector:
    blob: object                  # device float32 [MLP_NBLOB]
    mu: np.ndarray
    sigma: np.ndarray
    history: list


def init_blob(rng, mu, sigma):
    """He-uniform weights, zero biases, then the feature mean and std."""
    shapes = ((64, 16), (64,), (64, 64), (64,), (3, 64), (3,))
    parts = []
    for shp in shapes:
        if len(shp) == 2:
            lim = math.sqrt(6.0 / shp[1])
            parts.append(rng.uniform(-lim, lim, size=shp).ravel())
        else:
            parts.append(np.zeros(shp))
    parts += [mu, sigma]
    return np.concatenate(parts).astype(np.float32)


def train(feats: np.ndarray, labels: np.ndarray, steps=400, lr=3e-3, seed=0, device="cuda") -> Selector:
    """Full-batch Adam on the mean softmax cross-entropy, every step on the
    GPU (library backward + Adam kernels)."""
    import torch
    feats = np.ascontiguousarray(feats, dtype=np.float32)
    mu = feats.mean(axis=0).astype(np.float64)
    sigma = feats.std(axis=0).astype(np.float64)
    sigma = np.where(sigma > 1e-6, sigma, 1.0)
    rng = np.random.default_rng(seed)
    blob = torch.as_tensor(init_blob(rng, mu, sigma), device=device)
    X = torch.as_tensor(feats, device=device)
    y = torch.as_tensor(np.ascontiguousarray(labels, dtype=np.int32), device=device)
    tr = mb.MlpTrainer(len(labels), device)
    hist = []
    for step in range(steps):
        _, loss = tr.backward(blob, X, y)
        tr.adam(blob, lr=lr)
        if step % 50 == 0 or step == steps - 1:
            hist.append((step, float(loss.cpu())))
    return Selector(blob, mu, sigma, hist)


def predict_tags(sel: Selector, feats: np.ndarray):
    import torch
    X = torch.as_tensor(np.ascontiguousarray(feats, dtype=np.float32), device=sel.blob.device)
    _, tags = mb.mlp_forward(sel.blob, X, want_logits=False, want_tags=True)
    return tags.cpu().numpy()


@dataclass
class EvalRow:
    policy: str
    iters: int
    status: int
    setup_ms: float
    solve_ms: float
    hist: list
    low_bytes: int


def evaluate(A: mb.DeviceCSR, block_ptr, b, policies: dict, tol=1e-10, maxit=5000, solver=None, reps=2):
    """Time setup + solve for each named policy (best of reps)."""
    import torch
    solver = solver or mb.Solver(A.n, A.val.device)
    bt = torch.as_tensor(np.ascontiguousarray(b), device=A.val.device)
    rows = {}
    for name, pol in policies.items():
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            M = mb.BlockJacobi(A, block_ptr, pol)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = solver.solve(A, M, bt, tol=tol, maxit=maxit, raise_on_error=False)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            row = EvalRow(name, r.iters, r.status, 1e3 * (t1 - t0), 1e3 * (t2 - t1),
                          M.info()["blocks_per_prec"], M.info()["low_bytes"])
            if best is None or row.setup_ms + row.solve_ms < best.setup_ms + best.solve_ms:
                best = row
        rows[name] = best
    return rows


def solve_with_fallback(A: mb.DeviceCSR, block_ptr, b, sel: Selector, tol=1e-10, maxit=5000, solver=None):
    """Solve with the learned map; if it breaks down or misses the tolerance,
    solve again with the per-block rule, then with FP64. Returns (result,
    policy name used)."""
    import torch
    solver = solver or mb.Solver(A.n, A.val.device)
    bt = torch.as_tensor(np.ascontiguousarray(b), device=A.val.device)
    chain = (("learned", mb.Policy(mode=mb.LEARNED, mlp_blob=sel.blob)), ("rule", mb.Policy(mode=mb.RULE)),
             ("fp64", mb.Policy(mode=mb.UNIFORM)))
    res = None
    for name, pol in chain:
        M = mb.BlockJacobi(A, block_ptr, pol)
        res = solver.solve(A, M, bt, tol=tol, maxit=maxit, raise_on_error=False)
        if res.status == mb.OK:
            return res, name
    return res, "fp64"
