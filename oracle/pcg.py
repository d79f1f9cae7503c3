"""Preconditioned conjugate gradient with fixed and adaptive mixed-precision
block-Jacobi, plain FP64.

Test infrastructure only (see the package docstring).

The paper takes PCG (Hestenes-Stiefel, cited in Sec. 3.2) without printing it;
this is the textbook recurrence, x0 = 0 (Sec. 4.2). Readings:
  * stopping test ||r_j||_2 / ||r_0||_2 <= tol on the recursive residual,
    checked right after the r update; the iteration count is the number of x
    updates (Sec. 4.2: the relative residual 2-norm stopping test);
  * the adaptive switch of Algorithms 3.2 / 3.3 is evaluated every time the
    preconditioner is applied, with the current recursive relres; the first
    application (to r_0) sees relres = +inf (so hl starts high and lh starts
    low, consistent with Sec. 4.4.2's statement that lh at adp_tol = 10 runs
    its first iteration in low precision); the switch does not latch.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import blocks as B
from . import precision as P

TEMPORAL_NONE, TEMPORAL_HL, TEMPORAL_LH = 0, 1, 2

CONVERGED, MAXIT, BREAKDOWN = 0, 1, -3


@dataclass
class Result:
    x: np.ndarray
    iters: int
    status: int
    relres: float
    history: list = field(default_factory=list)   # recursive relres after each x update
    used_high: list = field(default_factory=list)  # per preconditioner application


def use_high(temporal: int, relres: float, adp_tol: float) -> bool:
    """Algorithm 3.2 (hl): high precision while relres >= adp_tol.
    Algorithm 3.3 (lh): low precision while relres >= adp_tol."""
    if temporal == TEMPORAL_HL:
        return relres >= adp_tol
    if temporal == TEMPORAL_LH:
        return not (relres >= adp_tol)
    return False


def pcg(matvec, b, precond, tol, maxit, temporal=TEMPORAL_NONE, adp_tol=math.inf,
        precond_high=None) -> Result:
    """Textbook PCG. ``precond(r)`` is the (possibly low-precision) map;
    ``precond_high(r)`` the working-precision one used when the adaptive
    switch asks for high precision."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    r0 = float(np.sqrt(r @ r))
    res = Result(x, 0, CONVERGED, 0.0)
    if r0 == 0.0:
        return res

    def P_(rv, relres):
        hi = temporal != TEMPORAL_NONE and use_high(temporal, relres, adp_tol)
        res.used_high.append(bool(hi))
        return (precond_high if hi else precond)(rv)

    z = P_(r, math.inf)
    p = z.copy()
    rho = float(r @ z)
    if not (rho > 0):
        res.status = BREAKDOWN
        return res
    for j in range(1, maxit + 1):
        q = matvec(p)
        pq = float(p @ q)
        if not (pq > 0):
            res.status, res.iters = BREAKDOWN, j - 1
            return res
        alpha = rho / pq
        x += alpha * p
        r -= alpha * q
        relres = float(np.sqrt(r @ r)) / r0
        res.history.append(relres)
        res.iters, res.relres = j, relres
        if relres <= tol:
            res.status = CONVERGED
            return res
        z = P_(r, relres)
        rho_new = float(r @ z)
        if not (rho_new > 0):
            res.status = BREAKDOWN
            return res
        p = z + (rho_new / rho) * p
        rho = rho_new
    res.status = MAXIT
    return res


def pcg_single_reduction(matvec, b, precond, tol, maxit) -> Result:
    """PCG with one reduction phase per iteration: the Chronopoulos-Gear
    recurrence (Chronopoulos and Gear, J. Comput. Appl. Math. 25, 1989), which
    in exact arithmetic produces the iterates of the textbook PCG above. Each
    iteration forms u = M^-1 r and w = A u first, then takes the three inner
    products (r, r), (r, u) and (w, u) together; the direction p and its image
    s = A p are updated by the same recurrence, so A p is never formed:
        gamma = (r, u), delta = (w, u), beta = gamma / gamma_old,
        alpha = gamma / (delta - beta * gamma / alpha_old),
        p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s
    (beta = 0 and alpha = gamma / delta in the first iteration). The stopping
    test and the iteration count are those of ``pcg`` (Sec. 4.2, x0 = 0)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    r0 = float(np.sqrt(r @ r))
    res = Result(x, 0, CONVERGED, 0.0)
    if r0 == 0.0:
        return res
    p = np.zeros_like(b)
    s = np.zeros_like(b)
    gamma_old = alpha_old = 0.0
    for j in range(0, maxit + 1):
        if j > 0:
            relres = float(np.sqrt(r @ r)) / r0
            res.history.append(relres)
            res.iters, res.relres = j, relres
            if relres <= tol:
                res.status = CONVERGED
                return res
            if j == maxit:
                break
        u = precond(r)
        w = matvec(u)
        gamma = float(r @ u)
        delta = float(w @ u)
        if not (gamma > 0):
            res.status = BREAKDOWN
            return res
        if j == 0:
            beta, denom = 0.0, delta
        else:
            beta = gamma / gamma_old
            denom = delta - beta * gamma / alpha_old
        if not (denom > 0):
            res.status = BREAKDOWN
            return res
        alpha = gamma / denom
        p = u + beta * p
        s = w + beta * s
        x += alpha * p
        r -= alpha * s
        gamma_old, alpha_old = gamma, alpha
    res.status = MAXIT
    return res


def solve_bjac_single_reduction(A, block_ptr, b, tags=None, tol=1e-10, maxit=5000, M=None) -> Result:
    """Block-Jacobi PCG in the single-reduction (Chronopoulos-Gear) form."""
    M = BJAC(A, block_ptr, tags) if M is None else M
    S = A.to_scipy()
    return pcg_single_reduction(lambda v: S @ v, b, M.low, tol, maxit)


def true_relres(A, x, b) -> float:
    """||b - A x||_2 / ||b||_2 recomputed in FP64 (Sec. 4.5.1, true RelResNorm)."""
    S = A.to_scipy()
    r = b - S @ x
    return float(np.linalg.norm(r) / np.linalg.norm(b))


class BJAC:
    """Block-Jacobi with one outer step and exact block inverses stored per the
    precision map ``tags`` (eq. 3-1 with k = 1, Algorithm 3.1 for reduced
    blocks). ``high`` is the all-FP64 map used by the adaptive switch."""

    def __init__(self, A, block_ptr, tags=None, H=None, band=False, band_rtol=None):
        self.A = A
        self.block_ptr = np.asarray(block_ptr, dtype=np.int64)
        self.H = B.invert_blocks(A, block_ptr) if H is None else H
        nb = len(self.block_ptr) - 1
        self.tags = np.zeros(nb, dtype=np.uint8) if tags is None else np.asarray(tags, dtype=np.uint8)
        if band:
            # band-truncated storage of both maps (see blocks.band_width)
            self.store = B.store_blocks_band(self.H, self.tags, band_rtol)
            self.store_high = B.store_blocks_band(self.H, np.zeros(nb, dtype=np.uint8), band_rtol)
        else:
            self.store = B.store_blocks(self.H, self.tags)
            self.store_high = B.store_blocks(self.H, np.zeros(nb, dtype=np.uint8))

    def low(self, r):
        return B.apply(self.store, self.block_ptr, r)

    def high(self, r):
        return B.apply(self.store_high, self.block_ptr, r)


def solve_bjac(A, block_ptr, b, tags=None, tol=1e-10, maxit=5000, temporal=TEMPORAL_NONE,
               adp_tol=math.inf, M=None) -> Result:
    """PCG preconditioned by block-Jacobi with the given precision map."""
    M = BJAC(A, block_ptr, tags) if M is None else M
    S = A.to_scipy()
    return pcg(lambda v: S @ v, b, M.low, tol, maxit, temporal, adp_tol, M.high)


# -------------------------------------------------- paper-mode BJAC(k, t)
class PolyBJAC:
    """The paper's BJAC with k outer steps (eq. 3-1 / 3-2) and, for the block
    solve, either the exact FP64 inverse or t point-Jacobi sweeps inside each
    block (eq. 3-3). ``low=True`` evaluates the whole preconditioner in fp32
    (Sec. 3.2: all floating-point computations of M^-1(p_l) in p_l, with r
    converted on entry and z widened on exit, Algorithm 3.1)."""

    def __init__(self, A, block_ptr, k=2, t=2, exact=False, low=False):
        self.k, self.t, self.exact, self.low = k, t, exact, low
        self.bp = np.asarray(block_ptr, dtype=np.int64)
        dt = np.float32 if low else np.float64
        self.dt = dt
        S = A.to_scipy()
        self.S = S.astype(dt)
        # block-diagonal part D_b and its diagonal D
        rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr.astype(np.int64)))
        cols = A.col_idx.astype(np.int64)
        inb = B.block_of_rows(self.bp, rows) == B.block_of_rows(self.bp, cols)
        import scipy.sparse as sp
        self.Db = sp.csr_matrix((A.val[inb], (rows[inb], cols[inb])), shape=(A.n, A.n)).astype(dt)
        self.dinv = (1.0 / S.diagonal()).astype(dt)
        if exact:
            H = B.invert_blocks(A, block_ptr)
            self.H = [h.astype(dt) for h in H]

    def block_solve(self, v):
        """D_b-hat^-1 v: exact block inverses, or t sweeps of
        y <- y + D^-1 (v - A_ii y) from y = 0 inside every block (eq. 3-3)."""
        if self.exact:
            out = np.empty_like(v)
            for kk, h in enumerate(self.H):
                a, b = self.bp[kk], self.bp[kk + 1]
                out[a:b] = h @ v[a:b]
            return out
        y = self.dinv * v
        for _ in range(self.t - 1):
            y = y + self.dinv * (v - self.Db @ y)
        return y

    def __call__(self, r):
        v = np.asarray(r).astype(self.dt)
        z = self.block_solve(v)
        for _ in range(self.k - 1):
            z = z + self.block_solve(v - self.S @ z)
        return z.astype(np.float64)


def solve_poly(A, block_ptr, b, k=2, t=2, low=False, tol=1e-10, maxit=5000, temporal=TEMPORAL_NONE,
               adp_tol=math.inf, exact=False) -> Result:
    S = A.to_scipy()
    Mlow = PolyBJAC(A, block_ptr, k, t, exact, low=low)
    Mhigh = PolyBJAC(A, block_ptr, k, t, exact, low=False) if temporal != TEMPORAL_NONE else Mlow
    return pcg(lambda v: S @ v, b, Mlow, tol, maxit, temporal, adp_tol, Mhigh)
