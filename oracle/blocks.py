"""Block-Jacobi setup and application, plain FP64.

Test infrastructure only (see the package docstring).

Paper Sec. 3.1: A is partitioned into blocks A_ij, D_b = diag{A_ii}, and the
block-Jacobi preconditioner with one outer step (k = 1 in eq. 3-1) applies
D_b^-1, i.e. z_blk = A_ii^-1 r_blk for every diagonal block. The paper assumes
equal blocks n/nb; here blocks are contiguous row ranges given by ``block_ptr``
(the last one holds the remainder).

The block inverse is formed in FP64 (a textbook Cholesky factorisation and
forward/backward substitution against the identity), then stored in the
block's precision (Sec. 3.2: the low-precision preconditioner M^-1(p_l)), and
applied to the FP32 copy of r (Algorithm 3.1). The oracle accumulates the
products of the stored values exactly enough (FP64) to be the reference the
GPU's FP32 accumulation is bounded against.
"""
from __future__ import annotations

import numpy as np

from . import precision as P

NFEAT = 16
FEATURE_NAMES = (
    "size_over_64", "log10_min_dom", "log10_mean_dom", "log10_min_dom_inblock",
    "offin_over_diag_fro", "offout_over_diag_fro", "max_log10_tau", "mean_log10_tau",
    "log10_coef_contrast", "gersh_lo_over_maxdiag", "gersh_hi_over_maxdiag",
    "log10_gersh_cond", "log10_diag_ratio", "log10_kappa1", "log10_inv_diag_ratio",
    "frac_inv_below_2m24",
)
DOM_CAP = 1e8          # dominance ratios are capped at 1e8 (no off-diagonals)
GERSH_FLOOR = 1e-16    # Gershgorin condition estimate capped at 1e16


class NotSPD(ValueError):
    def __init__(self, blocks):
        super().__init__(f"non-positive pivot in block(s) {list(blocks)[:8]}")
        self.blocks = list(blocks)


def block_sizes(block_ptr) -> np.ndarray:
    bp = np.asarray(block_ptr, dtype=np.int64)
    return bp[1:] - bp[:-1]


def block_of_rows(block_ptr, rows) -> np.ndarray:
    return np.searchsorted(np.asarray(block_ptr, dtype=np.int64), rows, side="right") - 1


def extract_blocks(A, block_ptr):
    """Dense diagonal blocks A_ii (Sec. 3.1, D_b = diag{A_ii}). Returns a dict
    size -> (block indices, array (count, size, size))."""
    bp = np.asarray(block_ptr, dtype=np.int64)
    sizes = block_sizes(bp)
    rows = np.repeat(np.arange(A.n, dtype=np.int64), np.diff(A.row_ptr.astype(np.int64)))
    cols = A.col_idx.astype(np.int64)
    brow = block_of_rows(bp, rows)
    bcol = block_of_rows(bp, cols)
    keep = brow == bcol
    rows, cols, brow, vals = rows[keep], cols[keep], brow[keep], A.val[keep]
    out = {}
    for b in np.unique(sizes):
        ids = np.nonzero(sizes == b)[0]
        slot = np.full(len(sizes), -1, dtype=np.int64)
        slot[ids] = np.arange(len(ids))
        sel = slot[brow] >= 0
        dense = np.zeros((len(ids), int(b), int(b)))
        k = slot[brow[sel]]
        dense[k, rows[sel] - bp[brow[sel]], cols[sel] - bp[brow[sel]]] = vals[sel]
        out[int(b)] = (ids, dense)
    return out


def cholesky(Ab: np.ndarray):
    """Textbook Cholesky A = L L^T of a stack of SPD matrices, column by column:
    L_kk = sqrt(a_kk - sum_j L_kj^2), L_ik = (a_ik - sum_j L_ij L_kj) / L_kk.
    Returns (L, ok) with ok[i] False where a pivot was not positive."""
    Ab = np.asarray(Ab, dtype=np.float64)
    cnt, b, _ = Ab.shape
    L = np.zeros_like(Ab)
    ok = np.ones(cnt, dtype=bool)
    for k in range(b):
        d = Ab[:, k, k] - np.einsum("ij,ij->i", L[:, k, :k], L[:, k, :k])
        bad = ~(d > 0)
        ok &= ~bad
        d = np.where(bad, 1.0, d)
        L[:, k, k] = np.sqrt(d)
        if k + 1 < b:
            s = Ab[:, k + 1:, k] - np.einsum("irj,ij->ir", L[:, k + 1:, :k], L[:, k, :k])
            L[:, k + 1:, k] = s / L[:, k, k][:, None]
    return L, ok


def inverse_from_cholesky(L: np.ndarray) -> np.ndarray:
    """A^-1 = L^-T L^-1 by forward substitution L Y = I then back substitution
    L^T X = Y, column-block at a time over the stack."""
    cnt, b, _ = L.shape
    Y = np.zeros_like(L)
    eye = np.eye(b)
    for i in range(b):
        acc = eye[i][None, :] - np.einsum("ij,ijc->ic", L[:, i, :i], Y[:, :i, :])
        Y[:, i, :] = acc / L[:, i, i][:, None]
    X = np.zeros_like(L)
    for i in range(b - 1, -1, -1):
        acc = Y[:, i, :] - np.einsum("ij,ijc->ic", L[:, i + 1:, i], X[:, i + 1:, :])
        X[:, i, :] = acc / L[:, i, i][:, None]
    return X


def invert_blocks(A, block_ptr):
    """FP64 inverses of all diagonal blocks (Sec. 3.1, D_b^-1 of eq. 3-1),
    returned as a list indexed by block. Raises NotSPD on a failed pivot."""
    nb = len(block_ptr) - 1
    H = [None] * nb
    bad = []
    for b, (ids, dense) in extract_blocks(A, block_ptr).items():
        L, ok = cholesky(dense)
        X = inverse_from_cholesky(L)
        for j, k in enumerate(ids):
            H[k] = X[j]
        bad += [int(k) for k in ids[~ok]]
    if bad:
        raise NotSPD(sorted(bad))
    return H


# ------------------------------------------------------------------ features
def row_quantities(A, block_ptr):
    """Per-row FP64 quantities of the full CSR rows used by the block features."""
    n = A.n
    bp = np.asarray(block_ptr, dtype=np.int64)
    rp = A.row_ptr.astype(np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    cols = A.col_idx.astype(np.int64)
    v = A.val
    a = np.abs(v)
    isdiag = rows == cols
    inblk = block_of_rows(bp, rows) == block_of_rows(bp, cols)
    off = ~isdiag

    def rsum(w):
        return np.bincount(rows, weights=w, minlength=n)

    q = {}
    q["d"] = rsum(np.where(isdiag, v, 0.0))
    q["off_full"] = rsum(np.where(off, a, 0.0))
    q["off_in"] = rsum(np.where(off & inblk, a, 0.0))
    q["off2_in"] = rsum(np.where(off & inblk, v * v, 0.0))
    q["off2_out"] = rsum(np.where(~inblk, v * v, 0.0))
    big = np.inf
    tmax = np.full(n, -big)
    np.maximum.at(tmax, rows[off], a[off])
    tmin = np.full(n, big)
    offnz = off & (a > 0)
    np.minimum.at(tmin, rows[offnz], a[offnz])
    has = np.isfinite(tmin) & (tmax > 0)
    q["log10_tau"] = np.where(has, np.log10(np.where(has, tmax / np.where(has, tmin, 1.0), 1.0)), 0.0)
    amax = np.full(n, -big)
    nzr = a > 0
    np.maximum.at(amax, rows[nzr], a[nzr])
    amin = np.full(n, big)
    np.minimum.at(amin, rows[nzr], a[nzr])
    q["amax"], q["amin"] = amax, amin
    return q


def block_features(A, block_ptr, H):
    """The 16 block features (FP64) and the raw quantities the precision rule
    uses. Dominance follows the row sums of Sec. 4.5.2, the multiscale
    strength tau_i is eq. 4-5, the condition number is ||A_ii||_1 ||A_ii^-1||_1.
    Returns (features (nb, 16) float64, raw dict of per-block arrays)."""
    bp = np.asarray(block_ptr, dtype=np.int64)
    nb = len(bp) - 1
    q = row_quantities(A, bp)
    F = np.zeros((nb, NFEAT))
    raw = {k: np.zeros(nb) for k in ("kappa1", "min_dom", "normH1", "normA1")}
    for k in range(nb):
        s, e = bp[k], bp[k + 1]
        b = e - s
        d = q["d"][s:e]
        dom = d / np.maximum(q["off_full"][s:e], d / DOM_CAP)
        dom_in = d / np.maximum(q["off_in"][s:e], d / DOM_CAP)
        gl = np.min(d - q["off_in"][s:e])
        gu = np.max(d + q["off_in"][s:e])
        dmax = np.max(d)
        Hk = H[k]
        aH = np.abs(Hk)
        normH1 = np.max(np.sum(aH, axis=0))
        normA1 = gu            # ||A_ii||_1 = max row sum of |A_ii| for symmetric A_ii with d > 0
        hmax = np.max(aH)
        hdiag = np.diag(Hk)
        F[k, 0] = b / 64.0
        F[k, 1] = np.log10(np.min(dom))
        F[k, 2] = np.log10(np.mean(dom))
        F[k, 3] = np.log10(np.min(dom_in))
        F[k, 4] = np.sqrt(np.sum(q["off2_in"][s:e])) / np.sqrt(np.sum(d * d))
        F[k, 5] = np.sqrt(np.sum(q["off2_out"][s:e])) / np.sqrt(np.sum(d * d))
        F[k, 6] = np.max(q["log10_tau"][s:e])
        F[k, 7] = np.mean(q["log10_tau"][s:e])
        F[k, 8] = np.log10(np.max(q["amax"][s:e]) / np.min(q["amin"][s:e]))
        F[k, 9] = gl / dmax
        F[k, 10] = gu / dmax
        F[k, 11] = np.log10(gu / max(gl, gu * GERSH_FLOOR))
        F[k, 12] = np.log10(dmax / np.min(d))
        F[k, 13] = np.log10(normA1 * normH1)
        F[k, 14] = np.log10(np.max(hdiag) / np.min(hdiag))
        F[k, 15] = np.count_nonzero(aH < np.ldexp(hmax, -24)) / float(b * b)
        raw["kappa1"][k] = normA1 * normH1
        raw["min_dom"][k] = np.min(dom)
        raw["normH1"][k] = normH1
        raw["normA1"][k] = normA1
    return F, raw


# ------------------------------------------------------------ precision maps
RULE_THETA = 1e-2
RULE_D16 = 1.0
DOM_SLACK = 1e-12
U16, U32 = 2.0 ** -11, 2.0 ** -24


def select_rule(raw, theta=RULE_THETA, d16=RULE_D16):
    """Per-block precision rule (adaptive per-block storage in the style of the
    condition-based choice cited in Sec. 2, combined with the finding of
    Sec. 4.5.2 that weak diagonal dominance increases delay): the lowest of
    FP16 / FP32 / FP64 whose unit roundoff u satisfies kappa_1(A_ii) u <= theta;
    FP16 further needs every row's dominance ratio >= d16, tested with a
    relative slack of 1e-12 so that row sums equal in exact arithmetic are not
    misjudged by their rounding."""
    kap = raw["kappa1"]
    dom_ok = raw["min_dom"] * (1.0 + DOM_SLACK) >= d16
    tags = np.full(kap.shape, P.FP64, dtype=np.uint8)
    tags[kap * U32 <= theta] = P.FP32
    tags[(kap * U16 <= theta) & dom_ok] = P.FP16
    return tags


def store_blocks(H, tags):
    """Emulated storage: list of (Hhat, s, tag)."""
    return [P.store_block(Hk, int(t)) + (int(t),) for Hk, t in zip(H, tags)]


# ------------------------------------------------- band-truncated storage
# Cheaper storage of the same preconditioner (not in the paper; the paper's
# M^-1(p_l) stores the whole block inverse in p_l, Sec. 3.2). The inverse of a
# diagonally dominant banded block decays away from its diagonal, so most
# entries are below the resolution of a 16- or 32-bit format relative to the
# block. Band storage keeps the diagonals |i - j| <= w of each block, with the
# smallest w whose dropped part is no larger, in Frobenius norm, than the unit
# roundoff of the block's format times the whole inverse:
#     sum_{|i-j| > w} H_ij^2 <= u_p^2 * sum_ij H_ij^2.
# The kept band is symmetric, taken from the upper triangle
# (entry (i, j) -> H[min(i, j), max(i, j)]), and rounded with the same scale
# as full storage (the block's max|H_ij|).
UNIT_ROUNDOFF = {P.FP64: 2.0 ** -53, P.FP32: 2.0 ** -24, P.BF16: 2.0 ** -8, P.FP16: 2.0 ** -11}


def band_width(H: np.ndarray, rtol: float) -> int:
    """Smallest w >= 0 with sum_{|i-j| > w} H_ij^2 <= rtol^2 sum_ij H_ij^2."""
    H = np.asarray(H, dtype=np.float64)
    b = H.shape[0]
    dist = np.abs(np.subtract.outer(np.arange(b), np.arange(b)))
    total = float(np.sum(H * H))
    for w in range(b):
        dropped = float(np.sum(np.where(dist > w, H * H, 0.0)))
        if dropped <= rtol * rtol * total:
            return w
    return b - 1


def band_part(H: np.ndarray, w: int) -> np.ndarray:
    """Symmetric band of H from its upper triangle: (i, j) with |i - j| <= w
    takes H[min(i, j), max(i, j)], every other entry is zero."""
    H = np.asarray(H, dtype=np.float64)
    U = np.triu(H)
    S = U + np.triu(H, 1).T
    dist = np.abs(np.subtract.outer(np.arange(H.shape[0]), np.arange(H.shape[0])))
    return np.where(dist <= w, S, 0.0)


def store_blocks_band(H, tags, rtol=None):
    """Emulated band storage: list of (Hhat, s, tag, w), Hhat dense with zeros
    outside the band. ``rtol`` None takes each block's unit roundoff."""
    out = []
    for Hk, t in zip(H, tags):
        t = int(t)
        w = band_width(Hk, UNIT_ROUNDOFF[t] if rtol is None else rtol)
        s = P.block_scale(float(np.max(np.abs(Hk))), t)
        out.append((P.round_to_format(band_part(Hk, w) / s, t), s, t, w))
    return out


def band_bytes(store, block_ptr) -> int:
    """Stored bytes of a band map in the GPU layout: block k keeps w_k + 1
    diagonals of bpad_k entries (bpad = size rounded up to 16)."""
    sizes = block_sizes(block_ptr)
    return int(sum(((int(b) + 15) // 16 * 16) * (e[3] + 1) * P.BYTES[e[2]] for b, e in zip(sizes, store)))


def apply(store, block_ptr, r):
    """z = M^-1 r for k = 1 (eq. 3-1): per block z_blk = s * Hhat r_in with
    r_in = r for FP64 blocks and the FP32 copy of r otherwise (Algorithm 3.1,
    ConvertPrecision before the product, widening after)."""
    bp = np.asarray(block_ptr, dtype=np.int64)
    r = np.asarray(r, dtype=np.float64)
    z = np.empty_like(r)
    r32 = P.rhat(r)
    for k, e in enumerate(store):
        Hh, s, t = e[:3]
        a, b = bp[k], bp[k + 1]
        rin = r[a:b] if t == P.FP64 else r32[a:b]
        z[a:b] = s * (Hh @ rin)
    return z


def apply_abs(store, block_ptr, r):
    """|z|-bound helper: per block s * |Hhat| |r_in| (for rounding-error bounds)."""
    bp = np.asarray(block_ptr, dtype=np.int64)
    r32 = P.rhat(r)
    out = np.empty_like(np.asarray(r, dtype=np.float64))
    for k, e in enumerate(store):
        Hh, s, t = e[:3]
        a, b = bp[k], bp[k + 1]
        rin = r[a:b] if t == P.FP64 else r32[a:b]
        out[a:b] = s * (np.abs(Hh) @ np.abs(rin))
    return out
