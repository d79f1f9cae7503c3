"""Seeded synthetic inputs: sparse SPD diffusion matrices in CSR form, right-hand
sides and contiguous row-block partitions.

This module is shared by the GPU path, the tests and the CPU oracle's callers.
It holds only the discretisation of the model PDE (the *input* of the method),
never any step of the preconditioner or of the Krylov solver.

Discretisation (paper Sec. 4.1.1, eq. 4-1 and Table 4.1):
  * interior points of a vertex-centred grid on (0,1)^3, x_i = i/(N+1), ordered
    lexicographically with x fastest, Dirichlet unknowns eliminated;
  * 7-point finite differences; the coefficient on the face between two grid
    points is the harmonic mean of their point coefficients (this reading
    reproduces the multiscale distributions of Table 4.3);
  * a face to an eliminated boundary point uses the interior point's own
    coefficient; no h^2 scaling (it changes no iteration count);
  * anisotropy multiplies the x / y / z face coefficients (Sec. 4.1.1 item 2).
The resulting matrix has nnz = N^3 + 6 N^2 (N - 1) (Table 4.1: 14,581,760 at
N = 128) and is a symmetric, weakly diagonally dominant M-matrix.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class CSR:
    """Square sparse matrix. int32 row_ptr[n+1], int32 col_idx[nnz] (sorted per
    row), float64 val[nnz]."""
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.val.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.n))


def _csr_from_coo(n, rows, cols, vals) -> CSR:
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("matrix too large for int32 CSR")
    return CSR(n, row_ptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64))


def diffusion3d(kappa: np.ndarray, aniso=(1.0, 1.0, 1.0)) -> CSR:
    """7-point matrix for -div(K grad u) with point coefficients ``kappa``
    (shape (nz, ny, nx)) and K = diag(aniso) * kappa. Assembled row by row in
    column order (-z, -y, -x, centre, +x, +y, +z), so the CSR needs no sort."""
    kappa = np.asarray(kappa, dtype=np.float64)
    nz, ny, nx = kappa.shape
    n = nx * ny * nz
    if 7 * n >= 2**31:
        raise ValueError("matrix too large for int32 CSR")
    idx = np.arange(n, dtype=np.int64).reshape(nz, ny, nx)
    diag = np.zeros((nz, ny, nx))
    cols = np.full((nz, ny, nx, 7), -1, dtype=np.int64)
    vals = np.zeros((nz, ny, nx, 7))
    # slot of the lower / upper neighbour along x, y, z in the row order above
    for axis, a, (slo, shi) in zip((2, 1, 0), aniso, ((2, 4), (1, 5), (0, 6))):
        k0 = np.moveaxis(kappa, axis, 0)
        i0 = np.moveaxis(idx, axis, 0)
        d0 = np.moveaxis(diag, axis, 0)
        c0 = np.moveaxis(cols, axis, 0)
        v0 = np.moveaxis(vals, axis, 0)
        lo, hi = k0[:-1], k0[1:]
        face = a * (2.0 * lo * hi / (lo + hi))          # interior faces
        d0[:-1] += face
        d0[1:] += face
        d0[0] += a * k0[0]                               # Dirichlet faces
        d0[-1] += a * k0[-1]
        c0[:-1, ..., shi] = i0[1:]                       # row at lower point -> upper neighbour
        v0[:-1, ..., shi] = -face
        c0[1:, ..., slo] = i0[:-1]
        v0[1:, ..., slo] = -face
    cols[..., 3] = idx
    vals[..., 3] = diag
    cols = cols.reshape(n, 7)
    vals = vals.reshape(n, 7)
    keep = cols >= 0
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(keep.sum(axis=1), out=row_ptr[1:])
    A = CSR(n, row_ptr.astype(np.int32), cols[keep].astype(np.int32), vals[keep])
    A.meta.update(shape=(nz, ny, nx), aniso=tuple(float(a) for a in aniso))
    return A


def poisson2d(nx: int, ny: int) -> CSR:
    """5-point Laplacian on an nx x ny interior grid (diag 4, off-diagonals -1)."""
    n = nx * ny
    idx = np.arange(n, dtype=np.int64).reshape(ny, nx)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [np.full(n, 4.0)]
    for a, b in ((idx[:, :-1], idx[:, 1:]), (idx[:-1, :], idx[1:, :])):
        a, b = a.ravel(), b.ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [np.full(a.size, -1.0), np.full(a.size, -1.0)]
    A = _csr_from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))
    A.meta.update(shape=(ny, nx))
    return A


# ---------------------------------------------------------------- coefficients
def grid_coords(N: int) -> np.ndarray:
    """Vertex-centred interior coordinates i/(N+1), i = 1..N."""
    return np.arange(1, N + 1, dtype=np.float64) / (N + 1)


def kappa_const(N):
    return np.ones((N, N, N))


def kappa_dis(N, s):
    """Diff3D-Dis(s): kappa = s on [0.25, 0.75]^3, 1 elsewhere (Sec. 4.1.1 item 3)."""
    x = grid_coords(N)
    inside = (x >= 0.25) & (x <= 0.75)
    m = inside[:, None, None] & inside[None, :, None] & inside[None, None, :]
    return np.where(m, float(s), 1.0)


def kappa_rand(N, s, rng):
    """Diff3D-Rand(s): kappa = s**delta, delta i.i.d. U[0,1] per grid point."""
    return float(s) ** rng.uniform(0.0, 1.0, size=(N, N, N))


def kappa_loguniform(shape, rng, lo=-2.0, hi=2.0):
    """Point coefficients 10**U(lo, hi)."""
    return 10.0 ** rng.uniform(lo, hi, size=shape)


def kappa_subcube_jumps(N, rng, ncubes=16, jump=1e4):
    """Piecewise-constant coefficient: jump on the union of ``ncubes`` random
    axis-aligned subcubes with integer edges in [N/16, N/4] and uniform corners."""
    kap = np.ones((N, N, N))
    lo_e, hi_e = max(1, N // 16), max(1, N // 4)
    for _ in range(ncubes):
        e = rng.integers(lo_e, hi_e + 1, size=3)
        c = [rng.integers(0, N - e[d] + 1) for d in range(3)]
        kap[c[0]:c[0] + e[0], c[1]:c[1] + e[1], c[2]:c[2] + e[2]] = jump
    return kap


# ----------------------------------------------------------------- partitions
def uniform_blocks(n: int, b: int) -> np.ndarray:
    """Contiguous row blocks of b rows; the last block holds the remainder."""
    starts = np.arange(0, n, b, dtype=np.int64)
    return np.append(starts, n).astype(np.int32)


def random_blocks(n: int, rng, sizes=(16, 32, 48, 64)) -> np.ndarray:
    """Contiguous row blocks with sizes drawn i.i.d. from ``sizes``; the last
    block is truncated at n."""
    ptr = [0]
    while ptr[-1] < n:
        ptr.append(min(n, ptr[-1] + int(rng.choice(sizes))))
    return np.asarray(ptr, dtype=np.int32)


def rhs_uniform(n: int, rng, ncols: int | None = None) -> np.ndarray:
    shape = (n,) if ncols is None else (n, ncols)
    return rng.uniform(-1.0, 1.0, size=shape)


# ------------------------------------------------------------ named workloads
@dataclass
class Problem:
    name: str
    A: CSR
    block_ptr: np.ndarray
    b: np.ndarray
    tol: float
    maxit: int


def config1(seed=0) -> Problem:
    """2D 5-point Poisson 64x64, row blocks of 64, RHS U[-1,1], tol 1e-8."""
    rng = np.random.default_rng(seed)
    A = poisson2d(64, 64)
    return Problem("poisson2d_64x64_b64", A, uniform_blocks(A.n, 64), rhs_uniform(A.n, rng), 1e-8, 1000)


def config2(seed=0, N=128, b=32, contrast=2.0) -> Problem:
    """3D 7-point diffusion, point coefficients 10**U(-c, c) (c = 2: the
    benchmark workload; c = 0: constant coefficient), row blocks of 32."""
    rng = np.random.default_rng(seed)
    kap = kappa_loguniform((N, N, N), rng, -contrast, contrast)
    A = diffusion3d(kap)
    return Problem(f"diff3d_loguniform{contrast:g}_{N}^3_b{b}", A, uniform_blocks(A.n, b),
                   rhs_uniform(A.n, rng), 1e-10, 5000)


def aniso_jump_problem(seed=0, N=160, b=48, name="aniso_jump", ratio=1e3, strong="x") -> Problem:
    """Anisotropic diffusion K = diag(ratio, 1, 1) * kappa, kappa = 1e4 on 16
    random subcubes and 1 elsewhere, row blocks of 48. The strong coupling runs
    along x, the fastest index, so that the contiguous row blocks contain it.
    strong="yz" gives the orientation of the paper's Ani(s), K = diag(1, s, s):
    the strong axes then run across the blocks, and block-Jacobi with 48-row
    blocks drops every strong coupling."""
    rng = np.random.default_rng(seed)
    kap = kappa_subcube_jumps(N, rng)
    A = diffusion3d(kap, aniso=(ratio, 1.0, 1.0) if strong == "x" else (1.0, ratio, ratio))
    return Problem(f"{name}_{N}^3_b{b}", A, uniform_blocks(A.n, b), rhs_uniform(A.n, rng), 1e-10, 5000)


def config3(seed=0, N=160, b=48) -> Problem:
    return aniso_jump_problem(seed, N, b, "diff3d_aniso1e3_jump1e4")


def config5_eval(seed=100, N=192, b=48) -> Problem:
    return aniso_jump_problem(seed, N, b, "diff3d_aniso1e3_jump1e4")


@dataclass
class BatchSystem:
    A: CSR
    block_ptr: np.ndarray
    B: np.ndarray          # (n, nrhs) right-hand sides


def config4(seed=0, nsys=256, edge=(32, 96), nrhs=(1, 8)) -> list:
    """Independent SPD 7-point systems: grid edges U{edge}, coefficients
    10**U(-2,2), blocks i.i.d. from {16,32,48,64}, nrhs U{nrhs} columns."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nsys):
        nx, ny, nz = (int(v) for v in rng.integers(edge[0], edge[1] + 1, size=3))
        kap = kappa_loguniform((nz, ny, nx), rng)
        A = diffusion3d(kap)
        bp = random_blocks(A.n, rng)
        m = int(rng.integers(nrhs[0], nrhs[1] + 1))
        out.append(BatchSystem(A, bp, rhs_uniform(A.n, rng, m)))
    return out


def spd_exact_inverse_blocks(nb: int, b: int, rng) -> CSR:
    """Block-diagonal SPD matrix whose diagonal blocks are L L^T with L unit lower
    bidiagonal (sub-diagonal -1), permuted symmetrically by a random sign
    diagonal. Each block's inverse is an integer matrix (entries b - max(i,j)
    up to sign), so every exact elimination reaches it without rounding."""
    n = nb * b
    rows, cols, vals = [], [], []
    for k in range(nb):
        sgn = rng.choice([-1.0, 1.0], size=b)
        base = k * b
        i = np.arange(b)
        d = np.full(b, 2.0)
        d[0] = 1.0
        rows += [base + i, base + i[1:], base + i[:-1]]
        cols += [base + i, base + i[:-1], base + i[1:]]
        off = -sgn[1:] * sgn[:-1]
        vals += [d, off, off]
    A = _csr_from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))
    return A


@dataclass
class StackedBatch:
    """Independent systems stacked into one block-diagonal CSR: system s owns
    rows sys_row[s] .. sys_row[s+1]-1; its block partition is shifted by
    sys_row[s]; b is system-major, row-major (rows_s, m_s) per system."""
    A: CSR
    block_ptr: np.ndarray
    sys_row: np.ndarray
    sys_m: np.ndarray
    b: np.ndarray

    def system_slice(self, s: int) -> slice:
        off = int(np.sum(np.diff(self.sys_row[:s + 1]).astype(np.int64) * self.sys_m[:s]))
        return slice(off, off + int(self.sys_row[s + 1] - self.sys_row[s]) * int(self.sys_m[s]))


def stack_batch(systems: list) -> StackedBatch:
    sizes = np.array([bs.A.n for bs in systems], dtype=np.int64)
    sys_row = np.zeros(len(systems) + 1, dtype=np.int64)
    np.cumsum(sizes, out=sys_row[1:])
    nnz = np.array([bs.A.nnz for bs in systems], dtype=np.int64)
    if sys_row[-1] >= 2**31 or nnz.sum() >= 2**31:
        raise ValueError("batch too large for int32 CSR")
    nnz_off = np.concatenate([[0], np.cumsum(nnz)])
    row_ptr = np.concatenate([bs.A.row_ptr[:-1].astype(np.int64) + nnz_off[i] for i, bs in enumerate(systems)]
                             + [[nnz_off[-1]]])
    col_idx = np.concatenate([bs.A.col_idx.astype(np.int64) + sys_row[i] for i, bs in enumerate(systems)])
    val = np.concatenate([bs.A.val for bs in systems])
    bp = np.concatenate([bs.block_ptr[:-1].astype(np.int64) + sys_row[i] for i, bs in enumerate(systems)]
                        + [[sys_row[-1]]])
    sys_m = np.array([bs.B.shape[1] for bs in systems], dtype=np.int32)
    b = np.concatenate([np.ascontiguousarray(bs.B).ravel() for bs in systems])
    A = CSR(int(sys_row[-1]), row_ptr.astype(np.int32), col_idx.astype(np.int32), val)
    return StackedBatch(A, bp.astype(np.int32), sys_row.astype(np.int32), sys_m, b)


# ------------------------------------------- radiation-diffusion-like systems
def rhd3t_like(N: int, seed=0, interlace=True) -> CSR:
    """Synthetic coupled three-temperature system with the block structure of
    eq. 4-3: each diagonal block a 7-point
    diffusion operator plus a positive diagonal (heat capacity over time step
    and the exchange terms), the couplings D_RE = D_ER = -w_er and D_EI = D_IE =
    -w_ei diagonal. The RHD3D matrices themselves are not available. As in
    Table 4.3, the diffusion coefficients vary mildly inside each temperature
    (the single-temperature rows stay below multiscale strength 10) while the
    exchange coefficients and the temperatures' diffusion scales differ by many
    decades, which spreads the coupled rows' strength (eq. 4-5) over 1 to 10^12:
      K_r = 10^(3 + U(-1/2, 1/2)), K_e = 10^U(-1/2, 1/2), K_i = 10^(-5 + U(-1/2, 1/2)),
      w_er = 10^U(-2, 0), w_ei = 10^U(0, 6), c_r = 10^U(-2, 0), c_e, c_i = 10^U(-1, 1).
    The radiation block is dominated by its diffusion (its smallest
    eigenvalues near 3 pi^2 K_r / (N+1)^2 compete with c_r + w_er), so its
    single-temperature system needs hundreds of iterations like RHD3D-1T.
    Symmetric, strictly diagonally dominant, off-diagonals <= 0 (an M-matrix).
    nnz = 3 (N^3 + 6 N^2 (N - 1)) + 4 N^3 (52,133,888 at N = 128).
    Ordering: interlace=False is eq. 4-3's [T_r; T_e; T_i]; interlace=True
    (default) numbers the three temperatures of a cell consecutively (a
    symmetric permutation of it), so that contiguous row blocks hold the
    exchange couplings, which reach 10^6 times the smallest diagonal terms
    and which row blocks of the [T_r; T_e; T_i] ordering cannot see."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    shape = (N, N, N)
    K = [10.0 ** (m + rng.uniform(-0.5, 0.5, size=shape)) for m in (3.0, 0.0, -5.0)]
    w_er = (10.0 ** rng.uniform(-2, 0, size=shape)).ravel()
    w_ei = (10.0 ** rng.uniform(0, 6, size=shape)).ravel()
    c = [(10.0 ** rng.uniform(lo, hi, size=shape)).ravel() for lo, hi in ((-2, 0), (-1, 1), (-1, 1))]
    L = [diffusion3d(k).to_scipy() for k in K]
    diag_add = [c[0] + w_er, c[1] + w_er + w_ei, c[2] + w_ei]
    blocks = [[(L[i] + sp.diags(diag_add[i])) if i == j else None for j in range(3)] for i in range(3)]
    Der = sp.diags(-w_er)
    Dei = sp.diags(-w_ei)
    blocks[0][1] = Der
    blocks[1][0] = Der
    blocks[1][2] = Dei
    blocks[2][1] = Dei
    S = sp.bmat(blocks, format="csr")
    n = S.shape[0]
    if interlace:
        m = N ** 3
        new = np.empty(n, dtype=np.int64)            # new index of old unknown (temperature t, cell i)
        cell = np.arange(m)
        for t in range(3):
            new[t * m + cell] = 3 * cell + t
        P = sp.csr_matrix((np.ones(n), (new, np.arange(n))), shape=(n, n))
        S = (P @ S @ P.T).tocsr()
    S.sort_indices()
    A = CSR(n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64))
    A.meta.update(shape=(3,) + shape, kind="rhd3t_like", interlace=bool(interlace))
    return A


def rhd1t_like(N: int, seed=0) -> CSR:
    """The single-temperature reduction: the radiation block A_R of
    rhd3t_like (same fields and draws)."""
    A3 = rhd3t_like(N, seed, interlace=False)
    n = N ** 3
    rp = A3.row_ptr[:n + 1].astype(np.int64)
    keep = A3.col_idx[:rp[-1]] < n
    rows = np.repeat(np.arange(n), np.diff(rp))[keep]
    return _csr_from_coo(n, rows, A3.col_idx[:rp[-1]][keep].astype(np.int64), A3.val[:rp[-1]][keep])


def with_pdiag(A: CSR, p: float) -> CSR:
    """Sec. 4.5.2's diagonal-dominance control: every diagonal entry gains
    p times the row's sum of off-diagonal magnitudes."""
    rp = A.row_ptr.astype(np.int64)
    rows = np.repeat(np.arange(A.n), np.diff(rp))
    off = rows != A.col_idx
    s = np.bincount(rows[off], weights=np.abs(A.val[off]), minlength=A.n)
    val = A.val.copy()
    d = ~off
    val[d] = val[d] + p * s[rows[d]]
    return CSR(A.n, A.row_ptr.copy(), A.col_idx.copy(), val, dict(A.meta, pdiag=p))
