"""Pins of the oracle's PCG and its block-Jacobi variants against facts the
mathematics fixes: finite termination, exact preconditioning, closed-form
spectra, degenerate cases of the adaptive switch."""
import math

import numpy as np
import pytest

from paper_2407_15973_amd import gen
from oracle import blocks as OB
from oracle import pcg as OP
from oracle import precision as P


def _spd(rng, n):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * np.exp(rng.uniform(0, 3, n))) @ Q.T


def _dense_csr(D):
    n = D.shape[0]
    r, c = np.nonzero(D)
    return gen._csr_from_coo(n, r, c, D[r, c])


@pytest.mark.parametrize("n", [1, 2, 5, 8, 10])
def test_tiny_spd_converges_within_n(n):
    rng = np.random.default_rng(n)
    D = _spd(rng, n)
    A = _dense_csr(D)
    b = rng.uniform(-1, 1, n)
    res = OP.solve_bjac(A, gen.uniform_blocks(n, 1), b, tol=1e-10, maxit=50)
    assert res.status == OP.CONVERGED and res.iters <= n
    np.testing.assert_allclose(D @ res.x, b, atol=1e-8)


def test_whole_matrix_block_is_exact_one_iteration():
    A = gen.poisson2d(16, 16)
    b = np.random.default_rng(0).uniform(-1, 1, A.n)
    res = OP.solve_bjac(A, gen.uniform_blocks(A.n, A.n), b, tol=1e-8, maxit=10)
    assert res.iters == 1 and res.status == OP.CONVERGED
    assert OP.true_relres(A, res.x, b) < 1e-12


def test_block_size_one_is_point_jacobi():
    rng = np.random.default_rng(2)
    A = gen.diffusion3d(gen.kappa_loguniform((8, 8, 8), rng))
    b = rng.uniform(-1, 1, A.n)
    S = A.to_scipy()
    d = S.diagonal()
    ref = OP.pcg(lambda v: S @ v, b, lambda r: r / d, 1e-10, 1000)
    res = OP.solve_bjac(A, gen.uniform_blocks(A.n, 1), b, tol=1e-10, maxit=1000)
    assert abs(res.iters - ref.iters) <= 1
    np.testing.assert_allclose(res.x, ref.x, rtol=0, atol=1e-9 * np.abs(ref.x).max())


def test_poisson1d_eigen_components_finite_termination():
    # 1D Laplacian tridiag(-1,2,-1): eigenvalues 2 - 2cos(j pi/(n+1)), vectors
    # sin(i j pi/(n+1)); block size 1 gives M^-1 A = A/2, so an RHS with m
    # eigen-components is solved in m steps
    n = 60
    i = np.arange(n)
    A = gen._csr_from_coo(n, np.concatenate([i, i[1:], i[:-1]]), np.concatenate([i, i[:-1], i[1:]]),
                          np.concatenate([np.full(n, 2.0), -np.ones(n - 1), -np.ones(n - 1)]))
    lam = 2 - 2 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    V = np.sin(np.outer(np.arange(1, n + 1), np.arange(1, n + 1)) * np.pi / (n + 1))
    np.testing.assert_allclose(A.to_scipy() @ V, V * lam, atol=1e-12)
    for m in (1, 3, 7):
        b = V[:, [4, 17, 31, 40, 50, 55, 58][:m]].sum(axis=1)
        res = OP.solve_bjac(A, gen.uniform_blocks(n, 1), b, tol=1e-10, maxit=100)
        assert res.iters == m


def _line_block_spectrum(m):
    mu = 2 - 2 * np.cos(np.arange(1, m + 1) * np.pi / (m + 1))
    # D_b^-1 A of the m x m 5-point Laplacian with grid-line blocks: the block
    # is T = tridiag(-1,4,-1) = K + 2I, A = K(x)I + I(x)K, so the spectrum is
    # (mu_j + mu_k)/(mu_k + 2) with mu the eigenvalues of K = tridiag(-1,2,-1)
    ev = (mu[:, None] + mu[None, :]) / (mu[None, :] + 2)
    return ev.max() / ev.min(), ev


def test_line_block_closed_form_spectrum():
    m = 20
    A = gen.poisson2d(m, m)
    bp = gen.uniform_blocks(A.n, m)
    H = OB.invert_blocks(A, bp)
    Dinv = np.zeros((A.n, A.n))
    for k, h in enumerate(H):
        Dinv[m * k:m * (k + 1), m * k:m * (k + 1)] = h
    ev_num = np.sort(np.linalg.eigvals(Dinv @ A.to_scipy().toarray()).real)
    _, ev = _line_block_spectrum(m)
    np.testing.assert_allclose(ev_num, np.sort(ev.ravel()), rtol=0, atol=1e-12)


def test_config1_closed_form_spectrum_and_cg_bound():
    p = gen.config1(0)
    kap, _ = _line_block_spectrum(64)
    assert abs(kap - 856.33) < 0.01
    bound = math.ceil(0.5 * math.sqrt(kap) * math.log(2 / 1e-8))
    assert bound == 280
    res = OP.solve_bjac(p.A, p.block_ptr, p.b, tol=p.tol, maxit=p.maxit)
    assert res.status == OP.CONVERGED and res.iters <= bound


def test_config1_single_mode_one_iteration():
    p = gen.config1(0)
    s = np.sin(np.arange(1, 65) * 3 * np.pi / 65)
    b = np.outer(np.sin(np.arange(1, 65) * 5 * np.pi / 65), s).ravel()
    res = OP.solve_bjac(p.A, p.block_ptr, b, tol=1e-8, maxit=10)
    assert res.iters == 1


def test_a_norm_error_monotone():
    rng = np.random.default_rng(4)
    A = gen.diffusion3d(gen.kappa_loguniform((10, 10, 10), rng))
    S = A.to_scipy()
    xs = rng.uniform(-1, 1, A.n)
    b = S @ xs
    bp = gen.uniform_blocks(A.n, 10)
    M = OP.BJAC(A, bp)
    errs = []
    for it in range(1, 40):
        res = OP.pcg(lambda v: S @ v, b, M.low, 0.0, it)
        e = res.x - xs
        errs.append(e @ (S @ e))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))


def _mixed_case():
    rng = np.random.default_rng(5)
    A = gen.diffusion3d(gen.kappa_loguniform((12, 12, 12), rng))
    bp = gen.uniform_blocks(A.n, 24)
    b = rng.uniform(-1, 1, A.n)
    return A, bp, b


def test_adaptive_degenerations_bitwise():
    A, bp, b = _mixed_case()
    tags = np.full(len(bp) - 1, P.FP16, np.uint8)
    M = OP.BJAC(A, bp, tags)
    uni = OP.solve_bjac(A, bp, b, np.zeros_like(tags), tol=1e-10, M=OP.BJAC(A, bp, None, H=M.H))
    fmp = OP.solve_bjac(A, bp, b, tags, tol=1e-10, M=M)
    # hl with adp_tol = 0 is always high: uniform BJAC; lh with adp_tol = 0 is always low: fMP
    hl0 = OP.solve_bjac(A, bp, b, tags, tol=1e-10, temporal=OP.TEMPORAL_HL, adp_tol=0.0, M=M)
    lh0 = OP.solve_bjac(A, bp, b, tags, tol=1e-10, temporal=OP.TEMPORAL_LH, adp_tol=0.0, M=M)
    assert np.array_equal(hl0.x, uni.x) and hl0.iters == uni.iters
    assert np.array_equal(lh0.x, fmp.x) and lh0.iters == fmp.iters
    # very large adp_tol: only the first application (relres = +inf) differs
    hlI = OP.solve_bjac(A, bp, b, tags, tol=1e-10, temporal=OP.TEMPORAL_HL, adp_tol=1e300, M=M)
    lhI = OP.solve_bjac(A, bp, b, tags, tol=1e-10, temporal=OP.TEMPORAL_LH, adp_tol=1e300, M=M)
    assert hlI.used_high[0] and not any(hlI.used_high[1:])
    assert not lhI.used_high[0] and all(lhI.used_high[1:])
    # the FP64 "low" map is uniform BJAC exactly
    same = OP.solve_bjac(A, bp, b, np.zeros_like(tags), tol=1e-10, M=OP.BJAC(A, bp, None, H=M.H))
    assert np.array_equal(same.x, uni.x)


def test_adaptive_switch_follows_relres():
    A, bp, b = _mixed_case()
    tags = np.full(len(bp) - 1, P.FP32, np.uint8)
    M = OP.BJAC(A, bp, tags)
    res = OP.solve_bjac(A, bp, b, tags, tol=1e-10, temporal=OP.TEMPORAL_HL, adp_tol=1e-4, M=M)
    rel = [math.inf] + res.history[:-1]           # relres seen by each application
    assert res.used_high == [rr >= 1e-4 for rr in rel]


def test_mixed_precision_true_residual_floor():
    # fMP and uniform reach the same limiting accuracy of the true residual (Sec. 4.5.1)
    A, bp, b = _mixed_case()
    M16 = OP.BJAC(A, bp, np.full(len(bp) - 1, P.FP16, np.uint8))
    r16 = OP.solve_bjac(A, bp, b, M16.tags, tol=1e-14, maxit=400, M=M16)
    r64 = OP.solve_bjac(A, bp, b, None, tol=1e-14, maxit=400)
    t16, t64 = OP.true_relres(A, r16.x, b), OP.true_relres(A, r64.x, b)
    assert t16 < 1e-12 and t64 < 1e-12 and t16 / t64 < 100


def test_poly_bjac_k_t_one_is_diagonal_scaling():
    # Sec. 3.1: k = t = 1 degenerates to D^-1
    rng = np.random.default_rng(6)
    A = gen.diffusion3d(gen.kappa_loguniform((6, 6, 6), rng))
    bp = gen.uniform_blocks(A.n, A.n // 4)
    M = OP.PolyBJAC(A, bp, k=1, t=1)
    r = rng.uniform(-1, 1, A.n)
    np.testing.assert_array_equal(M(r), (1.0 / A.to_scipy().diagonal()) * r)


def test_poly_bjac_polynomial_definition():
    # eq. 3-1 / 3-3 as explicit matrix polynomials on a small problem
    rng = np.random.default_rng(7)
    A = gen.diffusion3d(gen.kappa_loguniform((4, 4, 4), rng))
    S = A.to_scipy().toarray()
    bp = gen.uniform_blocks(A.n, 16)
    Db = np.zeros_like(S)
    for k in range(len(bp) - 1):
        Db[bp[k]:bp[k + 1], bp[k]:bp[k + 1]] = S[bp[k]:bp[k + 1], bp[k]:bp[k + 1]]
    Dd = np.diag(np.diag(S))
    I = np.eye(A.n)
    for k, t in ((1, 3), (2, 2), (3, 1), (2, 4)):
        Dhat = sum(np.linalg.matrix_power(I - np.linalg.solve(Dd, Db), i) for i in range(t)) @ np.linalg.inv(Dd)
        Mk = sum(np.linalg.matrix_power(I - Dhat @ S, j) for j in range(k)) @ Dhat
        r = rng.uniform(-1, 1, A.n)
        np.testing.assert_allclose(OP.PolyBJAC(A, bp, k=k, t=t)(r), Mk @ r, rtol=0, atol=1e-12)
    Mk = sum(np.linalg.matrix_power(I - np.linalg.solve(Db, S), j) for j in range(2)) @ np.linalg.inv(Db)
    r = rng.uniform(-1, 1, A.n)
    np.testing.assert_allclose(OP.PolyBJAC(A, bp, k=2, exact=True)(r), Mk @ r, rtol=0, atol=1e-12)


def test_paper_mode_const_replication():
    # Table 4.2 / Sec. 4.4.1: Diff3D-Const, 32 blocks, k = t = 2, tol 1e-10:
    # 148 (fp64) -> 165 (fp32 fMP). Partition, ordering and f are unstated, so soft (+-5%).
    # About a minute on one core: the full-size pin of the FP32 paper mode.
    N = 128
    A = gen.diffusion3d(gen.kappa_const(N))
    bp = gen.uniform_blocks(A.n, A.n // 32)
    b = np.ones(A.n)
    r64 = OP.solve_poly(A, bp, b, 2, 2, low=False, tol=1e-10)
    r32 = OP.solve_poly(A, bp, b, 2, 2, low=True, tol=1e-10)
    assert abs(r64.iters - 148) <= 0.05 * 148
    assert abs(r32.iters - 165) <= 0.05 * 165 and r32.iters > r64.iters


def test_band_storage_at_unit_roundoff_keeps_iterations():
    # truncation below each format's unit roundoff perturbs M no more than the
    # rounding already does: the PCG iteration counts stay within one
    rng = np.random.default_rng(11)
    A = gen.diffusion3d(gen.kappa_loguniform((12, 10, 8), rng))
    bp = gen.uniform_blocks(A.n, 12)
    b = rng.uniform(-1, 1, A.n)
    H = OB.invert_blocks(A, bp)
    for t in (P.FP64, P.FP32, P.FP16):
        tags = np.full(len(H), t, dtype=np.uint8)
        full = OP.solve_bjac(A, bp, b, M=OP.BJAC(A, bp, tags, H=H), tol=1e-10)
        band = OP.solve_bjac(A, bp, b, M=OP.BJAC(A, bp, tags, H=H, band=True), tol=1e-10)
        assert full.status == OP.CONVERGED and band.status == OP.CONVERGED
        assert abs(full.iters - band.iters) <= 1


# ------------------------------------------- FP32 paper mode (low=True) pins
# Sec. 3.2: in fMP every floating-point operation of M^-1(p_l) runs in p_l
# (fp32): r is rounded to fp32 on entry (Algorithm 3.1), A's values and the
# inverted diagonal are fp32 copies (the inversion 1/a_ii itself is set-up
# work, done in fp64 and then rounded), and z is widened on exit.

def test_poly_bjac_low_k_t_one_is_rounded_diagonal_scaling():
    # k = t = 1: z = fp64(fp32(1/a_ii) * fp32(r)), one fp32 multiply per entry
    rng = np.random.default_rng(21)
    A = gen.diffusion3d(gen.kappa_loguniform((6, 6, 6), rng))
    bp = gen.uniform_blocks(A.n, A.n // 4)
    r = rng.uniform(-1, 1, A.n)
    d = A.to_scipy().diagonal()
    ref = (np.float32(1.0) * (1.0 / d).astype(np.float32) * r.astype(np.float32)).astype(np.float64)
    got = OP.PolyBJAC(A, bp, k=1, t=1, low=True)(r)
    assert got.dtype == np.float64
    np.testing.assert_array_equal(got, ref)
    # and it is not the fp64 scaling (the fp32 rounding is visible)
    assert np.any(got != r / d)


def _tiny_chain():
    """1D tridiagonal SPD matrix of 6 rows in two blocks of 3, with entries and
    a right-hand side that fp32 cannot represent exactly."""
    n = 6
    diag = np.array([3.1, 2.7, 3.3, 2.9, 3.7, 3.05])
    off = np.array([-1.3, -0.7, -1.1, -0.9, -1.45])
    i = np.arange(n)
    A = gen._csr_from_coo(n, np.concatenate([i, i[1:], i[:-1]]), np.concatenate([i, i[:-1], i[1:]]),
                          np.concatenate([diag, off, off]))
    r = np.random.default_rng(23).uniform(-1, 1, n)
    return A, np.array([0, 3, 6]), r


def _scalar_chain(A, bp, r, k, t, residual_fp64=False, round_entry=True):
    """Eq. 3-1 (k outer steps) with eq. 3-3's block solve (t point-Jacobi
    sweeps from zero), one scalar operation at a time on numpy float32
    scalars (each + - * correctly rounded to fp32), row sums in column order.
    The flags produce the two plausible mistakes the test must tell apart."""
    f32 = np.float32
    n = A.n
    rp, ci, va = A.row_ptr, A.col_idx, A.val
    blk = np.searchsorted(bp, np.arange(n), side="right") - 1
    dinv = [f32(1.0 / va[[k for k in range(rp[i], rp[i + 1]) if ci[k] == i][0]]) for i in range(n)]
    v = [f32(x) if round_entry else np.float64(x) for x in r]

    def rowsum(i, y, same_block):
        acc = f32(0.0)
        for kk in range(rp[i], rp[i + 1]):
            j = ci[kk]
            if same_block and blk[j] != blk[i]:
                continue
            acc = acc + f32(va[kk]) * y[j]
        return acc

    def dhat(w):
        y = [dinv[i] * w[i] for i in range(n)]
        for _ in range(t - 1):
            y = [y[i] + dinv[i] * (w[i] - rowsum(i, y, True)) for i in range(n)]
        return y

    z = dhat(v)
    for _ in range(k - 1):
        if residual_fp64:
            res = [f32(float(v[i]) - sum(float(va[kk]) * float(z[ci[kk]]) for kk in range(rp[i], rp[i + 1])))
                   for i in range(n)]
        else:
            res = [v[i] - rowsum(i, z, False) for i in range(n)]
        d = dhat(res)
        z = [z[i] + d[i] for i in range(n)]
    return np.array([float(x) for x in z])


def test_poly_bjac_low_matches_scalar_fp32_chain():
    A, bp, r = _tiny_chain()
    for k, t in ((1, 2), (2, 1), (2, 2), (3, 3)):
        got = OP.PolyBJAC(A, bp, k=k, t=t, low=True)(r)
        np.testing.assert_array_equal(got, _scalar_chain(A, bp, r, k, t))
    # the inputs separate the plausible mistakes: an fp64 residual r - A z,
    # an unrounded r, or the fp64 evaluation all give other values
    got = OP.PolyBJAC(A, bp, k=2, t=2, low=True)(r)
    assert np.any(got != _scalar_chain(A, bp, r, 2, 2, residual_fp64=True))
    assert np.any(got != _scalar_chain(A, bp, r, 2, 2, round_entry=False))
    assert np.any(got != OP.PolyBJAC(A, bp, k=2, t=2, low=False)(r))


def test_poly_bjac_low_exact_on_representable_values():
    # 5-point Laplacian (diagonal 4: 1/4 exact, off-diagonals -1) and a dyadic
    # right-hand side: every fp32 operation is exact, so the low mode equals
    # the fp64 evaluation bit for bit
    A = gen.poisson2d(8, 8)
    bp = gen.uniform_blocks(A.n, 8)
    r = np.random.default_rng(23).integers(-8, 9, A.n) / 8.0
    for k, t in ((1, 2), (2, 2), (3, 2)):
        lo = OP.PolyBJAC(A, bp, k=k, t=t, low=True)(r)
        hi = OP.PolyBJAC(A, bp, k=k, t=t, low=False)(r)
        np.testing.assert_array_equal(lo, hi)
