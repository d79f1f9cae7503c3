"""Pins of the oracle's block extraction, FP64 inverse, features, precision
rule and application: library inverses, closed forms, exact special cases."""
import numpy as np
import pytest

from paper_2407_15973_amd import gen
from oracle import blocks as OB
from oracle import precision as P


def _rand_spd(rng, b, cond=1e4):
    Q, _ = np.linalg.qr(rng.standard_normal((b, b)))
    ev = np.exp(rng.uniform(0, np.log(cond), b))
    return (Q * ev) @ Q.T


@pytest.mark.parametrize("b", [1, 2, 5, 16, 33, 48, 64])
def test_inverse_matches_library(b):
    rng = np.random.default_rng(b)
    Ab = np.stack([_rand_spd(rng, b) for _ in range(4)])
    Ab = 0.5 * (Ab + np.transpose(Ab, (0, 2, 1)))
    L, ok = OB.cholesky(Ab)
    assert ok.all()
    np.testing.assert_allclose(L @ np.transpose(L, (0, 2, 1)), Ab, rtol=0, atol=1e-12 * np.abs(Ab).max())
    X = OB.inverse_from_cholesky(L)
    ref = np.linalg.inv(Ab)
    np.testing.assert_allclose(X, ref, rtol=0, atol=1e4 * 64 * 2e-16 * np.abs(ref).max())


def test_inverse_of_size_one_blocks_is_reciprocal():
    rng = np.random.default_rng(0)
    A = gen.diffusion3d(gen.kappa_loguniform((4, 4, 4), rng))
    H = OB.invert_blocks(A, gen.uniform_blocks(A.n, 1))
    d = A.to_scipy().diagonal()
    got = np.array([h[0, 0] for h in H])
    np.testing.assert_allclose(got, 1.0 / d, rtol=5e-16)   # sqrt, 1/L, /L: <= 4 roundings


def _cheb_u(k):
    u = [1.0, 4.0]
    for _ in range(k):
        u.append(4 * u[-1] - u[-2])
    return u


def test_poisson_line_block_closed_form():
    # config 1: the 64-row blocks of the 2D 5-point Laplacian are tridiag(-1,4,-1);
    # (T^-1)_ij = U_{i-1}(2) U_{m-j}(2) / U_m(2), i <= j (1-based), U = Chebyshev 2nd kind
    p = gen.config1(0)
    H = OB.invert_blocks(p.A, p.block_ptr)
    m = 64
    U = _cheb_u(m)
    T = np.empty((m, m))
    for i in range(1, m + 1):
        for j in range(i, m + 1):
            T[i - 1, j - 1] = T[j - 1, i - 1] = U[i - 1] * U[m - j] / U[m]
    for h in H:
        np.testing.assert_allclose(h, T, rtol=1e-13, atol=1e-300)


def test_exact_integer_inverse_family():
    rng = np.random.default_rng(5)
    for b in (16, 32, 48, 64):
        A = gen.spd_exact_inverse_blocks(3, b, rng)
        H = OB.invert_blocks(A, gen.uniform_blocks(A.n, b))
        i = np.arange(b)
        mag = b - np.maximum(i[:, None], i[None, :])
        for k, h in enumerate(H):
            assert np.array_equal(np.abs(h), mag.astype(float))
            Ab = A.to_scipy()[k * b:(k + 1) * b, k * b:(k + 1) * b].toarray()
            assert np.array_equal(h @ Ab, np.eye(b))


def test_not_spd_detected():
    A = gen.poisson2d(4, 4)
    A.val[A.row_ptr[5]:A.row_ptr[6]][A.col_idx[A.row_ptr[5]:A.row_ptr[6]] == 5] = -1.0
    with pytest.raises(OB.NotSPD) as e:
        OB.invert_blocks(A, gen.uniform_blocks(A.n, 4))
    assert e.value.blocks == [1]


def test_extract_matches_dense_submatrix_uneven():
    rng = np.random.default_rng(6)
    A = gen.diffusion3d(gen.kappa_loguniform((5, 6, 7), rng))
    bp = gen.random_blocks(A.n, rng)
    D = A.to_scipy().toarray()
    for b, (ids, dense) in OB.extract_blocks(A, bp).items():
        for j, k in enumerate(ids):
            s, e = bp[k], bp[k + 1]
            assert np.array_equal(dense[j], D[s:e, s:e])


def test_features_hand_values_1d_poisson():
    # tridiag(-1, 2, -1), n = 8, blocks of 4: rows 0 and 7 strictly dominant (2 vs 1)
    n = 8
    from paper_2407_15973_amd.gen import _csr_from_coo
    i = np.arange(n)
    A = _csr_from_coo(n, np.concatenate([i, i[1:], i[:-1]]), np.concatenate([i, i[:-1], i[1:]]),
                      np.concatenate([np.full(n, 2.0), -np.ones(n - 1), -np.ones(n - 1)]))
    bp = gen.uniform_blocks(n, 4)
    H = OB.invert_blocks(A, bp)
    F, raw = OB.block_features(A, bp, H)
    assert F[0, 0] == 4 / 64
    assert F[0, 1] == 0.0                        # min full-row dominance 2/2 = 1
    np.testing.assert_allclose(F[0, 2], np.log10((2 + 1 + 1 + 1) / 4))
    np.testing.assert_allclose(F[0, 3], 0.0)     # rows 1, 2 in-block: 2 / 2
    np.testing.assert_allclose(F[0, 4], np.sqrt(6) / np.sqrt(16))
    np.testing.assert_allclose(F[0, 5], 1 / np.sqrt(16))     # one coupling to block 1
    assert F[0, 6] == 0.0 and F[0, 7] == 0.0     # tau = 1 everywhere
    assert F[0, 8] == np.log10(2.0)
    assert F[0, 9] == 0.0 and F[0, 10] == 2.0    # Gershgorin [0, 4] over max diag 2
    assert F[0, 11] == 16.0                      # lower bound 0 -> capped estimate
    assert F[0, 12] == 0.0
    # A_ii = tridiag(-1,2,-1) of size 4: ||A||_1 = 4, ||A^-1||_1 = max col sum of
    # (1/5)[[4,3,2,1],[3,6,4,2],[2,4,6,3],[1,2,3,4]] = 15/5 = 3
    np.testing.assert_allclose(raw["kappa1"][0], 12.0, rtol=1e-14)
    np.testing.assert_allclose(F[0, 14], np.log10(6 / 4))       # diag of A_ii^-1: 4,6,6,4 /5
    assert F[0, 15] == 0.0


def test_features_multiscale_anisotropy():
    for s in (1.0, 10.0, 1000.0):
        A = gen.diffusion3d(gen.kappa_const(6), aniso=(1, s, s))
        bp = gen.uniform_blocks(A.n, 6)
        F, _ = OB.block_features(A, bp, OB.invert_blocks(A, bp))
        np.testing.assert_allclose(F[:, 6], np.log10(s), atol=1e-15)   # eq. 4-5: tau = s


def test_rule_thresholds():
    raw = {"kappa1": np.array([10.0, 20.48, 20.49, 1e5, 1.6e5, 1.7e5, 10.0]),
           "min_dom": np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 0.5])}
    tags = OB.select_rule(raw, theta=1e-2, d16=1.0)
    # kappa * 2^-11 <= 1e-2  <=> kappa <= 20.48 ; kappa * 2^-24 <= 1e-2 <=> kappa <= 167772.16
    assert tags.tolist() == [P.FP16, P.FP16, P.FP32, P.FP32, P.FP32, P.FP64, P.FP32]


def test_apply_fp64_equals_dense_inverse_and_low_bound():
    rng = np.random.default_rng(7)
    A = gen.diffusion3d(gen.kappa_loguniform((6, 6, 6), rng))
    bp = gen.random_blocks(A.n, rng)
    H = OB.invert_blocks(A, bp)
    r = rng.uniform(-1, 1, A.n)
    z64 = OB.apply(OB.store_blocks(H, np.zeros(len(H), np.uint8)), bp, r)
    Dinv = np.zeros((A.n, A.n))
    for k, h in enumerate(H):
        Dinv[bp[k]:bp[k + 1], bp[k]:bp[k + 1]] = h
    np.testing.assert_allclose(z64, Dinv @ r, rtol=0, atol=1e-13 * np.abs(Dinv).sum(1).max())
    # the block solves invert the diagonal blocks
    D = A.to_scipy().toarray()
    for k in range(len(H)):
        s, e = bp[k], bp[k + 1]
        np.testing.assert_allclose(D[s:e, s:e] @ z64[s:e], r[s:e], atol=1e-11)
    for prec, u in ((P.FP32, 2.0 ** -24), (P.FP16, 2.0 ** -11), (P.BF16, 2.0 ** -8)):
        tags = np.full(len(H), prec, np.uint8)
        z = OB.apply(OB.store_blocks(H, tags), bp, r)
        bound = (2 * u + u * u) * (np.abs(Dinv) @ np.abs(r)) + 1e-300
        assert np.all(np.abs(z - z64) <= bound * 1.0001 + 2.0 ** -38 * np.abs(Dinv).max() * 64)


# ---------------------------------------------------- band-truncated storage
def _geometric_tail(n, rho, a):
    """sum_{d=a}^{n-1} 2 (n - d) rho^(2d) in closed form: with x = rho^2,
    k = n - d, y = 1/x and m = n - a, it is 2 x^n sum_{k=1}^{m} k y^k and
    sum_{k=1}^{m} k y^k = y (1 - (m+1) y^m + m y^(m+1)) / (1 - y)^2."""
    if a >= n:
        return 0.0
    x = rho * rho
    y = 1.0 / x
    m = n - a
    return 2.0 * x ** n * y * (1.0 - (m + 1) * y ** m + m * y ** (m + 1)) / (1.0 - y) ** 2


@pytest.mark.parametrize("n,rho,u", [(32, 0.3, 2.0 ** -11), (48, 0.5, 2.0 ** -24), (64, 0.17, 2.0 ** -8),
                                     (16, 0.9, 2.0 ** -11)])
def test_band_width_geometric_closed_form(n, rho, u):
    # H_ij = rho^|i-j|: the energy of diagonal d is 2 (n - d) rho^(2d) (d >= 1)
    # and n for d = 0; the width is the first w whose closed-form tail beyond w
    # is within u^2 of the closed-form total
    idx = np.arange(n)
    H = rho ** np.abs(np.subtract.outer(idx, idx))
    total = n + _geometric_tail(n, rho, 1)
    want = next(w for w in range(n) if _geometric_tail(n, rho, w + 1) <= u * u * total * (1 + 1e-12))
    # the closed form and the explicit sum agree to rounding: skip near-ties
    margin = abs(_geometric_tail(n, rho, want + 1) - u * u * total) / (u * u * total)
    assert margin > 1e-9
    assert OB.band_width(H, u) == want


def test_band_width_minimal_and_bounded_brute_force():
    rng = np.random.default_rng(7)
    A = gen.diffusion3d(gen.kappa_loguniform((8, 6, 5), rng))
    H = OB.invert_blocks(A, gen.uniform_blocks(A.n, 16))
    for Hk in H:
        for u in (2.0 ** -11, 2.0 ** -24, 1e-3):
            w = OB.band_width(Hk, u)
            b = Hk.shape[0]
            dropped = [Hk[i, j] ** 2 for i in range(b) for j in range(b) if abs(i - j) > w]
            assert np.sqrt(sum(dropped)) <= u * np.linalg.norm(Hk, "fro") * (1 + 1e-12)
            if w > 0:
                more = [Hk[i, j] ** 2 for i in range(b) for j in range(b) if abs(i - j) > w - 1]
                assert np.sqrt(sum(more)) > u * np.linalg.norm(Hk, "fro")


def test_band_exact_zero_structure():
    # a diagonal matrix keeps one diagonal; a tridiagonal one at most three,
    # however small the tolerance; the band part mirrors the upper triangle
    rng = np.random.default_rng(8)
    D = np.diag(rng.uniform(1, 2, 20))
    assert OB.band_width(D, 1e-300) == 0
    T = np.diag(rng.uniform(3, 4, 20)) + np.diag(rng.uniform(-1, 0, 19), 1)
    T = T + np.triu(T, 1).T
    assert OB.band_width(T, 1e-300) == 1
    M = rng.standard_normal((10, 10))
    Bm = OB.band_part(M, 2)
    assert np.array_equal(Bm, Bm.T)
    for i in range(10):
        for j in range(10):
            want = M[min(i, j), max(i, j)] if abs(i - j) <= 2 else 0.0
            assert Bm[i, j] == want


def test_band_store_scale_and_bytes():
    rng = np.random.default_rng(9)
    A = gen.diffusion3d(gen.kappa_loguniform((8, 8, 8), rng))
    bp = gen.uniform_blocks(A.n, 32)
    H = OB.invert_blocks(A, bp)
    tags = np.array([P.FP16, P.FP32, P.BF16, P.FP64] * (len(H) // 4), dtype=np.uint8)
    st = OB.store_blocks_band(H, tags)
    for Hk, t, (Hh, s, tt, w) in zip(H, tags, st):
        assert tt == t and s == P.block_scale(float(np.max(np.abs(Hk))), int(t))
        # in-band entries are the format's rounding of the (mirrored) inverse
        Bk = OB.band_part(Hk, w)
        assert np.array_equal(Hh, P.round_to_format(Bk / s, int(t)))
        assert w == OB.band_width(Hk, OB.UNIT_ROUNDOFF[int(t)])
    # w + 1 diagonals of 32 entries per block
    assert OB.band_bytes(st, bp) == sum(32 * (e[3] + 1) * P.BYTES[e[2]] for e in st)


def test_band_with_vanishing_tolerance_is_full_symmetrised_storage():
    rng = np.random.default_rng(10)
    A = gen.diffusion3d(gen.kappa_loguniform((6, 5, 4), rng))
    bp = gen.uniform_blocks(A.n, 24)
    H = OB.invert_blocks(A, bp)
    tags = np.full(len(H), P.FP16, dtype=np.uint8)
    st = OB.store_blocks_band(H, tags, rtol=1e-300)
    for Hk, (Hh, s, t, w) in zip(H, st):
        assert w == Hk.shape[0] - 1
        Sym = np.triu(Hk) + np.triu(Hk, 1).T
        assert np.array_equal(Hh, P.round_to_format(Sym / s, P.FP16))
