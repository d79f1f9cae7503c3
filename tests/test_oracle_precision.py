"""Pins of the oracle's storage rounding against library conversions and a
brute-force nearest-value search (not against its own formula)."""
import numpy as np

from oracle import precision as P


def _edge_values(rng, n=20000):
    mags = np.ldexp(1.0, rng.integers(-160, 130, size=n)) * rng.uniform(1, 2, size=n)
    vals = np.concatenate([mags, -mags])
    # exact ties of the 16-bit and fp32 formats, subnormal ties, boundaries
    m = rng.integers(1, 2 ** 10, size=2000)
    ties16 = np.ldexp(2 * m + 1.0, rng.integers(-40, 5, size=2000) - 11)
    m32 = rng.integers(1, 2 ** 23, size=2000)
    ties32 = np.ldexp(2 * m32 + 1.0, rng.integers(-170, 100, size=2000) - 24)
    special = np.array([0.0, -0.0, 65504.0, 65519.99, 65520.0, 65536.0, 2.0 ** -24, 2.0 ** -25,
                        3 * 2.0 ** -26, 2.0 ** -14, 2.0 ** -149, 2.0 ** -150, 3 * 2.0 ** -151,
                        1e-300, 1e300, np.inf, -np.inf])
    return np.concatenate([vals, ties16, -ties16, ties32, -ties32, special])


def test_fp16_matches_numpy_cast():
    x = _edge_values(np.random.default_rng(0))
    got = P.round_to_format(x, P.FP16)
    ref = x.astype(np.float16).astype(np.float64)        # NumPy: direct RNE double->half
    np.testing.assert_array_equal(got, ref)
    assert np.array_equal(np.signbit(got), np.signbit(ref))


def test_fp32_matches_numpy_cast():
    x = _edge_values(np.random.default_rng(1))
    with np.errstate(over="ignore"):
        ref = x.astype(np.float32).astype(np.float64)
    np.testing.assert_array_equal(P.round_to_format(x, P.FP32), ref)


def _all_bf16():
    bits = (np.arange(2 ** 16, dtype=np.uint32) << 16)
    v = bits.view(np.float32).astype(np.float64)
    ok = np.isfinite(v) & (v >= 0)
    return np.sort(v[ok]), (np.arange(2 ** 16)[ok])


def test_bf16_matches_bruteforce_nearest():
    grid, _ = _all_bf16()                         # every non-negative finite bf16
    bits = (np.arange(2 ** 16, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)
    even = {}
    for i in range(2 ** 15):                      # non-negative patterns
        if np.isfinite(bits[i]):
            even[bits[i]] = (i % 2 == 0)
    rng = np.random.default_rng(2)
    x = np.abs(_edge_values(rng, 4000))
    x = x[np.isfinite(x) & (x < float.fromhex("0x1.fep127"))]
    got = P.round_to_format(x, P.BF16)
    j = np.clip(np.searchsorted(grid, x), 1, len(grid) - 1)
    lo, hi = grid[j - 1], grid[j]
    for xi, gi, l, h in zip(x, got, lo, hi):
        if xi == h:
            exp = h
        elif xi - l < h - xi:
            exp = l
        elif xi - l > h - xi:
            exp = h
        else:
            exp = l if even[l] else h
        assert gi == exp, (xi, gi, exp)


def test_block_scale_window():
    rng = np.random.default_rng(3)
    for v in np.concatenate([np.ldexp(1.0, np.arange(-60, 60)), rng.uniform(1e-30, 1e30, 500)]):
        for prec in (P.FP16, P.BF16):
            s = P.block_scale(v, prec)
            m, _ = np.frexp(s)
            assert m == 0.5                              # a power of two
            assert 2.0 ** 14 < v / s <= 2.0 ** 15
        assert P.block_scale(v, P.FP32) == 1.0


def test_store_block_error_bound():
    # |s Hhat - H| <= u |H| for entries in the normal range, <= s * half the
    # smallest subnormal spacing below it (the precision's own error bound)
    rng = np.random.default_rng(4)
    H = rng.standard_normal((32, 32)) * np.exp(rng.uniform(-20, 0, (32, 32)))
    for prec, u, tiny in ((P.FP16, 2.0 ** -11, 2.0 ** -25), (P.BF16, 2.0 ** -8, 2.0 ** -134),
                          (P.FP32, 2.0 ** -24, 2.0 ** -150)):
        Hh, s = P.store_block(H, prec)
        err = np.abs(s * Hh - H)
        assert np.all(err <= u * np.abs(H) + s * tiny)
