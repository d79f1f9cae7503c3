"""Band-truncated storage of the block inverses on the GPU against the oracle
(blocks.band_width / band_part / store_blocks_band; the low-precision map of
Sec. 3.2 stored as the diagonals |i - j| <= w of each block).

Widths: equal to the oracle's except where the dropped sum sits on the
threshold within the rounding of the two FP64 inverses. Stored values: the
oracle's rounding of its band, up to one ulp where the two FP64 inverses
straddle a rounding boundary (FP64 blocks: within the inverses' difference).
Application: within the dot-product bound gamma_{2w+1} of the accumulation
precision plus that ulp. PCG: iteration counts within 2 of the oracle's.
"""
import numpy as np
import pytest

from oracle import blocks as OB
from oracle import pcg as OP
from oracle import precision as OPr
from paper_2407_15973_amd import binding as mb
from paper_2407_15973_amd import gen

from gpu_helpers import dev, gamma, tensor, ulp

pytestmark = pytest.mark.gpu

ULP_REL = {OPr.FP64: 2.0 ** -52, OPr.FP32: 2.0 ** -23, OPr.BF16: 2.0 ** -7, OPr.FP16: 2.0 ** -10}


def _case(seed=3, shape=(12, 10, 9), sizes=None, b=32, lo=-2.0, hi=2.0):
    rng = np.random.default_rng(seed)
    A = gen.diffusion3d(gen.kappa_loguniform(shape, rng, lo, hi))
    bp = gen.random_blocks(A.n, rng, sizes) if sizes else gen.uniform_blocks(A.n, b)
    return A, bp, rng


def _tail(Hk, w):
    d = np.abs(np.subtract.outer(np.arange(Hk.shape[0]), np.arange(Hk.shape[0])))
    return float(np.sum(np.where(d > w, Hk * Hk, 0.0)))


def _width_agrees(Hk, wg, wo, u):
    """Equal widths, or a decision at the smaller one that sits on the
    threshold within the inverses' rounding."""
    if wg == wo:
        return True
    w = min(wg, wo)
    thr = u * u * float(np.sum(Hk * Hk))
    return abs(_tail(Hk, w) - thr) <= 1e-8 * thr


def _band_policy(**kw):
    return mb.Policy(storage=mb.STORE_BAND, **kw)


@pytest.mark.parametrize("prec", [OPr.FP64, OPr.FP32, OPr.BF16, OPr.FP16])
@pytest.mark.parametrize("b,sizes", [(32, None), (0, (16, 32, 48, 64)), (0, (5, 13, 40))])
def test_band_widths_and_values_match_oracle(prec, b, sizes):
    A, bp, _ = _case(b=b, sizes=sizes)
    nb = len(bp) - 1
    pol = _band_policy(mode=mb.FIXED, low=prec) if prec != OPr.FP64 else _band_policy(mode=mb.UNIFORM)
    M = mb.BlockJacobi(mb.DeviceCSR(A, dev()), bp, pol)
    H = OB.invert_blocks(A, bp)
    store = OB.store_blocks_band(H, np.full(nb, prec, np.uint8))
    wg = M.band_widths()
    u = OB.UNIT_ROUNDOFF[prec]
    equal = 0
    for k in range(nb):
        Hh, s_ref, _, wo = store[k]
        assert _width_agrees(H[k], int(wg[k]), wo, u), (k, wg[k], wo)
        got, s = M.block(k)
        assert s == s_ref
        if wg[k] != wo:
            continue
        equal += 1
        if prec == OPr.FP64:
            kap = np.linalg.cond(H[k], 1)
            np.testing.assert_allclose(got, Hh, rtol=0, atol=4 * H[k].shape[0] * kap * 2.0 ** -53 * np.abs(Hh).max())
        else:
            d = np.abs(got - Hh)
            assert np.all(d <= ulp(Hh, prec) * 1.0000001), (prec, k)
            assert np.count_nonzero(d) <= max(2, d.size // 50)
    assert equal >= nb - max(1, nb // 50)
    # stored bytes: w + 1 diagonals of the padded size per block
    info = M.info()
    pad = (np.diff(bp) + 15) // 16 * 16
    assert info["low_bytes"] == int(np.sum(pad * (wg.astype(np.int64) + 1))) * OPr.BYTES[prec]
    assert info["low_bytes"] < int(np.sum(pad * pad)) * OPr.BYTES[prec]


def _apply_bound(store, bp, r, tags, H):
    zb = OB.apply_abs(store, bp, r)
    w = np.array([e[3] for e in store])
    per_row_ulp = np.repeat([ULP_REL[int(t)] for t in tags], np.diff(bp))
    acc_u = np.repeat([2.0 ** -53 if t == OPr.FP64 else 2.0 ** -24 for t in tags], np.diff(bp))
    terms = np.repeat(2 * w + 1, np.diff(bp))
    kap = max(np.linalg.cond(h, 1) for h in H)
    bmax = int(np.max(np.diff(bp)))
    return (terms * acc_u / (1 - terms * acc_u) + per_row_ulp + 8 * bmax * kap * 2.0 ** -53) * zb


@pytest.mark.parametrize("sizes", [None, (16, 32, 48, 64), (7, 33, 64)])
def test_band_apply_mixed_map_within_bound(sizes):
    A, bp, rng = _case(seed=5, shape=(16, 12, 10), sizes=sizes)
    nb = len(bp) - 1
    tags = rng.choice([OPr.FP64, OPr.FP32, OPr.BF16, OPr.FP16], size=nb).astype(np.uint8)
    M = mb.BlockJacobi(mb.DeviceCSR(A, dev()), bp, _band_policy(mode=mb.EXPLICIT, explicit_tags=tags))
    H = OB.invert_blocks(A, bp)
    store = OB.store_blocks_band(H, tags)
    wg = M.band_widths()
    for k in range(nb):
        assert _width_agrees(H[k], int(wg[k]), store[k][3], OB.UNIT_ROUNDOFF[int(tags[k])])
    # compare against the oracle with the GPU's widths (a near-tie width
    # changes which entries are kept, not the bound)
    store = [(OPr.round_to_format(OB.band_part(Hk, int(w)) / s, int(t)), s, t, int(w))
             for Hk, (_, s, t, _), w in zip(H, store, wg)]
    for trial in range(2):
        r = rng.uniform(-1, 1, A.n) * np.exp(rng.uniform(-20, 0, A.n))
        z = M.apply(tensor(r)).cpu().numpy()
        ref = OB.apply(store, bp, r)
        assert np.all(np.abs(z - ref) <= _apply_bound(store, bp, r, tags, H) + 1e-300)


@pytest.mark.parametrize("prec", [OPr.FP64, OPr.FP32, OPr.FP16])
def test_band_apply_uniform_precision_within_bound(prec):
    A, bp, rng = _case(seed=8, shape=(20, 14, 12), b=48)
    nb = len(bp) - 1
    tags = np.full(nb, prec, np.uint8)
    pol = _band_policy(mode=mb.FIXED, low=prec) if prec != OPr.FP64 else _band_policy(mode=mb.UNIFORM)
    M = mb.BlockJacobi(mb.DeviceCSR(A, dev()), bp, pol)
    H = OB.invert_blocks(A, bp)
    wg = M.band_widths()
    store = [(OPr.round_to_format(OB.band_part(Hk, int(w)) / s, int(prec)), s, int(prec), int(w))
             for Hk, w, s in zip(H, wg, [OPr.block_scale(float(np.max(np.abs(h))), int(prec)) for h in H])]
    r = rng.uniform(-1, 1, A.n)
    z = M.apply(tensor(r)).cpu().numpy()
    ref = OB.apply(store, bp, r)
    assert np.all(np.abs(z - ref) <= _apply_bound(store, bp, r, tags, H) + 1e-300)


def test_band_rtol_override_and_diagonal_blocks():
    # a loose tolerance keeps few diagonals, equal to the oracle's widths
    A, bp, rng = _case(seed=9, shape=(10, 10, 10), b=32)
    H = OB.invert_blocks(A, bp)
    M = mb.BlockJacobi(mb.DeviceCSR(A, dev()), bp, _band_policy(mode=mb.FIXED, low=mb.FP32, band_rtol=0.3))
    wg = M.band_widths()
    for k, Hk in enumerate(H):
        assert _width_agrees(Hk, int(wg[k]), OB.band_width(Hk, 0.3), 0.3)
    assert wg.max() <= 3
    # a diagonal matrix: every block keeps one diagonal and z = round(1/a_ii) r
    n = 200
    d = np.exp(rng.uniform(-3, 3, n))
    D = gen._csr_from_coo(n, np.arange(n), np.arange(n), d)
    bpd = gen.uniform_blocks(n, 32)
    Md = mb.BlockJacobi(mb.DeviceCSR(D, dev()), bpd, _band_policy(mode=mb.UNIFORM))
    assert np.all(Md.band_widths() == 0)
    r = rng.uniform(-1, 1, n)
    z = Md.apply(tensor(r)).cpu().numpy()
    np.testing.assert_array_equal(z, (1.0 / d) * r)


@pytest.mark.parametrize("prec,slack", [(OPr.FP64, 1), (OPr.FP32, 2), (OPr.FP16, 2)])
def test_band_pcg_matches_oracle(prec, slack):
    A, bp, rng = _case(seed=11, shape=(24, 20, 16), b=32)
    nb = len(bp) - 1
    b = rng.uniform(-1, 1, A.n)
    Ad = mb.DeviceCSR(A, dev())
    pol = _band_policy(mode=mb.FIXED, low=prec) if prec != OPr.FP64 else _band_policy(mode=mb.UNIFORM)
    M = mb.BlockJacobi(Ad, bp, pol)
    res = mb.Solver(A.n, dev()).solve(Ad, M, tensor(b), tol=1e-10, maxit=3000)
    tags = np.full(nb, prec, np.uint8)
    ref = OP.solve_bjac(A, bp, b, M=OP.BJAC(A, bp, tags, band=True), tol=1e-10, maxit=3000)
    full = OP.solve_bjac(A, bp, b, tags, tol=1e-10, maxit=3000)
    print(f"band {OPr.NAMES[prec]}: gpu {res.iters} oracle {ref.iters} (full storage {full.iters})")
    assert res.status == mb.OK and ref.status == OP.CONVERGED
    assert abs(res.iters - ref.iters) <= slack
    assert OP.true_relres(A, res.x.cpu().numpy(), b) <= 2e-10


def test_band_temporal_and_rule():
    A, bp, rng = _case(seed=12, shape=(20, 16, 12), b=48)
    nb = len(bp) - 1
    b = rng.uniform(-1, 1, A.n)
    Ad = mb.DeviceCSR(A, dev())
    H = OB.invert_blocks(A, bp)
    # temporal hl: both maps banded, the FP64 map at u_64
    M = mb.BlockJacobi(Ad, bp, _band_policy(mode=mb.FIXED, low=mb.FP16, temporal=mb.TEMPORAL_HL, adp_tol=1e-4))
    w_hi = M.band_widths(1)
    for k, Hk in enumerate(H):
        assert _width_agrees(Hk, int(w_hi[k]), OB.band_width(Hk, 2.0 ** -53), 2.0 ** -53)
    info = M.info()
    assert info["high_bytes"] == int(np.sum(48 * (w_hi.astype(np.int64) + 1))) * 8
    res = mb.Solver(A.n, dev()).solve(Ad, M, tensor(b), tol=1e-10, maxit=3000)
    ref = OP.solve_bjac(A, bp, b, M=OP.BJAC(A, bp, np.full(nb, OPr.FP16, np.uint8), H=H, band=True), tol=1e-10,
                        maxit=3000, temporal=OP.TEMPORAL_HL, adp_tol=1e-4)
    assert res.status == mb.OK and abs(res.iters - ref.iters) <= 2
    # the rule picks the same tags with either storage
    Mr = mb.BlockJacobi(Ad, bp, _band_policy(mode=mb.RULE))
    Mf = mb.BlockJacobi(Ad, bp, mb.Policy(mode=mb.RULE))
    assert np.array_equal(Mr.tags(), Mf.tags())
    res_r = mb.Solver(A.n, dev()).solve(Ad, Mr, tensor(b), tol=1e-10, maxit=3000)
    assert res_r.status == mb.OK
    assert OP.true_relres(A, res_r.x.cpu().numpy(), b) <= 2e-10


def test_band_errors():
    A, bp, rng = _case(seed=13, shape=(8, 8, 8), b=32)
    Ad = mb.DeviceCSR(A, dev())
    for pol in (mb.Policy(storage=7), _band_policy(band_rtol=1.0), _band_policy(band_rtol=float("nan"))):
        with pytest.raises(mb.MpbjacError) as e:
            mb.BlockJacobi(Ad, bp, pol)
        assert e.value.code == mb.EINVAL
    M = mb.BlockJacobi(Ad, bp, _band_policy(mode=mb.FIXED, low=mb.FP16))
    with pytest.raises(mb.MpbjacError):
        M.band_widths(1)                       # no FP64 map without the temporal switch
    with pytest.raises(mb.MpbjacError):
        mb.BlockJacobi(Ad, bp, mb.Policy()).band_widths()
    # paper-mode handles have no stored blocks: the multi-column entry points refuse them
    P = mb.PaperBJAC(Ad, bp, k=1, t=1)
    with pytest.raises(mb.MpbjacError):
        P.apply_multi(tensor(np.zeros((A.n, 2))))


def test_band_full_width_equals_full_storage():
    # a vanishing tolerance keeps every diagonal (w = b - 1: eight rounds of
    # eight diagonals for 64-row blocks); the band application then multiplies
    # the symmetrised full inverse: within rounding of the full-storage result
    A, bp, rng = _case(seed=14, shape=(16, 16, 8), b=64)
    Ad = mb.DeviceCSR(A, dev())
    for prec in (OPr.FP32, OPr.FP64):
        pol = dict(mode=mb.FIXED, low=prec) if prec != OPr.FP64 else dict(mode=mb.UNIFORM)
        Mb = mb.BlockJacobi(Ad, bp, _band_policy(band_rtol=1e-300, **pol))
        Mf = mb.BlockJacobi(Ad, bp, mb.Policy(**pol))
        assert np.all(Mb.band_widths() == np.diff(bp) - 1)
        r = rng.uniform(-1, 1, A.n)
        zb = Mb.apply(tensor(r)).cpu().numpy()
        zf = Mf.apply(tensor(r)).cpu().numpy()
        H = OB.invert_blocks(A, bp)
        store = OB.store_blocks(H, np.full(len(H), prec, np.uint8))
        u = 2.0 ** -24 if prec == OPr.FP32 else 2.0 ** -53
        # both within the accumulation bound of the same products, plus the
        # asymmetry of the computed inverse (the band mirrors its upper triangle)
        kap = max(np.linalg.cond(h, 1) for h in H)
        bound = (2 * gamma(64, u) + ULP_REL[prec] + 16 * 64 * kap * 2.0 ** -53) * OB.apply_abs(store, bp, r)
        assert np.all(np.abs(zb - zf) <= bound + 1e-300)


def test_band_full_size_sampled_parity():
    # the 128^3 benchmark workload with FP16 band storage: sampled blocks
    # against the oracle (widths, stored values, application rows), and the
    # PCG iteration count of full storage (truncation at u_16 leaves it)
    p = gen.config2(seed=0)
    nb = len(p.block_ptr) - 1
    Ad = mb.DeviceCSR(p.A, dev())
    M = mb.BlockJacobi(Ad, p.block_ptr, _band_policy(mode=mb.FIXED, low=mb.FP16))
    rng = np.random.default_rng(15)
    ks = rng.choice(nb, size=48, replace=False)
    sub = np.concatenate([[0], np.cumsum(np.diff(p.block_ptr)[ks])]).astype(np.int32)
    rows = np.concatenate([np.arange(p.block_ptr[k], p.block_ptr[k + 1]) for k in ks])
    S = p.A.to_scipy()[rows][:, rows]
    Asub = gen.CSR(len(rows), S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data)
    H = OB.invert_blocks(Asub, sub)
    tags = np.full(len(ks), OPr.FP16, np.uint8)
    wg = M.band_widths()[ks]
    ref = OB.store_blocks_band(H, tags)
    for j in range(len(ks)):
        assert _width_agrees(H[j], int(wg[j]), ref[j][3], 2.0 ** -11)
    store = [(OPr.round_to_format(OB.band_part(Hk, int(w)) / s, OPr.FP16), s, OPr.FP16, int(w))
             for Hk, w, (_, s, _, _) in zip(H, wg, ref)]
    r = rng.uniform(-1, 1, p.A.n)
    z = M.apply(tensor(r)).cpu().numpy()
    zref = OB.apply(store, sub, r[rows])
    assert np.all(np.abs(z[rows] - zref) <= _apply_bound(store, sub, r[rows], tags, H) + 1e-300)
    for j, k in enumerate(ks[:8]):
        got, s = M.block(int(k))
        assert s == store[j][1] and np.all(np.abs(got - store[j][0]) <= ulp(store[j][0], OPr.FP16) * 1.0000001)
    S = mb.Solver(p.A.n, dev())
    res = S.solve(Ad, M, tensor(p.b), tol=1e-10, maxit=5000)
    Mf = mb.BlockJacobi(Ad, p.block_ptr, mb.Policy(mode=mb.FIXED, low=mb.FP16))
    res_f = S.solve(Ad, Mf, tensor(p.b), tol=1e-10, maxit=5000)
    print(f"128^3 FP16: band {res.iters} iterations, full {res_f.iters}")
    assert res.status == mb.OK and abs(res.iters - res_f.iters) <= 2
    assert OP.true_relres(p.A, res.x.cpu().numpy(), p.b) <= 2e-10


def _band_store(H, tags, wg):
    return [(OPr.round_to_format(OB.band_part(Hk, int(w)) / OPr.block_scale(float(np.max(np.abs(Hk))), int(t)), int(t)),
             OPr.block_scale(float(np.max(np.abs(Hk))), int(t)), int(t), int(w)) for Hk, t, w in zip(H, tags, wg)]


@pytest.mark.parametrize("sizes,m", [((16, 32, 48, 64), 5), ((7, 33, 64, 16), 8), ((32,), 1)])
def test_band_apply_multi_matches_oracle(sizes, m):
    # several columns at once (the batched application's element-by-element
    # band products): every column within the single-column bound
    A, bp, rng = _case(seed=16, shape=(11, 9, 13), sizes=sizes)
    nb = len(bp) - 1
    tags = rng.choice([OPr.FP64, OPr.FP32, OPr.BF16, OPr.FP16], size=nb).astype(np.uint8)
    M = mb.BlockJacobi(mb.DeviceCSR(A, dev()), bp, _band_policy(mode=mb.EXPLICIT, explicit_tags=tags))
    H = OB.invert_blocks(A, bp)
    store = _band_store(H, tags, M.band_widths())
    R = rng.uniform(-1, 1, (A.n, m)) * np.exp(rng.uniform(-20, 0, (A.n, m)))
    Z = M.apply_multi(tensor(R)).cpu().numpy()
    for c in range(m):
        ref = OB.apply(store, bp, R[:, c])
        assert np.all(np.abs(Z[:, c] - ref) <= _apply_bound(store, bp, R[:, c], tags, H) + 1e-300), c


def _sub_csr(A, r0, r1):
    a, b = int(A.row_ptr[r0]), int(A.row_ptr[r1])
    return gen.CSR(r1 - r0, (A.row_ptr[r0:r1 + 1] - a).astype(np.int32), (A.col_idx[a:b] - r0).astype(np.int32),
                   A.val[a:b].copy())


@pytest.mark.parametrize("prec", [OPr.FP16, OPr.FP64])
def test_band_batched_pcg_matches_oracle(prec):
    # batched systems with 1-8 right-hand sides and band storage: every column
    # against the oracle's band PCG on its system
    st = gen.stack_batch(gen.config4(3, nsys=5, edge=(5, 14), nrhs=(1, 8)))
    Ad = mb.DeviceCSR(st.A, dev())
    pol = _band_policy(mode=mb.FIXED, low=prec) if prec != OPr.FP64 else _band_policy(mode=mb.UNIFORM)
    M = mb.BlockJacobi(Ad, st.block_ptr, pol)
    bs = mb.BatchSolver(Ad, M, st.sys_row, st.sys_m)
    res = bs.solve(tensor(st.b), tol=1e-10, maxit=3000)
    assert res.status == mb.OK
    x = res.x.cpu().numpy()
    col = 0
    for s in range(len(st.sys_m)):
        r0, r1 = int(st.sys_row[s]), int(st.sys_row[s + 1])
        m = int(st.sys_m[s])
        k0, k1 = int(np.searchsorted(st.block_ptr, r0)), int(np.searchsorted(st.block_ptr, r1))
        bp = (st.block_ptr[k0:k1 + 1] - r0).astype(np.int32)
        sub = _sub_csr(st.A, r0, r1)
        Mo = OP.BJAC(sub, bp, np.full(k1 - k0, prec, np.uint8), band=True)
        Bs = st.b[st.system_slice(s)].reshape(r1 - r0, m)
        xs = x[st.system_slice(s)].reshape(r1 - r0, m)
        for c in range(m):
            ref = OP.solve_bjac(sub, bp, Bs[:, c], tol=1e-10, maxit=3000, M=Mo)
            assert ref.status == OP.CONVERGED and res.col_status[col] == mb.OK
            assert abs(int(res.col_iters[col]) - ref.iters) <= max(3, int(0.05 * ref.iters)), (s, c)
            assert OP.true_relres(sub, xs[:, c], Bs[:, c]) <= 2e-10
            col += 1
