"""Batched multi-right-hand-side path against the FP64 oracle.

* bjac_apply_multi: every column of Z = M^-1 R (matrix-core block products)
  against the oracle's per-column application, within the FP32 (FP64)
  accumulation bound gamma_b(u) |Hhat| |r_in| of Algorithm 3.1;
* pcg_solve_batched: every (system, column) pair is an independent CG
  (Sec. 3.2, stopping test of Sec. 4.2); iteration counts against the oracle's
  PCG on that system and column, the FP64-recomputed true residual, and x;
* chunking and the autotuner change nothing but speed; bad partitions are
  rejected.
"""
import numpy as np
import pytest

from oracle import blocks as OB
from oracle import pcg as OP
from oracle import precision as OPr
from paper_2407_15973_amd import binding as mb
from paper_2407_15973_amd import gen

from gpu_helpers import dev, gamma, oracle_setup, tensor

pytestmark = pytest.mark.gpu

U = {OPr.FP64: 2.0 ** -53, OPr.FP32: 2.0 ** -24, OPr.BF16: 2.0 ** -24, OPr.FP16: 2.0 ** -24}


def _cols(rng, n, m):
    return rng.uniform(-1, 1, (n, m)) * np.exp(rng.uniform(-20, 0, (n, m)))


@pytest.mark.parametrize("prec", [OPr.FP64, OPr.FP32, OPr.BF16, OPr.FP16])
@pytest.mark.parametrize("m", [1, 3, 8])
def test_apply_multi_exact_family(prec, m):
    # integer inverses: the stored values are exact in every format, so the
    # only difference is the accumulation order of the matrix-core products
    rng = np.random.default_rng(20 + m)
    A = gen.spd_exact_inverse_blocks(30, 48, rng)
    bp = gen.uniform_blocks(A.n, 48)
    tags = np.full(len(bp) - 1, prec, np.uint8)
    H, store = oracle_setup(A, bp, tags)
    M = mb.BlockJacobi(mb.DeviceCSR(A, dev()), bp, mb.Policy(mode=mb.FIXED, low=prec))
    R = _cols(rng, A.n, m)
    Z = M.apply_multi(tensor(R)).cpu().numpy()
    for c in range(m):
        ref = OB.apply(store, bp, R[:, c])
        bound = gamma(48, U[prec]) * OB.apply_abs(store, bp, R[:, c])
        assert np.all(np.abs(Z[:, c] - ref) <= bound + 1e-300), c


@pytest.mark.parametrize("sizes,m", [((16, 32, 48, 64), 5), ((7, 33, 64, 16), 8), ((64,), 2)])
def test_apply_multi_mixed_map_ragged(sizes, m):
    rng = np.random.default_rng(31)
    kap = gen.kappa_loguniform((9, 11, 13), rng)
    A = gen.diffusion3d(kap)
    bp = gen.random_blocks(A.n, rng, sizes)
    nb = len(bp) - 1
    tags = rng.choice([OPr.FP64, OPr.FP32, OPr.BF16, OPr.FP16], size=nb).astype(np.uint8)
    M = mb.BlockJacobi(mb.DeviceCSR(A, dev()), bp, mb.Policy(mode=mb.EXPLICIT, explicit_tags=tags))
    H, store = oracle_setup(A, bp, tags)
    R = _cols(rng, A.n, m)
    Z = M.apply_multi(tensor(R)).cpu().numpy()
    # one storage ulp where the two FP64 inverses straddle a rounding boundary,
    # the inverse's own error, and the accumulation bound
    ulp_rel = np.array([{0: 2.0 ** -52, 1: 2.0 ** -23, 2: 2.0 ** -7, 3: 2.0 ** -10}[t] for t in tags])
    per_row = np.repeat(ulp_rel, np.diff(bp))
    bmax = int(np.max(np.diff(bp)))
    kap1 = max(np.linalg.cond(h, 1) for h in H)
    for c in range(m):
        ref = OB.apply(store, bp, R[:, c])
        bound = (gamma(bmax, 2.0 ** -24) + per_row + 8 * bmax * kap1 * 2.0 ** -53) * OB.apply_abs(store, bp, R[:, c])
        assert np.all(np.abs(Z[:, c] - ref) <= bound + 1e-300), c


def test_apply_multi_single_column_agrees_with_apply():
    # the vector apply and the matrix-core apply take the same stored bytes;
    # both are within the accumulation bound of the oracle, hence of each other
    rng = np.random.default_rng(4)
    A = gen.diffusion3d(gen.kappa_loguniform((8, 8, 16), rng))
    bp = gen.uniform_blocks(A.n, 32)
    M = mb.BlockJacobi(mb.DeviceCSR(A, dev()), bp, mb.Policy(mode=mb.FIXED, low=mb.FP16))
    H, store = oracle_setup(A, bp, np.full(len(bp) - 1, OPr.FP16, np.uint8))
    r = rng.uniform(-1, 1, A.n)
    z1 = M.apply(tensor(r)).cpu().numpy()
    zm = M.apply_multi(tensor(r[:, None].copy())).cpu().numpy()[:, 0]
    ab = OB.apply_abs(store, bp, r)
    assert np.all(np.abs(z1 - zm) <= 2 * (gamma(32, 2.0 ** -24) + 2.0 ** -10) * ab)


# ---------------------------------------------------------------- batched PCG
def _batch(seed, nsys, edge, nrhs):
    return gen.stack_batch(gen.config4(seed, nsys=nsys, edge=edge, nrhs=nrhs))


def _oracle_cols(st, tags_all, tol, maxit):
    """Oracle PCG for every system and column: (iters, status, x) lists."""
    out = []
    for s in range(len(st.sys_m)):
        r0, r1 = int(st.sys_row[s]), int(st.sys_row[s + 1])
        m = int(st.sys_m[s])
        k0 = int(np.searchsorted(st.block_ptr, r0))
        k1 = int(np.searchsorted(st.block_ptr, r1))
        bp = (st.block_ptr[k0:k1 + 1] - r0).astype(np.int32)
        sub = _sub_csr(st.A, r0, r1)
        Mo = OP.BJAC(sub, bp, tags_all[k0:k1])
        Bs = st.b[st.system_slice(s)].reshape(r1 - r0, m)
        for c in range(m):
            res = OP.solve_bjac(sub, bp, Bs[:, c], tol=tol, maxit=maxit, M=Mo)
            out.append((res.iters, res.status, res.x, sub, Bs[:, c]))
    return out


def _sub_csr(A, r0, r1):
    a, b = int(A.row_ptr[r0]), int(A.row_ptr[r1])
    return gen.CSR(r1 - r0, (A.row_ptr[r0:r1 + 1] - a).astype(np.int32), (A.col_idx[a:b] - r0).astype(np.int32),
                   A.val[a:b].copy())


def _run(st, policy, tol=1e-10, maxit=3000, cfg=(0, 0), chunk=16):
    Ad = mb.DeviceCSR(st.A, dev())
    M = mb.BlockJacobi(Ad, st.block_ptr, policy)
    bs = mb.BatchSolver(Ad, M, st.sys_row, st.sys_m)
    res = bs.solve(tensor(st.b), tol=tol, maxit=maxit, cfg=cfg, chunk=chunk)
    return M, bs, res


@pytest.mark.parametrize("prec,slack", [(OPr.FP64, 2), (OPr.FP32, 2), (OPr.FP16, 3)])
def test_batched_pcg_matches_oracle(prec, slack):
    st = _batch(3, nsys=7, edge=(5, 14), nrhs=(1, 8))
    pol = mb.Policy(mode=mb.UNIFORM) if prec == OPr.FP64 else mb.Policy(mode=mb.FIXED, low=prec)
    M, bs, res = _run(st, pol)
    assert res.status == mb.OK
    tags = M.tags()
    assert np.all(tags == prec)
    ref = _oracle_cols(st, tags, 1e-10, 3000)
    x = res.x.cpu().numpy()
    col = 0
    for s in range(len(st.sys_m)):
        m = int(st.sys_m[s])
        xs = x[st.system_slice(s)].reshape(-1, m)
        for c in range(m):
            it, status, xo, sub, bcol = ref[col]
            assert status == OP.CONVERGED
            assert res.col_status[col] == mb.OK
            assert abs(int(res.col_iters[col]) - it) <= max(slack, int(0.05 * it)), (s, c, res.col_iters[col], it)
            assert res.col_relres[col] <= 1e-10
            assert OP.true_relres(sub, xs[:, c], bcol) <= 2e-10
            col += 1
    assert res.iters == int(res.col_iters.max())


def test_batched_rule_map_and_uneven_chunks():
    st = _batch(5, nsys=5, edge=(6, 12), nrhs=(2, 6))
    M, bs, res = _run(st, mb.Policy(mode=mb.RULE), cfg=(1, 2, 1, 64))
    assert res.status == mb.OK
    ref = _oracle_cols(st, M.tags(), 1e-10, 3000)
    for col, (it, status, xo, sub, bcol) in enumerate(ref):
        assert abs(int(res.col_iters[col]) - it) <= max(3, int(0.05 * it))
    # a different apply chunking reorders only the per-column dot reductions
    res2 = bs.solve(tensor(st.b), tol=1e-10, maxit=3000, cfg=(8, 32, 2))
    assert res2.status == mb.OK
    assert np.all(np.abs(res2.col_iters - res.col_iters) <= 1)


def test_batched_spmv_launch_shape_does_not_change_results():
    # the matrix-vector chunks and their partial sums are fixed by the batch;
    # the grab size and the grid only change which wave computes a chunk, so
    # the iterates are bit for bit the same
    st = _batch(12, nsys=7, edge=(6, 14), nrhs=(1, 8))
    M, bs, res = _run(st, mb.Policy(mode=mb.FIXED, low=mb.FP16), cfg=(1, 32, 32, 512))
    assert res.status == mb.OK
    x1 = res.x.cpu().numpy().copy()
    for cfg in ((4, 32, 2, 512), (64, 32, 1, 512)):
        r2 = bs.solve(tensor(st.b), tol=1e-10, maxit=3000, cfg=cfg)
        assert np.array_equal(r2.col_iters, res.col_iters) and np.array_equal(r2.col_relres, res.col_relres)
        assert np.array_equal(r2.x.cpu().numpy(), x1)


def test_batched_zero_column_and_single_system():
    rng = np.random.default_rng(9)
    A = gen.diffusion3d(gen.kappa_loguniform((6, 7, 9), rng))
    bp = gen.random_blocks(A.n, rng)
    B = rng.uniform(-1, 1, (A.n, 4))
    B[:, 2] = 0.0
    st = gen.stack_batch([gen.BatchSystem(A, bp, B)])
    M, bs, res = _run(st, mb.Policy(mode=mb.FIXED, low=mb.FP32))
    assert res.status == mb.OK
    assert res.col_iters[2] == 0 and res.col_relres[2] == 0.0
    x = res.x.cpu().numpy().reshape(A.n, 4)
    assert np.all(x[:, 2] == 0.0)
    for c in (0, 1, 3):
        assert OP.true_relres(A, x[:, c], B[:, c]) <= 2e-10


def test_batched_maxit_reports_not_converged():
    st = _batch(6, nsys=3, edge=(8, 12), nrhs=(1, 3))
    M, bs, res = _run(st, mb.Policy(mode=mb.FIXED, low=mb.FP16), maxit=5, chunk=4)
    assert res.status == mb.NOT_CONVERGED
    assert np.all(res.col_iters == 5)
    assert np.all(res.col_status == mb.NOT_CONVERGED)


def test_batched_rejects_bad_partitions():
    st = _batch(7, nsys=3, edge=(5, 8), nrhs=(1, 2))
    Ad = mb.DeviceCSR(st.A, dev())
    # 16-row blocks placed so that one straddles the first system boundary
    r = int(st.sys_row[1])
    start = 8 if r % 16 == 0 else 0
    bp = np.unique(np.concatenate([[0], np.arange(start, st.A.n, 16), [st.A.n]])).astype(np.int32)
    assert r not in bp
    M = mb.BlockJacobi(Ad, bp, mb.Policy(mode=mb.FIXED, low=mb.FP32))
    bs = mb.BatchSolver(Ad, M, st.sys_row, st.sys_m)
    with pytest.raises(mb.MpbjacError):
        bs.solve(tensor(st.b))
    M2 = mb.BlockJacobi(Ad, st.block_ptr, mb.Policy(mode=mb.FIXED, low=mb.FP32))
    with pytest.raises(mb.MpbjacError):
        mb.BatchSolver(Ad, M2, st.sys_row, np.full(3, 9, np.int32)).solve(tensor(st.b))
    with pytest.raises(mb.MpbjacError):
        mb.BatchSolver(Ad, M2, st.sys_row[:-1], st.sys_m[:-1]).solve(tensor(st.b))


def test_autotuner_picks_a_candidate_and_it_solves():
    st = _batch(8, nsys=9, edge=(8, 16), nrhs=(1, 8))
    Ad = mb.DeviceCSR(st.A, dev())
    M = mb.BlockJacobi(Ad, st.block_ptr, mb.Policy(mode=mb.FIXED, low=mb.FP16))
    bs = mb.BatchSolver(Ad, M, st.sys_row, st.sys_m)
    cands = [(1, 2, 1), (4, 4, 2), (16, 16, 0)]
    best, ms = bs.tune(tensor(st.b), cands, iters=4)
    assert 0 <= best < len(cands)
    assert np.all(ms > 0) and ms[best] == ms.min()
    res = bs.solve(tensor(st.b), cfg=cands[best])
    assert res.status == mb.OK
    ref = _oracle_cols(st, M.tags(), 1e-10, 3000)
    for col, (it, *_r) in enumerate(ref):
        assert abs(int(res.col_iters[col]) - it) <= max(3, int(0.05 * it))


def test_autotune_cache_roundtrip(tmp_path):
    from paper_2407_15973_amd import autotune
    st = _batch(10, nsys=4, edge=(8, 12), nrhs=(1, 4))
    Ad = mb.DeviceCSR(st.A, dev())
    M = mb.BlockJacobi(Ad, st.block_ptr, mb.Policy(mode=mb.FIXED, low=mb.FP16))
    bs = mb.BatchSolver(Ad, M, st.sys_row, st.sys_m)
    path = str(tmp_path / "tune.json")
    cands = [(1, 2, 1, 256), (8, 4, 2, 4096)]
    cfg1, e1 = autotune.tuned_cfg(bs, tensor(st.b), candidates=cands, iters=3, cache_path=path)
    cfg2, e2 = autotune.tuned_cfg(bs, tensor(st.b), candidates=cands, iters=3, cache_path=path)
    assert cfg1 == cfg2 and cfg1 in cands and e1 == e2
    assert bs.solve(tensor(st.b), cfg=cfg1).status == mb.OK


def test_profile_mode_runs_the_same_iterations():
    st = _batch(11, nsys=4, edge=(8, 14), nrhs=(1, 8))
    M, bs, res = _run(st, mb.Policy(mode=mb.FIXED, low=mb.FP16))
    rp = bs.solve(tensor(st.b), tol=1e-10, maxit=3000, profile=True)
    # same kernels in the same order: bit-identical iterates
    assert np.array_equal(rp.col_iters, res.col_iters)
    assert np.array_equal(rp.x.cpu().numpy(), res.x.cpu().numpy())
    n_it = rp.kernel_ms["spmv"][1]
    assert n_it == res.iters and rp.kernel_ms["apply"][1] == n_it
    assert rp.kernel_ms["spmv"][0] > 0 and rp.kernel_ms["apply"][0] > 0


def test_full_size_batched_workload_sampled():
    # the 256-system batch the benchmark times (69 M rows, 1,114 columns), FP16
    # inverses: the multi-column products of sampled blocks against the oracle,
    # every column converged, and the FP64 true residual of sampled systems
    st = gen.stack_batch(gen.config4(seed=0))
    Ad = mb.DeviceCSR(st.A, dev())
    M = mb.BlockJacobi(Ad, st.block_ptr, mb.Policy(mode=mb.FIXED, low=mb.FP16))
    nb = len(st.block_ptr) - 1
    rng = np.random.default_rng(12)
    # multi-column application on the whole batch, 8 columns, sampled blocks
    R = rng.uniform(-1, 1, (st.A.n, 8))
    Z = M.apply_multi(tensor(R)).cpu().numpy()
    ks = rng.choice(nb, size=32, replace=False)
    sub = np.concatenate([[0], np.cumsum(np.diff(st.block_ptr)[ks])]).astype(np.int32)
    rows = np.concatenate([np.arange(st.block_ptr[k], st.block_ptr[k + 1]) for k in ks])
    S = st.A.to_scipy()[rows][:, rows]
    Asub = gen.CSR(len(rows), S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data)
    H = OB.invert_blocks(Asub, sub)
    store = OB.store_blocks(H, np.full(len(ks), OPr.FP16, np.uint8))
    bmax = int(np.max(np.diff(sub)))
    for c in range(8):
        ref = OB.apply(store, sub, R[rows, c])
        bound = (gamma(bmax, 2.0 ** -24) + 2.0 ** -10) * OB.apply_abs(store, sub, R[rows, c])
        assert np.all(np.abs(Z[rows, c] - ref) <= bound), c
    del Z, R
    bs = mb.BatchSolver(Ad, M, st.sys_row, st.sys_m)
    res = bs.solve(tensor(st.b), tol=1e-10, maxit=5000)
    assert res.status == mb.OK and np.all(res.col_status == mb.OK) and np.all(res.col_relres <= 1e-10)
    x = res.x.cpu().numpy()
    for s in rng.choice(len(st.sys_m), size=6, replace=False):
        r0, r1 = int(st.sys_row[s]), int(st.sys_row[s + 1])
        m = int(st.sys_m[s])
        A_s = _sub_csr(st.A, r0, r1)
        X = x[st.system_slice(s)].reshape(r1 - r0, m)
        Bm = st.b[st.system_slice(s)].reshape(r1 - r0, m)
        for c in range(m):
            assert OP.true_relres(A_s, X[:, c], Bm[:, c]) <= 2e-10, (s, c)


def test_batched_tiny_and_ragged_systems():
    # systems of 1, 2, 5, 17 and 70 rows, 1 and 8 columns, one block per
    # system where it fits (blocks never cross systems)
    rng = np.random.default_rng(13)
    systems = []
    for n, m in ((1, 1), (2, 8), (5, 3), (17, 8), (70, 1)):
        A = gen.poisson2d(n, 1) if n > 1 else gen._csr_from_coo(1, np.array([0]), np.array([0]), np.array([3.0]))
        bp = gen.uniform_blocks(n, 64) if n > 64 else np.array([0, n], np.int32)
        systems.append(gen.BatchSystem(A, bp, rng.uniform(-1, 1, (n, m))))
    st = gen.stack_batch(systems)
    M, bs, res = _run(st, mb.Policy())
    assert res.status == mb.OK
    x = res.x.cpu().numpy()
    col = 0
    for s, bsys in enumerate(systems):
        X = x[st.system_slice(s)].reshape(bsys.A.n, -1)
        for c in range(bsys.B.shape[1]):
            assert OP.true_relres(bsys.A, X[:, c], bsys.B[:, c]) <= 2e-10
            # one block per system of <= 64 rows is an exact solve: one iteration
            if bsys.A.n <= 64:
                assert res.col_iters[col] == 1
            col += 1


def test_batched_far_couplings_keep_32_bit_indices():
    # a 33000 x 2 grid couples rows 33000 apart, beyond the 16-bit row-relative
    # column copy: the products fall back to the 32-bit indices
    A = gen.poisson2d(33000, 2)
    rng = np.random.default_rng(31)
    B = rng.uniform(-1, 1, (A.n, 2))
    bp = gen.uniform_blocks(A.n, 32)
    st = gen.stack_batch([gen.BatchSystem(A, bp, B)])
    M, bs, res = _run(st, mb.Policy(mode=mb.FIXED, low=mb.FP32), maxit=200)
    assert res.status == mb.OK
    ref = _oracle_cols(st, M.tags(), 1e-10, 200)
    x = res.x.cpu().numpy().reshape(A.n, 2)
    for c, (it, status, xo, sub, bcol) in enumerate(ref):
        assert status == OP.CONVERGED
        assert abs(int(res.col_iters[c]) - it) <= max(2, int(0.05 * it))
        assert OP.true_relres(A, x[:, c], B[:, c]) <= 2e-10
