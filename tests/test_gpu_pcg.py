"""GPU block-Jacobi PCG against the CPU oracle: iteration counts (FP64 within 2
iterations; reduced maps report their delay), relative-residual histories,
the adaptive switch, degenerate cases, error paths, determinism, and the
full-size 128^3 workload on sampled outputs."""
import math

import numpy as np
import pytest

from oracle import blocks as OB
from oracle import pcg as OP
from oracle import precision as OPr
from paper_2407_15973_amd import binding as mb
from paper_2407_15973_amd import gen

from gpu_helpers import dev, gamma, tensor

pytestmark = pytest.mark.gpu


def _gpu_solve(A, bp, b, policy, tol, maxit, chunk=16, history=True, raise_on_error=True):
    Ad = mb.DeviceCSR(A, dev())
    M = mb.BlockJacobi(Ad, bp, policy)
    S = mb.Solver(A.n, dev())
    r = S.solve(Ad, M, tensor(b), tol=tol, maxit=maxit, chunk=chunk, history=history,
                raise_on_error=raise_on_error)
    return r, M


def _tags(prec, nb):
    return np.full(nb, prec, np.uint8)


def test_config1_fp64_matches_oracle():
    p = gen.config1(0)
    res, _ = _gpu_solve(p.A, p.block_ptr, p.b, mb.Policy(), p.tol, p.maxit)
    ref = OP.solve_bjac(p.A, p.block_ptr, p.b, tol=p.tol, maxit=p.maxit)
    assert res.status == mb.OK and ref.status == OP.CONVERGED
    assert abs(res.iters - ref.iters) <= 2
    m = min(res.iters, ref.iters) - 1
    np.testing.assert_allclose(res.relres_hist[:m], ref.history[:m], rtol=1e-6)
    x = res.x.cpu().numpy()
    assert OP.true_relres(p.A, x, p.b) <= 1.5 * p.tol
    assert np.linalg.norm(x - ref.x) <= 1e-7 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("prec", [OPr.FP64, OPr.FP32, OPr.BF16, OPr.FP16])
def test_config2_small_fixed_precision(prec):
    p = gen.config2(seed=1, N=24, b=32)
    nb = len(p.block_ptr) - 1
    pol = mb.Policy() if prec == OPr.FP64 else mb.Policy(mode=mb.FIXED, low=prec)
    res, _ = _gpu_solve(p.A, p.block_ptr, p.b, pol, 1e-10, 2000)
    ref = OP.solve_bjac(p.A, p.block_ptr, p.b, _tags(prec, nb), tol=1e-10, maxit=2000)
    ref64 = ref if prec == OPr.FP64 else OP.solve_bjac(p.A, p.block_ptr, p.b, tol=1e-10, maxit=2000)
    assert res.status == mb.OK
    delay = res.iters - ref64.iters
    print(f"prec {OPr.NAMES[prec]}: gpu {res.iters} oracle {ref.iters} oracle-fp64 {ref64.iters} delay {delay}")
    assert abs(res.iters - ref.iters) <= (2 if prec in (OPr.FP64, OPr.FP32) else 4)
    x = res.x.cpu().numpy()
    assert OP.true_relres(p.A, x, p.b) <= 2e-10


def test_uneven_blocks_mixed_explicit_map():
    rng = np.random.default_rng(8)
    A = gen.diffusion3d(gen.kappa_loguniform((20, 18, 16), rng))
    bp = gen.random_blocks(A.n, rng)
    nb = len(bp) - 1
    tags = rng.choice([OPr.FP64, OPr.FP32, OPr.FP16], size=nb).astype(np.uint8)
    b = rng.uniform(-1, 1, A.n)
    res, M = _gpu_solve(A, bp, b, mb.Policy(mode=mb.EXPLICIT, explicit_tags=tags), 1e-10, 2000)
    ref = OP.solve_bjac(A, bp, b, tags, tol=1e-10, maxit=2000)
    assert abs(res.iters - ref.iters) <= 3
    assert OP.true_relres(A, res.x.cpu().numpy(), b) <= 2e-10


def _amp_case():
    p = gen.config2(seed=2, N=20, b=32)
    return p.A, p.block_ptr, p.b


@pytest.mark.parametrize("temporal,adp", [(mb.TEMPORAL_HL, 1e-3), (mb.TEMPORAL_HL, 10.0), (mb.TEMPORAL_LH, 1e-4),
                                          (mb.TEMPORAL_LH, 10.0)])
def test_adaptive_switch_matches_oracle(temporal, adp):
    A, bp, b = _amp_case()
    nb = len(bp) - 1
    pol = mb.Policy(mode=mb.FIXED, low=mb.FP16, temporal=temporal, adp_tol=adp)
    res, _ = _gpu_solve(A, bp, b, pol, 1e-10, 2000)
    ref = OP.solve_bjac(A, bp, b, _tags(OPr.FP16, nb), tol=1e-10, maxit=2000, temporal=temporal, adp_tol=adp)
    assert abs(res.iters - ref.iters) <= 3
    # the switch sequence agrees wherever relres is not within rounding of adp_tol
    m = min(res.iters, ref.iters)
    seen = [math.inf] + ref.history[:m - 1]
    near = np.array([abs(v / adp - 1) < 1e-6 for v in seen])
    got = res.high_hist[:m].astype(bool)
    exp = np.array(ref.used_high[:m])
    assert np.array_equal(got[~near], exp[~near])
    assert res.high_applications == int(res.high_hist.sum())
    assert OP.true_relres(A, res.x.cpu().numpy(), b) <= 2e-10


def test_adaptive_degenerations_on_gpu():
    A, bp, b = _amp_case()
    uni, _ = _gpu_solve(A, bp, b, mb.Policy(), 1e-10, 2000)
    fmp, _ = _gpu_solve(A, bp, b, mb.Policy(mode=mb.FIXED, low=mb.FP16), 1e-10, 2000)
    hl0, _ = _gpu_solve(A, bp, b, mb.Policy(mode=mb.FIXED, low=mb.FP16, temporal=mb.TEMPORAL_HL, adp_tol=0.0),
                        1e-10, 2000)
    lh0, _ = _gpu_solve(A, bp, b, mb.Policy(mode=mb.FIXED, low=mb.FP16, temporal=mb.TEMPORAL_LH, adp_tol=0.0),
                        1e-10, 2000)
    assert hl0.iters == uni.iters and np.all(hl0.high_hist == 1)
    assert lh0.iters == fmp.iters and np.all(lh0.high_hist == 0)
    np.testing.assert_allclose(hl0.x.cpu().numpy(), uni.x.cpu().numpy(), rtol=0, atol=1e-12)
    np.testing.assert_allclose(lh0.x.cpu().numpy(), fmp.x.cpu().numpy(), rtol=0, atol=1e-12)


def test_rule_policy_matches_oracle_rule():
    p = gen.config3(seed=1, N=24, b=48)
    res, M = _gpu_solve(p.A, p.block_ptr, p.b, mb.Policy(mode=mb.RULE), 1e-10, 3000)
    H = OB.invert_blocks(p.A, p.block_ptr)
    F, raw = OB.block_features(p.A, p.block_ptr, H)
    tags = OB.select_rule(raw)
    ref = OP.solve_bjac(p.A, p.block_ptr, p.b, tags, tol=1e-10, maxit=3000)
    assert np.array_equal(M.tags(), tags)
    # mixed FP64/FP32 storage chosen per block
    assert len(set(tags.tolist())) >= 2
    assert abs(res.iters - ref.iters) <= max(3, 0.05 * ref.iters)
    assert OP.true_relres(p.A, res.x.cpu().numpy(), p.b) <= 2e-10


def test_fp64_long_anisotropic_solve_within_two_iterations():
    # the orientation of the paper's Ani(s) (strong y, z couplings across the
    # row blocks): ~1,100 iterations, where rounding differences accumulate
    rng = np.random.default_rng(1)
    A = gen.diffusion3d(gen.kappa_subcube_jumps(24, rng), aniso=(1.0, 1e3, 1e3))
    p = gen.Problem("ani", A, gen.uniform_blocks(A.n, 48), gen.rhs_uniform(A.n, rng), 1e-10, 3000)
    res, _ = _gpu_solve(p.A, p.block_ptr, p.b, mb.Policy(), 1e-10, 3000)
    ref = OP.solve_bjac(p.A, p.block_ptr, p.b, tol=1e-10, maxit=3000)
    print(f"fp64 anisotropic: gpu {res.iters} oracle {ref.iters}")
    assert abs(res.iters - ref.iters) <= 2


def test_chunk_size_and_determinism():
    A, bp, b = _amp_case()
    pol = mb.Policy(mode=mb.FIXED, low=mb.FP32)
    r2, _ = _gpu_solve(A, bp, b, pol, 1e-10, 2000, chunk=2)
    r16, _ = _gpu_solve(A, bp, b, pol, 1e-10, 2000, chunk=16)
    r16b, _ = _gpu_solve(A, bp, b, pol, 1e-10, 2000, chunk=16)
    assert r2.iters == r16.iters == r16b.iters
    assert np.array_equal(r16.x.cpu().numpy(), r16b.x.cpu().numpy())
    assert np.array_equal(r2.x.cpu().numpy(), r16.x.cpu().numpy())


def test_graph_reuse_across_right_hand_sides():
    A, bp, b = _amp_case()
    Ad = mb.DeviceCSR(A, dev())
    M = mb.BlockJacobi(Ad, bp, mb.Policy(mode=mb.FIXED, low=mb.FP16))
    S = mb.Solver(A.n, dev())
    x = tensor(np.zeros(A.n))
    rng = np.random.default_rng(9)
    for _ in range(3):
        bb = rng.uniform(-1, 1, A.n)
        r = S.solve(Ad, M, tensor(bb), tol=1e-10, maxit=2000, x=x)
        assert r.status == mb.OK
        assert OP.true_relres(A, r.x.cpu().numpy(), bb) <= 2e-10


@pytest.mark.parametrize("tol", [1e-10, 1e-12, 1e-15])
def test_verify_true_residual_and_restart(tol):
    # verify: when the recursive relres reaches tol, ||b - A x|| / ||b|| is
    # recomputed in FP64; above tol, r is replaced and CG restarts. Either the
    # FP64 true residual meets tol or every allowed restart was spent.
    rng = np.random.default_rng(3)
    A = gen.diffusion3d(gen.kappa_subcube_jumps(20, rng), aniso=(1e3, 1.0, 1.0))
    bp = gen.uniform_blocks(A.n, 48)
    b = gen.rhs_uniform(A.n, rng)
    Ad = mb.DeviceCSR(A, dev())
    # (an FP16 map of this small jump problem loses definiteness: breakdown)
    M = mb.BlockJacobi(Ad, bp, mb.Policy(mode=mb.FIXED, low=mb.FP32))
    S = mb.Solver(A.n, dev())
    r = S.solve(Ad, M, tensor(b), tol=tol, maxit=4000, verify=2, raise_on_error=False)
    x = r.x.cpu().numpy()
    host = OP.true_relres(A, x, b)
    assert r.true_relres > 0
    # both sides round A x in their own order: |delta ||b - A x||| <= 2 gamma_7 || |A| |x| ||
    S_abs = abs(A.to_scipy())
    bound = 2 * gamma(7, 2.0 ** -53) * np.linalg.norm(S_abs @ np.abs(x)) / np.linalg.norm(b)
    assert abs(r.true_relres - host) <= bound + 1e-6 * host
    if r.status == mb.OK:
        assert r.true_relres <= tol and host <= tol + bound
    else:
        assert r.status == mb.NOT_CONVERGED and r.restarts == 2
        assert host <= 1e-9
    print(f"tol {tol:g}: status {r.status}, iterations {r.iters}, restarts {r.restarts}, true relres {host:.3e}")
    # without verification the solve stops on the recursive residual alone
    r0 = S.solve(Ad, M, tensor(b), tol=tol, maxit=4000, raise_on_error=False)
    assert r0.restarts == 0 and r0.true_relres == -1.0
    assert r0.iters <= r.iters


def test_error_paths():
    A, bp, b = _amp_case()
    r, _ = _gpu_solve(A, bp, b, mb.Policy(), 1e-10, 1)
    assert r.status == mb.NOT_CONVERGED and r.iters == 1
    r, _ = _gpu_solve(A, bp, b, mb.Policy(), 1e-20, 30)
    assert r.status == mb.NOT_CONVERGED and r.iters == 30
    r, _ = _gpu_solve(A, bp, np.zeros(A.n), mb.Policy(), 1e-10, 30)
    assert r.status == mb.OK and r.iters == 0 and not np.any(r.x.cpu().numpy())
    bn = b.copy()
    bn[5] = np.nan
    r, _ = _gpu_solve(A, bp, bn, mb.Policy(), 1e-10, 30, raise_on_error=False)
    assert r.status == mb.EBREAKDOWN


def test_indefinite_matrix_breaks_down():
    # SPD (identity) diagonal blocks, indefinite A: p^T A p < 0 at the first step
    n, h = 64, 32
    rows = list(range(n)) + list(range(h)) + list(range(h, n))
    cols = list(range(n)) + list(range(h, n)) + list(range(h))
    vals = [1.0] * n + [2.0] * n
    A = gen._csr_from_coo(n, np.array(rows), np.array(cols), np.array(vals))
    b = np.concatenate([np.ones(h), -np.ones(h)])
    r, _ = _gpu_solve(A, gen.uniform_blocks(n, h), b, mb.Policy(), 1e-10, 30, raise_on_error=False)
    assert r.status == mb.EBREAKDOWN


def test_single_block_is_an_exact_solve():
    # block size n (Sec. 3.1 with one block): M^-1 = A^-1 and PCG converges in
    # one iteration with the FP64 map
    A = gen.poisson2d(8, 8)
    rng = np.random.default_rng(21)
    b = rng.uniform(-1, 1, A.n)
    res, _ = _gpu_solve(A, np.array([0, A.n], np.int32), b, mb.Policy(), 1e-10, 10)
    assert res.status == mb.OK and res.iters == 1
    assert OP.true_relres(A, res.x.cpu().numpy(), b) <= 1e-12


def test_unit_blocks_are_point_jacobi():
    # block size 1: the preconditioner is D^-1; iteration counts as the oracle's
    # point-Jacobi PCG
    rng = np.random.default_rng(22)
    A = gen.diffusion3d(gen.kappa_loguniform((9, 8, 7), rng))
    b = rng.uniform(-1, 1, A.n)
    bp = np.arange(A.n + 1, dtype=np.int32)
    res, _ = _gpu_solve(A, bp, b, mb.Policy(), 1e-10, 2000)
    d = A.to_scipy().diagonal()
    S = A.to_scipy()
    ref = OP.pcg(lambda v: S @ v, b, lambda r: r / d, 1e-10, 2000)
    assert res.status == mb.OK and abs(res.iters - ref.iters) <= 2


def test_one_row_system():
    A = gen._csr_from_coo(1, np.array([0]), np.array([0]), np.array([4.0]))
    res, _ = _gpu_solve(A, np.array([0, 1], np.int32), np.array([2.0]), mb.Policy(mode=mb.FIXED, low=mb.FP16), 1e-12, 5)
    assert res.status == mb.OK and res.iters == 1
    assert abs(res.x.cpu().numpy()[0] - 0.5) <= 1e-15


def _solve_pair(A, bp, b, maxit, pol=None):
    Ad = mb.DeviceCSR(A, dev())
    M = mb.BlockJacobi(Ad, bp, pol or mb.Policy(mode=mb.FIXED, low=mb.FP16))
    out = []
    for compact in (True, False):
        S = mb.Solver(A.n, dev(), compact_index=compact)
        out.append(S.solve(Ad, M, tensor(b), tol=1e-10, maxit=maxit, history=True, raise_on_error=False))
    return out


def test_compact_column_index_gives_identical_iterates():
    # the compact copy of the column indices (8-bit dictionary codes of
    # col - row here: 7 distinct offsets) changes only the bytes the SpMV
    # reads: the same products in the same order, identical iterates
    rng = np.random.default_rng(23)
    A = gen.diffusion3d(gen.kappa_loguniform((14, 12, 10), rng))
    b = rng.uniform(-1, 1, A.n)
    r1, r2 = _solve_pair(A, gen.uniform_blocks(A.n, 32), b, 2000)
    assert r1.status == mb.OK and r1.iters == r2.iters
    assert np.array_equal(r1.relres_hist, r2.relres_hist)
    assert np.array_equal(r1.x.cpu().numpy(), r2.x.cpu().numpy())


def _piecewise_constant(shape):
    # two coefficient values on two slabs: a handful of distinct matrix values
    k = np.ones(shape)
    k[: shape[0] // 2] = 100.0
    return gen.diffusion3d(k)


def test_value_codes_give_identical_iterates():
    # piecewise-constant coefficients: few distinct values, so the SpMV reads
    # 8-bit value codes beside the 8-bit column codes; against the CSR's own
    # arrays: the same products in the same order, identical iterates
    A = _piecewise_constant((14, 12, 10))
    assert len(np.unique(A.val)) <= 256
    b = np.random.default_rng(31).uniform(-1, 1, A.n)
    r1, r2 = _solve_pair(A, gen.uniform_blocks(A.n, 32), b, 2000)
    assert r1.status == mb.OK and r1.iters == r2.iters
    assert np.array_equal(r1.relres_hist, r2.relres_hist)
    assert np.array_equal(r1.x.cpu().numpy(), r2.x.cpu().numpy())


def _cycled_values_matrix(n, k):
    # symmetric 5-band matrix (offsets 0, +-1, +-2): the couplings cycle
    # through k distinct values, the diagonal is constant and dominant, and
    # two explicit zeros per 100 rows (stored +0.0 and -0.0, distinct keys of
    # the value dictionary); k + 3 distinct value patterns in all
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [np.full(n, 6.0)]
    e = 0
    for off in (1, 2):
        i = np.arange(n - off)
        v = -(1.0 + ((e + i) % k) / 1024.0)
        e += n
        rows += [i, i + off]
        cols += [i + off, i]
        vals += [v, v]
    z = np.arange(0, n - 3, 50)
    rows += [z, z + 3]
    cols += [z + 3, z]
    vals += [np.where(z % 100 == 0, 0.0, -0.0)] * 2
    return gen._csr_from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


@pytest.mark.parametrize("k", [253, 254])
def test_value_codes_at_the_dictionary_limit(k):
    # k = 253: 256 distinct values (bitwise), the dictionary's limit, so the
    # SpMV reads value codes; k = 254: 257, so it keeps the 8-byte values
    # (with the 8-bit column codes). Either way the iterates equal those of
    # the CSR's own arrays
    A = _cycled_values_matrix(3000, k)
    assert len(np.unique(A.val.view(np.uint64))) == k + 3
    b = np.random.default_rng(37).uniform(-1, 1, A.n)
    r1, r2 = _solve_pair(A, gen.uniform_blocks(A.n, 32), b, 2000)
    assert r1.status == mb.OK and r1.iters == r2.iters
    assert np.array_equal(r1.relres_hist, r2.relres_hist)
    assert np.array_equal(r1.x.cpu().numpy(), r2.x.cpu().numpy())


@pytest.mark.parametrize("coef", ["loguniform", "piecewise"])
def test_unaligned_matrix_arrays_read_unstaged_with_identical_iterates(coef):
    # values and indices not 16-byte aligned: the SpMV reads every tile's rows
    # straight from memory instead of staging 16-byte chunks (with 8-bit
    # value codes too for the piecewise-constant coefficients); the same
    # products in the same order, identical iterates
    import copy
    import torch
    rng = np.random.default_rng(29)
    A = (gen.diffusion3d(gen.kappa_loguniform((13, 11, 9), rng)) if coef == "loguniform"
         else _piecewise_constant((13, 11, 9)))
    b = rng.uniform(-1, 1, A.n)
    bp = gen.uniform_blocks(A.n, 32)
    Ad = mb.DeviceCSR(A, dev())
    Au = copy.copy(Ad)
    vbuf = torch.zeros(A.nnz + 1, dtype=torch.float64, device=dev())
    cbuf = torch.zeros(A.nnz + 1, dtype=torch.int32, device=dev())
    vbuf[1:] = Ad.val
    cbuf[1:] = Ad.col_idx
    Au.val, Au.col_idx = vbuf[1:], cbuf[1:]
    assert Au.val.data_ptr() % 16 == 8 and Au.col_idx.data_ptr() % 16 == 4
    Au.c = mb.bjac_csr(Au.n, Au.nnz, Au.row_ptr.data_ptr(), Au.col_idx.data_ptr(), Au.val.data_ptr())
    out = []
    for AA in (Ad, Au):
        M = mb.BlockJacobi(AA, bp, mb.Policy(mode=mb.FIXED, low=mb.FP16))
        for compact in (True, False):
            S = mb.Solver(A.n, dev(), compact_index=compact)
            out.append(S.solve(AA, M, tensor(b), tol=1e-10, maxit=2000, history=True, raise_on_error=False))
    assert out[0].status == mb.OK
    for r in out[1:]:
        assert r.status == mb.OK and r.iters == out[0].iters
        assert np.array_equal(r.relres_hist, out[0].relres_hist)
        assert np.array_equal(r.x.cpu().numpy(), out[0].x.cpu().numpy())


def _random_sparse_spd(n, per_row, far, rng):
    # diagonally dominant SPD matrix with `per_row` random couplings per row,
    # columns up to `far` rows away: hundreds of distinct offsets col - row
    rows = np.repeat(np.arange(n), per_row)
    cols = (rows + rng.integers(-far, far + 1, size=rows.size)) % n
    keep = cols != rows
    rows, cols = rows[keep], cols[keep]
    vals = -rng.uniform(0.1, 1.0, size=rows.size)
    r = np.concatenate([rows, cols])
    c = np.concatenate([cols, rows])
    v = np.concatenate([vals, vals])
    import scipy.sparse as sp
    S = sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()
    S.sum_duplicates()
    S = S + sp.diags(np.asarray(abs(S).sum(axis=1)).ravel() + 1.0)
    S = S.tocsr()
    S.sort_indices()
    return gen.CSR(n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data)


@pytest.mark.parametrize("n,far", [(6000, 3000), (70000, 35000)])
def test_compact_column_index_beyond_the_dictionary(n, far):
    # more than 256 distinct offsets: the dictionary overflows and the products
    # read the 16-bit offsets (n = 6000) or the CSR's 32-bit indices (offsets
    # beyond 16 bits), identical to the plain workspace either way
    rng = np.random.default_rng(25)
    A = _random_sparse_spd(n, 3, far, rng)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    assert len(np.unique(A.col_idx - rows)) > 256
    b = rng.uniform(-1, 1, A.n)
    r1, r2 = _solve_pair(A, gen.uniform_blocks(A.n, 32), b, 500)
    assert r1.status == mb.OK and r1.iters == r2.iters
    assert np.array_equal(r1.relres_hist, r2.relres_hist)
    assert np.array_equal(r1.x.cpu().numpy(), r2.x.cpu().numpy())


def test_compact_column_index_falls_back_for_far_couplings():
    # a 33000 x 2 grid couples rows 33000 apart, beyond 16 bits, with five
    # distinct offsets: the products read the 8-bit codes, identical to the
    # plain workspace
    A = gen.poisson2d(33000, 2)
    rng = np.random.default_rng(24)
    b = rng.uniform(-1, 1, A.n)
    r1, r2 = _solve_pair(A, gen.uniform_blocks(A.n, 32), b, 200)
    assert r1.status == mb.OK and r1.iters == r2.iters
    assert np.array_equal(r1.relres_hist, r2.relres_hist)
    assert np.array_equal(r1.x.cpu().numpy(), r2.x.cpu().numpy())


@pytest.mark.parametrize("b", [32, 48, 64])
@pytest.mark.parametrize("prec,slack", [(OPr.FP64, 1), (OPr.FP32, 2), (OPr.FP16, 2)])
def test_sym_storage_pcg_matches_oracle(prec, slack, b):
    # symmetric storage holds FULL's values (the lower quarters read as the
    # transposes of the upper ones): the oracle's full-storage PCG is the
    # reference
    rng = np.random.default_rng(41 + b)
    A = gen.diffusion3d(gen.kappa_loguniform((24, 20, 16), rng))
    bp = gen.uniform_blocks(A.n, b)
    nb = len(bp) - 1
    b = rng.uniform(-1, 1, A.n)
    Ad = mb.DeviceCSR(A, dev())
    pol = (mb.Policy(mode=mb.UNIFORM, storage=mb.STORE_SYM) if prec == OPr.FP64
           else mb.Policy(mode=mb.FIXED, low=prec, storage=mb.STORE_SYM))
    M = mb.BlockJacobi(Ad, bp, pol)
    res = mb.Solver(A.n, dev()).solve(Ad, M, tensor(b), tol=1e-10, maxit=3000)
    ref = OP.solve_bjac(A, bp, b, np.full(nb, prec, np.uint8), tol=1e-10, maxit=3000)
    assert res.status == mb.OK and ref.status == OP.CONVERGED
    assert abs(res.iters - ref.iters) <= slack, (res.iters, ref.iters)
    assert OP.true_relres(A, res.x.cpu().numpy(), b) <= 2e-10


def test_sym_storage_temporal_and_rule_maps():
    # both maps of a temporal handle and a per-block rule map (generic kernel)
    rng = np.random.default_rng(42)
    A = gen.diffusion3d(gen.kappa_loguniform((20, 16, 12), rng))
    bp = gen.uniform_blocks(A.n, 32)
    nb = len(bp) - 1
    b = rng.uniform(-1, 1, A.n)
    Ad = mb.DeviceCSR(A, dev())
    M = mb.BlockJacobi(Ad, bp, mb.Policy(mode=mb.FIXED, low=mb.FP16, temporal=mb.TEMPORAL_HL, adp_tol=1e-4,
                                         storage=mb.STORE_SYM))
    res = mb.Solver(A.n, dev()).solve(Ad, M, tensor(b), tol=1e-10, maxit=3000)
    ref = OP.solve_bjac(A, bp, b, np.full(nb, OPr.FP16, np.uint8), tol=1e-10, maxit=3000,
                        temporal=OP.TEMPORAL_HL, adp_tol=1e-4)
    assert res.status == mb.OK and abs(res.iters - ref.iters) <= 2, (res.iters, ref.iters)
    Mr = mb.BlockJacobi(Ad, bp, mb.Policy(mode=mb.RULE, storage=mb.STORE_SYM))
    Mf = mb.BlockJacobi(Ad, bp, mb.Policy(mode=mb.RULE))
    assert np.array_equal(Mr.tags(), Mf.tags())
    rr = mb.Solver(A.n, dev()).solve(Ad, Mr, tensor(b), tol=1e-10, maxit=3000)
    rf = mb.Solver(A.n, dev()).solve(Ad, Mf, tensor(b), tol=1e-10, maxit=3000)
    assert rr.status == mb.OK and abs(rr.iters - rf.iters) <= 2
    assert OP.true_relres(A, rr.x.cpu().numpy(), b) <= 2e-10
