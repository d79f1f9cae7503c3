"""Pins of the oracle's single-reduction PCG (Chronopoulos-Gear) against facts
the mathematics fixes: finite termination on tiny SPD systems (point Jacobi)
and on 1D Poisson right-hand sides with m eigen-components, the exact
preconditioner (one iteration), the A-norm error decreasing, and agreement
with the textbook recurrence (the two produce the same iterates in exact
arithmetic). A slip in the recurrence fails them."""
import numpy as np
import pytest

from paper_2407_15973_amd import gen
from oracle import pcg as OP
from oracle import precision as P


def _spd(rng, n):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * np.exp(rng.uniform(0, 3, n))) @ Q.T


def _poisson1d(n):
    i = np.arange(n)
    return gen._csr_from_coo(n, np.concatenate([i, i[1:], i[:-1]]), np.concatenate([i, i[:-1], i[1:]]),
                             np.concatenate([np.full(n, 2.0), -np.ones(n - 1), -np.ones(n - 1)]))


@pytest.mark.parametrize("n", [1, 2, 5, 8, 10])
def test_tiny_spd_converges_within_n(n):
    rng = np.random.default_rng(100 + n)
    D = _spd(rng, n)
    b = rng.uniform(-1, 1, n)
    d = np.diag(D).copy()
    res = OP.pcg_single_reduction(lambda v: D @ v, b, lambda r: r / d, 1e-10, 50)
    assert res.status == OP.CONVERGED and res.iters <= n
    np.testing.assert_allclose(D @ res.x, b, atol=1e-8)


def test_poisson1d_eigen_components_finite_termination():
    # tridiag(-1, 2, -1) with point Jacobi (M^-1 A = A / 2): an RHS made of m
    # eigenvectors sin(i j pi / (n+1)) is solved in exactly m steps
    n = 60
    A = _poisson1d(n)
    S = A.to_scipy()
    V = np.sin(np.outer(np.arange(1, n + 1), np.arange(1, n + 1)) * np.pi / (n + 1))
    for m in (1, 3, 7):
        b = V[:, [4, 17, 31, 40, 50, 55, 58][:m]].sum(axis=1)
        res = OP.pcg_single_reduction(lambda v: S @ v, b, lambda r: r / 2.0, 1e-10, 100)
        assert res.status == OP.CONVERGED and res.iters == m


def test_whole_matrix_block_is_exact_one_iteration():
    A = gen.poisson2d(16, 16)
    b = np.random.default_rng(7).uniform(-1, 1, A.n)
    res = OP.solve_bjac_single_reduction(A, gen.uniform_blocks(A.n, A.n), b, tol=1e-8, maxit=10)
    assert res.iters == 1 and res.status == OP.CONVERGED
    assert OP.true_relres(A, res.x, b) < 1e-12


def test_matches_textbook_recurrence():
    # same iterates in exact arithmetic: iteration counts within one and
    # solutions within the stopping tolerance's reach on a 3D diffusion case,
    # FP64 and FP16 block maps
    rng = np.random.default_rng(8)
    A = gen.diffusion3d(gen.kappa_loguniform((12, 10, 8), rng))
    bp = gen.uniform_blocks(A.n, 24)
    b = rng.uniform(-1, 1, A.n)
    for prec in (P.FP64, P.FP16):
        tags = np.full(len(bp) - 1, prec, np.uint8)
        M = OP.BJAC(A, bp, tags)
        hs = OP.solve_bjac(A, bp, b, tags, tol=1e-10, maxit=2000, M=M)
        cg = OP.solve_bjac_single_reduction(A, bp, b, tags, tol=1e-10, maxit=2000, M=M)
        assert hs.status == cg.status == OP.CONVERGED
        assert abs(hs.iters - cg.iters) <= 1, (hs.iters, cg.iters)
        k = min(len(hs.history), len(cg.history), 40)
        np.testing.assert_allclose(cg.history[:k], hs.history[:k], rtol=1e-6)
        assert OP.true_relres(A, cg.x, b) <= 2e-10


def test_a_norm_error_monotone():
    rng = np.random.default_rng(9)
    A = gen.diffusion3d(gen.kappa_loguniform((10, 10, 10), rng))
    S = A.to_scipy()
    xs = rng.uniform(-1, 1, A.n)
    b = S @ xs
    M = OP.BJAC(A, gen.uniform_blocks(A.n, 10))
    errs = []
    for it in range(1, 40):
        res = OP.pcg_single_reduction(lambda v: S @ v, b, M.low, 0.0, it)
        e = res.x - xs
        errs.append(e @ (S @ e))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-10) for i in range(len(errs) - 1))


def test_wrong_alpha_breaks_finite_termination():
    # the pins above fail for a plausible slip in the recurrence: with the
    # correction term's sign flipped (delta + beta gamma / alpha_old) a 1D
    # Poisson RHS of 3 eigen-components is no longer solved in 3 steps
    n = 60
    S = _poisson1d(n).to_scipy()
    V = np.sin(np.outer(np.arange(1, n + 1), np.arange(1, n + 1)) * np.pi / (n + 1))
    b = V[:, [4, 17, 31]].sum(axis=1)

    def slipped(matvec, b, precond, tol, maxit):
        x = np.zeros_like(b)
        r = b.copy()
        r0 = np.linalg.norm(r)
        p = np.zeros_like(b)
        s = np.zeros_like(b)
        go = ao = 0.0
        for j in range(maxit + 1):
            if j > 0 and np.linalg.norm(r) / r0 <= tol:
                return j
            u = precond(r)
            w = matvec(u)
            g, d = r @ u, w @ u
            beta = 0.0 if j == 0 else g / go
            a = g / (d if j == 0 else d + beta * g / ao)
            p, s = u + beta * p, w + beta * s
            x += a * p
            r -= a * s
            go, ao = g, a
        return maxit + 1

    assert slipped(lambda v: S @ v, b, lambda r: r / 2.0, 1e-10, 20) > 3
    res = OP.pcg_single_reduction(lambda v: S @ v, b, lambda r: r / 2.0, 1e-10, 20)
    assert res.iters == 3
