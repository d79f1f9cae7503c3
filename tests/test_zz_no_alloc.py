"""pcg_solve_noalloc (the solve without allocation, for callers that cannot
allocate) against pcg_solve: two calls in a row on the same GPU, the second
with a smaller system, each equal to pcg_solve's result on the same inputs
(the same kernels in the same order: identical iterates). All calls go
through the C ABI."""
import numpy as np
import pytest

from oracle import pcg as OP
from paper_2407_15973_amd import binding as mb
from paper_2407_15973_amd import gen

from gpu_helpers import dev, tensor

pytestmark = pytest.mark.gpu


def _case(seed, shape, b):
    rng = np.random.default_rng(seed)
    A = gen.diffusion3d(gen.kappa_loguniform(shape, rng))
    return A, gen.uniform_blocks(A.n, b), rng.uniform(-1, 1, A.n)


@pytest.mark.parametrize("variant", [mb.PCG_TEXTBOOK, mb.PCG_SINGLE_REDUCTION])
def test_noalloc_matches_pcg_solve_two_calls(variant):
    import torch
    big = _case(81, (40, 36, 32), 32)      # 46,080 rows
    small = _case(82, (20, 18, 12), 48)    # 4,320 rows: the second call
    pols = (mb.Policy(mode=mb.FIXED, low=mb.FP16, storage=mb.STORE_SYM), mb.Policy(mode=mb.RULE))
    for (A, bp, rhs), pol in zip((big, small), pols):
        print(f"[noalloc] variant {variant} n = {A.n}", flush=True)
        Ad = mb.DeviceCSR(A, dev())
        M = mb.BlockJacobi(Ad, bp, pol)
        bt = tensor(rhs)
        ref = mb.Solver(A.n, dev(), compact_index=False).solve(Ad, M, bt, tol=1e-10, maxit=3000, variant=variant,
                                                              verify=2)
        x = torch.full((A.n,), float("nan"), dtype=torch.float64, device=dev())
        got = mb.solve_noalloc(Ad, M, bt, x, tol=1e-10, maxit=3000, variant=variant, verify=2)
        torch.cuda.synchronize()
        assert got.status == ref.status == mb.OK
        assert got.iters == ref.iters and got.restarts == ref.restarts
        np.testing.assert_array_equal(x.cpu().numpy(), ref.x.cpu().numpy())
        assert OP.true_relres(A, x.cpu().numpy(), rhs) <= 2e-10


def test_noalloc_rejects_beyond_its_workspace():
    A = gen.poisson2d(1100, 1000)          # 1,100,000 rows > 1,048,576
    Ad = mb.DeviceCSR(A, dev())
    M = mb.BlockJacobi(Ad, gen.uniform_blocks(A.n, 64), mb.Policy(mode=mb.FIXED, low=mb.FP16))
    b = tensor(np.ones(A.n))
    import torch
    x = torch.empty_like(b)
    with pytest.raises(mb.MpbjacError) as e:
        mb.solve_noalloc(Ad, M, b, x, tol=1e-10, maxit=10)
    assert e.value.code == mb.ENOMEM
