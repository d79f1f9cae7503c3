"""Distinct handles used from distinct threads (the ABI's threading promise):
two PCG solves, each on its own handle, workspace and stream, run at the same
time from two host threads and return exactly the iterates they return when
run alone (the kernels are deterministic, so bit-identical)."""
import threading

import numpy as np
import pytest

from paper_2407_15973_amd import binding as mb
from paper_2407_15973_amd import gen

from gpu_helpers import dev, tensor

pytestmark = pytest.mark.gpu


def _case(seed, shape, b, policy):
    rng = np.random.default_rng(seed)
    A = gen.diffusion3d(gen.kappa_loguniform(shape, rng))
    return A, gen.uniform_blocks(A.n, b), rng.uniform(-1, 1, A.n), policy


def _solve(case, stream=None):
    import torch
    A, bp, b, pol = case
    with torch.cuda.stream(stream or torch.cuda.current_stream()):
        Ad = mb.DeviceCSR(A, dev())
        M = mb.BlockJacobi(Ad, bp, pol)
        res = mb.Solver(A.n, dev()).solve(Ad, M, tensor(b), tol=1e-10, maxit=3000, history=True)
        torch.cuda.current_stream().synchronize()
        return res.iters, res.status, res.x.cpu().numpy(), res.relres_hist


@pytest.mark.parametrize("rounds", [2])
def test_two_handles_from_two_threads(rounds):
    import torch
    cases = [_case(51, (24, 20, 16), 32, mb.Policy(mode=mb.FIXED, low=mb.FP16, storage=mb.STORE_SYM)),
             _case(52, (20, 18, 16), 48, mb.Policy(mode=mb.RULE))]
    alone = [_solve(c) for c in cases]
    for it, st, _, _ in alone:
        assert st == mb.OK and it > 10
    for _ in range(rounds):
        out = [None, None]
        errs = []

        def run(i):
            try:
                out[i] = _solve(cases[i], torch.cuda.Stream(device=dev()))
            except Exception as e:  # reported below
                errs.append(e)

        ts = [threading.Thread(target=run, args=(i,)) for i in range(2)]
        for t in ts:
            t.start()
        for t in ts:
            t.join(timeout=120)
        assert not errs, errs
        for (it, st, x, h), (it0, st0, x0, h0) in zip(out, alone):
            assert st == st0 and it == it0
            np.testing.assert_array_equal(x, x0)
            np.testing.assert_array_equal(h, h0)
