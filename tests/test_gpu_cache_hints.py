"""The streaming (non-temporal) and plain variants of a PCG iteration's
launches run the same arithmetic in the same order: forced either way
through the solve options, they give bitwise identical iterates, on the
arithmetic-tile path (uniform blocks, symmetric and full storage), on the
generic path (the per-block rule map, explicit mixed maps), with the
adaptive switch's split launches and in the single-reduction recurrence."""
import numpy as np
import pytest

from paper_2407_15973_amd import binding as mb
from paper_2407_15973_amd import gen

from gpu_helpers import dev, tensor

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,policy", [
    ("fp16_sym", dict(mode=mb.FIXED, low=mb.FP16, storage=mb.STORE_SYM)),
    ("fp64_sym", dict(storage=mb.STORE_SYM)),
    ("fp32_full", dict(mode=mb.FIXED, low=mb.FP32)),
    ("rule", dict(mode=mb.RULE)),
    ("mixed_sym", dict(mode=mb.EXPLICIT, storage=mb.STORE_SYM)),   # generic path, every precision
    ("mixed_full", dict(mode=mb.EXPLICIT)),
    ("temporal_hl", dict(mode=mb.FIXED, low=mb.FP16, temporal=mb.TEMPORAL_HL, adp_tol=1e-4)),   # split launches
    ("fp16_sym_single_reduction", dict(mode=mb.FIXED, low=mb.FP16, storage=mb.STORE_SYM, variant=mb.PCG_SINGLE_REDUCTION)),
])
def test_stream_and_plain_hints_give_identical_iterates(name, policy):
    p = gen.config2(seed=3, N=24, b=32)
    A = mb.DeviceCSR(p.A, dev())
    b = tensor(p.b)
    if policy.get("mode") == mb.EXPLICIT:
        nb = len(p.block_ptr) - 1
        policy = dict(policy, explicit_tags=np.array([mb.FP64, mb.FP32, mb.BF16, mb.FP16], np.uint8)[np.arange(nb) % 4])
    variant = policy.pop("variant", mb.PCG_TEXTBOOK)
    M = mb.BlockJacobi(A, p.block_ptr, mb.Policy(**policy))
    s = mb.Solver(p.A.n, dev())
    out = {}
    for hints in (mb.HINTS_PLAIN, mb.HINTS_STREAM, mb.HINTS_AUTO):
        r = s.solve(A, M, b, tol=1e-10, maxit=2000, history=True, cache_hints=hints, variant=variant)
        assert r.status == mb.OK
        out[hints] = (r.iters, r.x.cpu().numpy().copy(), r.relres_hist.copy())
    it0, x0, h0 = out[mb.HINTS_PLAIN]
    for hints in (mb.HINTS_STREAM, mb.HINTS_AUTO):
        it, x, h = out[hints]
        assert it == it0, (name, hints)
        assert np.array_equal(x, x0), (name, hints)
        assert np.array_equal(h, h0), (name, hints)


def test_cache_hints_out_of_range_rejected():
    p = gen.config2(seed=3, N=16, b=32)
    A = mb.DeviceCSR(p.A, dev())
    M = mb.BlockJacobi(A, p.block_ptr, mb.Policy())
    s = mb.Solver(p.A.n, dev())
    with pytest.raises(mb.MpbjacError):
        s.solve(A, M, tensor(p.b), cache_hints=3)
