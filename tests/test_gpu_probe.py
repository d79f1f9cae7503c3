"""The streaming probe (bjac_stream_probe, the measurement aid behind the
roofline ceilings): its outputs are the sums it defines, for every mix and
launch shape, including a ragged tail; invalid arguments are rejected."""
import numpy as np
import pytest

from paper_2407_15973_amd import binding as mb

from gpu_helpers import dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ni,no", [(1, 0), (0, 1), (1, 1), (4, 1), (6, 1), (8, 2)])
@pytest.mark.parametrize("grid,unroll", [(0, 1), (3, 2), (1024, 4)])
def test_stream_probe_outputs(ni, no, grid, unroll):
    import torch
    n = 2 * 100003            # even, not a multiple of a launch's stride
    rng = np.random.default_rng(ni * 10 + no)
    ins = [torch.as_tensor(rng.integers(-8, 8, size=n).astype(np.float64), device=dev()) for _ in range(ni)]
    outs = [torch.full((n,), np.nan, dtype=torch.float64, device=dev()) for _ in range(no)]
    sink = torch.zeros(8192 * 256, dtype=torch.float64, device=dev())
    mb.stream_probe(ins, outs, grid=grid, unroll=unroll, sink=sink)
    torch.cuda.synchronize()
    total = sum(t.cpu().numpy() for t in ins) if ins else np.zeros(n)
    for j, o in enumerate(outs):
        np.testing.assert_array_equal(o.cpu().numpy(), total + j)
    if no == 0:
        # the read-only mix leaves each thread's partial sum: all of them add up
        # to the sum of the inputs (integers: exact)
        assert float(sink.sum().cpu()) == float(total.sum())


def test_stream_probe_rejects_bad_arguments():
    import torch
    a = torch.zeros(64, dtype=torch.float64, device=dev())
    with pytest.raises(mb.MpbjacError):
        mb.stream_probe([a] * 9, [a])            # more than 8 inputs
    with pytest.raises(mb.MpbjacError):
        mb.stream_probe([a], [], sink=None)      # read-only mix without sink
    with pytest.raises(mb.MpbjacError):
        mb.stream_probe([a[:63]], [a[1:]])       # odd count
    with pytest.raises(mb.MpbjacError):
        mb.stream_probe([a], [a], unroll=3)
