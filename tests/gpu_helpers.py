"""Shared helpers of the GPU parity tests (device transfer, oracle runs)."""
import numpy as np

from oracle import blocks as OB
from oracle import pcg as OP
from oracle import precision as OPr


def dev():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return "cuda:0"


def tensor(a, device=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device=device or dev())


def ulp(x, prec):
    """Spacing of the format at |x| (for x = 0 the smallest subnormal)."""
    p, emin = {OPr.FP32: (24, -126), OPr.BF16: (8, -126), OPr.FP16: (11, -14), OPr.FP64: (53, -1022)}[prec]
    x = np.abs(np.asarray(x, dtype=np.float64))
    e = np.floor(np.log2(np.where(x > 0, x, 1.0)))
    e = np.where(x > 0, np.maximum(e, emin), emin)
    return np.ldexp(1.0, (e - (p - 1)).astype(np.int64))


def oracle_setup(A, bp, tags):
    H = OB.invert_blocks(A, bp)
    return H, OB.store_blocks(H, tags)


def gamma(b, u):
    return b * u / (1 - b * u)
