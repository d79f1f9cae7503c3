"""Pins of the oracle's label generation (oracle.labels): the ladder's
degenerate ends and its defining property, checked by brute force over the
ladder on small problems."""
import math

import numpy as np

from oracle import blocks as OB
from oracle import labels as OL
from oracle import pcg as OP
from oracle import precision as P
from paper_2407_15973_amd import gen


def test_tags_for_eta_ladder_ends_and_monotone():
    kap = np.array([1.0, 10.0, 1e3, 1e6, 1e9, 1e12])
    assert np.all(OL.tags_for_eta(kap, math.inf) == P.FP16)
    assert np.all(OL.tags_for_eta(kap, 0.0) == P.FP64)
    # kappa u <= eta, u = 2^-11 (FP16), 2^-24 (FP32)
    t = OL.tags_for_eta(kap, 1e-2)
    expect = [P.FP16 if k * 2.0 ** -11 <= 1e-2 else P.FP32 if k * 2.0 ** -24 <= 1e-2 else P.FP64 for k in kap]
    assert list(t) == expect
    # lowering eta never lowers a block's precision (classes 0 FP64 < 1 FP32 < 2 FP16)
    prev = None
    for eta in OL.ETAS:
        cls = np.array([OL.CLASS_OF_TAG[int(x)] for x in OL.tags_for_eta(kap, eta)])
        if prev is not None:
            assert np.all(cls <= prev)
        prev = cls


def test_poisson_labels_all_fp16():
    # the line-block 2D Poisson blocks are well conditioned: the first rung
    # (every block FP16) keeps the delay within 5 %
    p = gen.config1(0)
    lab = OL.make_labels(p.A, p.block_ptr, p.b, tol=p.tol, maxit=p.maxit)
    assert lab.eta == math.inf and np.all(lab.labels == 2)
    assert lab.iters <= 1.05 * lab.it64


def test_labels_are_the_largest_passing_rung_by_brute_force():
    # a high-contrast 3D problem: solve every rung of the ladder directly and
    # check the chosen map is the first (largest eta) within the delay bar
    rng = np.random.default_rng(3)
    A = gen.diffusion3d(gen.kappa_loguniform((12, 12, 12), rng, lo=-5, hi=5))
    bp = gen.uniform_blocks(A.n, 24)
    b = rng.uniform(-1, 1, A.n)
    lab = OL.make_labels(A, bp, b, tol=1e-10, maxit=3000)
    H = OB.invert_blocks(A, bp)
    _, raw = OB.block_features(A, bp, H)
    it64 = OP.solve_bjac(A, bp, b, np.zeros(len(H), np.uint8), tol=1e-10, maxit=3000).iters
    assert lab.it64 == it64
    for eta in OL.ETAS:
        tags = OL.tags_for_eta(raw["kappa1"], eta)
        r = OP.solve_bjac(A, bp, b, tags, tol=1e-10, maxit=3000)
        it = r.iters if r.status == OP.CONVERGED else 3001
        if it <= 1.05 * it64:
            assert lab.eta == eta
            assert np.array_equal(lab.labels, [OL.CLASS_OF_TAG[int(t)] for t in tags])
            break
    else:
        assert lab.eta == 0.0 and np.all(lab.labels == 0)


def test_no_passing_rung_gives_fp64():
    # a bar no map meets (half the FP64 iteration count, delay = -0.5): no
    # rung passes, not even eta = 0 (all FP64), and the labels are all FP64
    p = gen.config2(seed=1, N=8, b=32)
    lab = OL.make_labels(p.A, p.block_ptr, p.b, tol=1e-10, maxit=500, delay=-0.5)
    assert lab.eta == 0.0 and np.all(lab.labels == 0)
