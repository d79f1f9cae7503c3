"""GPU selector-network kernels against the FP64 oracle MLP: forward logits,
argmax tags, backward gradient of the mean cross-entropy, Adam step, and the
LEARNED precision policy in the setup."""
import numpy as np
import pytest

from oracle import mlp as OM
from oracle import precision as OPr
from paper_2407_15973_amd import binding as mb
from paper_2407_15973_amd import gen

from gpu_helpers import dev, tensor

pytestmark = pytest.mark.gpu


def _case(seed, N=300):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, 16)) * rng.uniform(0.5, 3, 16) + rng.uniform(-2, 2, 16)
    y = rng.integers(0, 3, size=N).astype(np.int32)
    mu = X.mean(axis=0)
    sig = X.std(axis=0) + 0.1
    th = OM.init_params(rng)
    th[-3:] = rng.standard_normal(3) * 0.2
    return X.astype(np.float32), y, mu, sig, th


def _blob(th, mu, sig):
    return tensor(np.concatenate([th, mu, sig]).astype(np.float32))


def _f64(x32):
    return np.asarray(x32, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("N", [1, 7, 300, 5000])
def test_forward_logits_and_tags(N):
    X, y, mu, sig, th = _case(1, N)
    blob = _blob(th, mu, sig)
    logits, tags = mb.mlp_forward(blob, tensor(X), want_logits=True, want_tags=True)
    ref, _ = OM.forward(_f64(th), _f64(X), _f64(mu.astype(np.float32)), _f64(sig.astype(np.float32)))
    got = logits.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got, ref, rtol=1e-4, atol=1e-4 * np.abs(ref).max())
    cls = np.argmax(ref, axis=1)
    clear = np.sort(ref, axis=1)[:, -1] - np.sort(ref, axis=1)[:, -2] > 1e-3 * np.abs(ref).max()
    tag_of = np.array([OPr.FP64, OPr.FP32, OPr.FP16])
    assert np.array_equal(tags.cpu().numpy()[clear], tag_of[cls[clear]])


@pytest.mark.parametrize("N", [5, 300, 4099])
def test_backward_matches_oracle_gradient(N):
    X, y, mu, sig, th = _case(2, N)
    blob = _blob(th, mu, sig)
    tr = mb.MlpTrainer(N, dev())
    g, loss = tr.backward(blob, tensor(X), tensor(y))
    args = (_f64(th.astype(np.float32)), _f64(X), y, _f64(mu.astype(np.float32)), _f64(sig.astype(np.float32)))
    gref = OM.backward(*args)
    lref = OM.loss(*args)
    got = g.cpu().numpy().astype(np.float64)
    assert abs(float(loss.cpu()) - lref) <= 1e-4 * max(1.0, abs(lref))
    scale = np.abs(gref).max()
    np.testing.assert_allclose(got, gref, rtol=0, atol=1e-4 * scale)
    rel = np.linalg.norm(got - gref) / np.linalg.norm(gref)
    assert rel < 1e-4


def test_backward_deterministic():
    X, y, mu, sig, th = _case(3, 2000)
    blob = _blob(th, mu, sig)
    tr = mb.MlpTrainer(2000, dev())
    g1 = tr.backward(blob, tensor(X), tensor(y))[0].cpu().numpy().copy()
    g2 = tr.backward(blob, tensor(X), tensor(y))[0].cpu().numpy().copy()
    assert np.array_equal(g1, g2)


def test_adam_step_matches_oracle():
    # a seeded gradient is written into the trainer's gradient buffer and fed
    # to the oracle's Adam: the update rule is what is compared
    X, y, mu, sig, th = _case(4, 500)
    blob = _blob(th, mu, sig)
    tr = mb.MlpTrainer(500, dev())
    rng = np.random.default_rng(11)
    th_ref = _f64(th.astype(np.float32))
    m = np.zeros(OM.NPARAM)
    v = np.zeros(OM.NPARAM)
    for t in range(1, 4):
        g = (rng.standard_normal(OM.NPARAM) * np.exp(rng.uniform(-6, 0, OM.NPARAM))).astype(np.float32)
        tr.grad.copy_(tensor(g))
        tr.adam(blob, lr=1e-2)
        th_ref, m, v = OM.adam_step(th_ref, _f64(g), m, v, t, lr=1e-2)
        got = blob.cpu().numpy()[:OM.NPARAM].astype(np.float64)
        np.testing.assert_allclose(got, th_ref, rtol=0, atol=2e-6)


def test_learned_policy_uses_network_tags():
    p = gen.config2(seed=3, N=20, b=32)
    Ad = mb.DeviceCSR(p.A, dev())
    M0 = mb.BlockJacobi(Ad, p.block_ptr, mb.Policy(mode=mb.UNIFORM))
    feat = M0.features()
    rng = np.random.default_rng(5)
    th = OM.init_params(rng)
    mu, sig = feat.mean(axis=0).astype(np.float64), feat.std(axis=0).astype(np.float64) + 1e-3
    blob = _blob(th, mu, sig)
    _, tags = mb.mlp_forward(blob, tensor(feat), want_logits=False, want_tags=True)
    M = mb.BlockJacobi(Ad, p.block_ptr, mb.Policy(mode=mb.LEARNED, mlp_blob=blob))
    assert np.array_equal(M.tags(), tags.cpu().numpy())
    res = mb.Solver(p.A.n, dev()).solve(Ad, M, tensor(p.b), tol=1e-10, maxit=3000)
    assert res.status == mb.OK
