"""GPU parity of the MLP training kernels (forward, backward, MSE of Eq. 17,
Adam) against the oracle, through the C ABI.

Gradients are compared with the oracle's FP64 chain rule on the same BF16
operands (``oracle.mlp.grad_bf16``): the GPU accumulates in FP32 and rounds
its own FP32 activations, so an operand can land one BF16 step away; the
bound is a relative Frobenius error of 1e-4 per tensor and 1e-3 of the
tensor's largest entry per element (measured: at most 4e-6)."""
import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from oracle import splitmix64
from paper_2506_05293_amd import lbm

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu case]", *a, flush=True)


def _data(n, seed=0):
    rng = np.random.default_rng(seed)
    x = (0.003 + 0.01 * rng.standard_normal((n, 27))).astype(np.float32)
    t = (1e-4 * rng.standard_normal((n, 3)) + 2e-5).astype(np.float32)
    return x, t


def _weights(seed, scale=1.0):
    rng = np.random.default_rng(seed)

    def glorot(o, i):
        a = np.sqrt(6.0 / (o + i)) * scale
        return rng.uniform(-a, a, (o, i)).astype(np.float32)
    return {"w1": glorot(64, 27), "b1": (0.05 * rng.standard_normal(64)).astype(np.float32),
            "w2": glorot(64, 64), "b2": (0.05 * rng.standard_normal(64)).astype(np.float32),
            "w3": glorot(3, 64), "b3": (0.05 * rng.standard_normal(3)).astype(np.float32)}


def _trainer(x, t, **kw):
    return lbm.Trainer(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(), **kw)


def test_sampler_matches_splitmix64():
    x, t = _data(5003)
    _say("train sampler")
    tr = _trainer(x, t, batch=256, seed=77)
    for step in (0, 1, 9):
        rows = tr.sample_rows(step)
        out = splitmix64.sequence(77, (step + 1) * 256)[step * 256:]
        ref = ((out >> np.uint64(32)) * np.uint64(5003)) >> np.uint64(32)
        np.testing.assert_array_equal(rows, ref.astype(np.int32))


def test_standardisation_matches_numpy():
    x, t = _data(100_001, seed=3)
    _say("train stats")
    tr = _trainer(x, t, batch=64)
    tr.set_weights(_weights(1))
    W = tr.weights()
    np.testing.assert_allclose(W["mu_in"], x.astype(np.float64).mean(0), rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(W["sd_in"], x.astype(np.float64).std(0), rtol=1e-6)
    np.testing.assert_allclose(W["mu_out"], t.astype(np.float64).mean(0), rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(W["sd_out"], t.astype(np.float64).std(0), rtol=1e-6)


def _oracle_params(W, P):
    Q = {k: np.asarray(P[k], np.float64) for k in omlp.PARAM_NAMES}
    for k in ("mu_in", "sd_in", "mu_out", "sd_out"):
        Q[k] = np.asarray(W[k], np.float32)
    return Q


@pytest.mark.parametrize("n_rows", [64, 1024])
def test_gradient_matches_oracle(n_rows):
    x, t = _data(20_000, seed=5)
    P = _weights(2)
    _say("train gradient", n_rows)
    tr = _trainer(x, t, batch=64)
    tr.set_weights(P)
    rows = np.random.default_rng(n_rows).integers(0, 20_000, n_rows).astype(np.int32)
    g, loss = tr.gradient(rows)
    Q = _oracle_params(tr.weights(), P)
    ref_loss, ref = omlp.grad_bf16(x[rows].astype(np.float64), t[rows].astype(np.float64), Q)
    assert abs(loss - ref_loss) < 2e-3 * ref_loss
    G = lbm.unflatten_params(g)
    for k in omlp.PARAM_NAMES:
        err = np.linalg.norm(G[k] - ref[k]) / np.linalg.norm(ref[k])
        print(f"{k}: rel err {err:.2e}", flush=True)
        assert err < 1e-4, k
        assert np.max(np.abs(G[k] - ref[k])) < 1e-3 * np.max(np.abs(ref[k])), k


def test_adam_step_matches_oracle():
    x, t = _data(30_000, seed=6)
    P = _weights(3)
    _say("train adam")
    tr = _trainer(x, t, batch=512, lr=2e-3, seed=9)
    tr.set_weights(P)
    W0 = tr.weights()
    Q = {k: np.asarray(P[k], np.float64) for k in omlp.PARAM_NAMES}
    opt = omlp.Adam(Q, lr=2e-3)
    for step in range(3):
        rows = tr.sample_rows(step)
        g, _ = tr.gradient(rows)            # the gradient the step will use
        tr.step(1)
        opt.step(Q, {k: v.astype(np.float64) for k, v in lbm.unflatten_params(g).items()})
    W = tr.weights()
    for k in omlp.PARAM_NAMES:
        np.testing.assert_allclose(W[k], Q[k], rtol=2e-5, atol=2e-7)
        assert np.max(np.abs(W[k] - W0[k])) > 1e-3      # it moved


def test_training_fits_a_teacher_and_is_reproducible():
    # targets from a fixed random "teacher" network of the same shape
    rng = np.random.default_rng(11)
    x = (0.01 * rng.standard_normal((50_000, 27))).astype(np.float32)
    T = _weights(12, scale=1.5)
    z = x / 0.01
    h = np.tanh(np.tanh(z @ T["w1"].T + T["b1"]) @ T["w2"].T + T["b2"])
    t = (1e-4 * (h @ T["w3"].T + T["b3"])).astype(np.float32)
    _say("train teacher")
    a = _trainer(x, t, batch=1024, lr=3e-3, seed=1)
    b = _trainer(x, t, batch=1024, lr=3e-3, seed=1)
    P = _weights(13)
    a.set_weights(P)
    b.set_weights(P)
    a.step(1)
    first = a.loss()
    a.step(599)
    b.step(600)
    last = a.loss()
    print(f"teacher fit: loss {first:.4f} -> {last:.4f}", flush=True)
    assert last < 0.1 * first
    Wa, Wb = a.weights(), b.weights()
    for k in omlp.PARAM_NAMES:
        np.testing.assert_array_equal(Wa[k], Wb[k])
