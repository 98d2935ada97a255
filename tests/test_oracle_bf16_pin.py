"""Pin of the BF16 rounding points of the oracle's MFMA-emulating network
passes (``oracle.mlp.forward_bf16``, ``grad_bf16``; Sec. 3.1 Eq. 16 and the
Eq. 17 loss) against a worked single-path example.

tests/golden/bf16_single_path.json holds every intermediate value of a
1-1-1-3 network on 16 samples, derived in scalar arithmetic by
tests/golden/make_bf16_single_path.py (FP32 through numpy.float32, BF16
through torch's conversion, tanh from math; no oracle code).  The example
is chosen so that dropping, adding or moving any one rounding point changes
some output or gradient entry by >= 5.9e-8 relative; the oracle must match
to 1e-12."""
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import mlp

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bf16_single_path.json")
TOL = 1e-12


@pytest.fixture(scope="module")
def fx():
    with open(GOLDEN) as f:
        return json.load(f)


def _bf16(v):
    return float(torch.tensor(np.float32(v)).to(torch.bfloat16).float())


def _params(fx):
    # the network as the library holds it: every value rounded to FP32 (the
    # lbm_mlp arrays are float), which is the form the oracle is given
    P = fx["P"]
    return {k: np.asarray(v, np.float32).astype(np.float64) for k, v in _raw(P).items()}


def _raw(P):
    return {"w1": np.array([[P["w1"]]]), "b1": np.array([P["b1"]]),
            "w2": np.array([[P["w2"]]]), "b2": np.array([P["b2"]]),
            "w3": np.array([[P["w3"]], [0.0], [0.0]]), "b3": np.array(P["b3"]),
            "mu_in": np.array([P["mu_in"]]), "sd_in": np.array([P["sd_in"]]),
            "mu_out": np.array(P["mu_out"]), "sd_out": np.array(P["sd_out"])}


def test_fixture_chain_is_consistent(fx):
    # every stored intermediate follows from the previous ones by one FP32
    # operation, one BF16 rounding or one tanh: the example checks by hand
    P = fx["P"]
    for x, r in zip(fx["x"], fx["rows"]):
        z32 = np.float32(x) - np.float32(P["mu_in"])
        assert r["z32"] == float(z32 * (np.float32(1.0) / np.float32(P["sd_in"])))
        assert r["zb"] == _bf16(r["z32"])
        assert (r["W1"], r["W2"], r["W3"]) == (_bf16(P["w1"]), _bf16(P["w2"]), _bf16(P["w3"]))
        assert r["a1"] == r["W1"] * r["zb"] + r["b1"] and r["h1"] == math.tanh(r["a1"])
        assert r["h1b"] == _bf16(r["h1"])
        assert r["a2"] == r["W2"] * r["h1b"] + r["b2"] and r["h2"] == math.tanh(r["a2"])
        assert r["h2b"] == _bf16(r["h2"])
        assert r["o"][0] == r["W3"] * r["h2b"] + r["b3"][0]
    # the first sample sits on a BF16 tie in FP32 and below it in FP64
    r0 = fx["rows"][0]
    assert r0["zb"] == 1 + 2.0**-6 and _bf16((fx["x"][0] - P["mu_in"]) / P["sd_in"]) == 1 + 2.0**-7


def test_forward_bf16_rounding_points(fx):
    P = _params(fx)
    x = np.array(fx["x"])[:, None]
    s = mlp.forward_bf16(x, P)
    ref = np.array(fx["s"])
    np.testing.assert_allclose(s, ref, rtol=TOL, atol=0)
    # every plausible misplacement of a rounding is resolved by the tolerance
    for name, m in fx["forward_mistakes"].items():
        if m["max_rel_change"] > 0:
            assert np.max(np.abs(np.array(m["s0"]) - s[:, 0]) / np.abs(s[:, 0])) > 1e3 * TOL, name


def test_grad_bf16_rounding_points(fx):
    P = _params(fx)
    x = np.array(fx["x"])[:, None]
    t = np.array(fx["t"])
    loss, g = mlp.grad_bf16(x, t, P)
    ref = fx["grad"]
    assert abs(loss - fx["loss"]) <= TOL * fx["loss"]
    for k in ("w1", "w2", "b1", "b2"):
        assert abs(float(np.ravel(g[k])[0]) - ref[k]) <= TOL * abs(ref[k]), k
    np.testing.assert_allclose(np.ravel(g["w3"]), ref["w3"], rtol=TOL, atol=0)
    np.testing.assert_allclose(g["b3"], ref["b3"], rtol=TOL, atol=0)
    got = [loss, float(np.ravel(g["w1"])[0]), float(np.ravel(g["w2"])[0]),
           float(np.ravel(g["b1"])[0]), float(np.ravel(g["b2"])[0])] + list(np.ravel(g["w3"])) \
        + list(g["b3"])
    for name, m in fx["gradient_mistakes"].items():
        gm = m["grad"]
        alt = [m["loss"], gm["w1"], gm["w2"], gm["b1"], gm["b2"]] + gm["w3"] + gm["b3"]
        assert max(abs(a - b) / abs(b) for a, b in zip(alt, got)) > 1e3 * TOL, name


def _skip_call(k):
    """bf16_round with its k-th call (0-based) left out: a rounding point
    planted wrong in the oracle."""
    calls = {"n": 0}
    orig = mlp.bf16_round

    def wrapped(v):
        i = calls["n"]
        calls["n"] += 1
        return np.asarray(v, np.float64) if i == k else orig(v)
    return wrapped


@pytest.mark.parametrize("k", range(6))
def test_the_pin_catches_a_dropped_forward_rounding(fx, k, monkeypatch):
    # forward_bf16 rounds z, W1, h1, W2, h2, W3: leaving out any one of them
    # must break the pin
    monkeypatch.setattr(mlp, "bf16_round", _skip_call(k))
    s = mlp.forward_bf16(np.array(fx["x"])[:, None], _params(fx))
    assert np.max(np.abs(s - np.array(fx["s"])) / np.abs(np.array(fx["s"]))) > 1e3 * TOL


@pytest.mark.parametrize("k", range(10))
def test_the_pin_catches_a_dropped_gradient_rounding(fx, k, monkeypatch):
    # grad_bf16 rounds z, W1, W2, W3, h1, h2, d_o (for dW3), dz2 (for dW2),
    # dz2 (for dz1), dz1 (for dW1): leaving out any one of them must break it
    monkeypatch.setattr(mlp, "bf16_round", _skip_call(k))
    loss, g = mlp.grad_bf16(np.array(fx["x"])[:, None], np.array(fx["t"]), _params(fx))
    ref = fx["grad"]
    got = [loss] + [float(np.ravel(g[n])[0]) for n in ("w1", "w2", "b1", "b2")] \
        + list(np.ravel(g["w3"])) + list(g["b3"])
    want = [fx["loss"]] + [ref[n] for n in ("w1", "w2", "b1", "b2")] + ref["w3"] + ref["b3"]
    assert max(abs(a - b) / abs(b) for a, b in zip(got, want)) > 1e3 * TOL
