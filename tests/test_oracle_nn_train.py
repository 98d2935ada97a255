"""Pins of the oracle's closed-loop training of the Eq. 16 reconstruction
network (Sec. 3.1 network, Sec. 4.2 training procedure).

The torch re-expression of the step is fixed to the numpy solver's Eq. 16
outlet (with the solver's network evaluated in FP64 instead of its BF16
inference form, and no fallback); its reverse-mode gradient to central
finite differences of the numpy solver's loss (Richardson-extrapolated);
a zero output layer to exactly zero hidden-layer gradients and to the copy
outflow; and the dependence cone (2 n_t columns; the trainer's strip holds
2 n_t + 3) to exact invariance under changes further upstream."""
import numpy as np
import pytest
import torch

import oracle.solver as solver_mod
from oracle import d2q9, mlp, nn_train
from oracle.d2q9 import CS2
from oracle.solver import Lattice

CS = np.sqrt(CS2)
NX, NY, TAU, U0 = 40, 22, 0.6, 0.1
CFG = dict(tau=TAU, u_in=U0)


def _net(seed, out_scale=1.0):
    rng = np.random.default_rng(seed)
    return {"w1": 0.5 * rng.standard_normal((20, 9)), "b1": 0.3 * rng.standard_normal(20),
            "w2": 0.3 * rng.standard_normal((20, 20)), "b2": 0.3 * rng.standard_normal(20),
            "w3": 0.5 * out_scale * rng.standard_normal((3, 20)),
            "b3": 0.3 * out_scale * rng.standard_normal(3),
            "mu_in": 1e-3 * rng.standard_normal(9), "sd_in": np.full(9, 2e-2),
            "mu_out": 1e-4 * rng.standard_normal(3), "sd_out": np.full(3, 1e-3)}


def _f64_forward(x, P):
    """The solver's network in FP64 (no BF16 roundings)."""
    z = (np.asarray(x, np.float64) - P["mu_in"]) / P["sd_in"]
    _, o = mlp.forward_f64(z, P)
    return o * P["sd_out"] + P["mu_out"]


@pytest.fixture(autouse=True)
def _fp64_network(monkeypatch):
    monkeypatch.setattr(solver_mod, "forward_bf16", _f64_forward)


def _solver(net):
    lat = Lattice(np.zeros((NY, NX), np.uint8), TAU, lateral="periodic", u_in=U0)
    if net is not None:
        lat.set_outflow_nn(net, mass_bound=1e9)
    return lat


def _state(seed=0, steps=6):
    """A post-collision state with a vortex at the outlet (numpy solver,
    Zou & He outlet)."""
    y, x = np.mgrid[0:NY, 0:NX].astype(float)
    xc, yc, rc, b = NX - 6.5 + 0.3 * seed, NY / 2 - 0.4, 4.0, 0.4
    r2 = (x - xc) ** 2 + (y - yc) ** 2
    e = np.exp(-r2 / (2 * rc**2))
    lat = _solver(None)
    lat.set_equilibrium(np.exp(-(b * U0) ** 2 / (2 * CS2) * np.exp(-r2 / rc**2)),
                        U0 - b * U0 * (y - yc) / rc * e, b * U0 * (x - xc) / rc * e)
    lat.step(steps)
    return lat.post_collision()


def _ref(a0, n_t):
    """Reference moments: the same state advanced with the Zou & He outlet."""
    lat = _solver(None)
    a = a0
    for _ in range(n_t):
        a, _ = lat.advance_post(a)
    return np.stack(d2q9.moments(a[:, :, -n_t:]))


def _np_loss(segments, net):
    tot = 0.0
    for a0, ref in segments:
        n_t = ref.shape[2]
        lat = _solver(net)
        a = a0
        for _ in range(n_t):
            a, _ = lat.advance_post(a)
        assert lat.n_fallback == 0
        rho, u, v = d2q9.moments(a[:, :, -n_t:])
        tot += np.mean((rho - ref[0]) ** 2) + np.mean((u - ref[1]) ** 2 + (v - ref[2]) ** 2)
    return tot / len(segments)


@pytest.mark.parametrize("n_t", [1, 4, 7])
def test_rollout_matches_numpy_solver(n_t):
    net = _net(1)
    a0 = _state()
    states = nn_train.rollout(a0, nn_train._theta(net, False), net, CFG, n_t)
    lat = _solver(net)
    a = a0
    for k in range(n_t):
        a, _ = lat.advance_post(a)
        err = np.max(np.abs(states[k + 1].detach().numpy() - a))
        assert err < 1e-14, (k, err)
    assert lat.n_fallback == 0


def test_gradient_matches_finite_differences():
    net = _net(2)
    segs = [(_state(0), _ref(_state(0), 5)), (_state(1, 4), _ref(_state(1, 4), 3))]
    loss, g = nn_train.loss_and_grad(segs, net, CFG)
    assert loss == pytest.approx(_np_loss(segs, net), rel=1e-12)
    rng = np.random.default_rng(9)
    for trial in range(3):
        d = {k: rng.standard_normal(np.shape(net[k])) for k in nn_train.PARAMS}
        ana = sum(float(np.sum(g[k] * d[k])) for k in nn_train.PARAMS)

        def at(eps):
            p = dict(net)
            for k in nn_train.PARAMS:
                p[k] = np.asarray(net[k]) + eps * d[k]
            return _np_loss(segs, p)
        h = 2e-3
        c1 = (at(h) - at(-h)) / (2 * h)
        c2 = (at(h / 2) - at(-h / 2)) / h
        fd = (4 * c2 - c1) / 3                      # Richardson: O(h^4)
        assert abs(fd - ana) <= 1e-6 * abs(ana) + 1e-22, (trial, fd, ana)


def test_zero_output_layer_gives_the_copy_outflow_and_no_hidden_gradient():
    net = _net(3)
    net["w3"] = np.zeros((3, 20))
    net["b3"] = np.zeros(3)
    net["mu_out"] = np.zeros(3)
    a0 = _state()
    # s = 0: the unknowns are the streamed values of column L-1, the rest of
    # the outlet column is its own streamed values
    f = nn_train.stream(torch.as_tensor(a0))
    g = nn_train.outlet(f[:, :, -1], f[:, :, -2], nn_train._theta(net, False), net).numpy()
    fn = f.numpy()
    for q in range(9):
        want = fn[q, :, -2] if q in (3, 6, 7) else fn[q, :, -1]
        np.testing.assert_array_equal(g[q], want)
    segs = [(a0, _ref(a0, 4))]
    _, grad = nn_train.loss_and_grad(segs, net, CFG)
    for k in ("w1", "b1", "w2", "b2"):
        assert np.all(grad[k] == 0.0), k
    assert np.any(grad["w3"] != 0.0) and np.any(grad["b3"] != 0.0)


@pytest.mark.parametrize("n_t", [2, 5])
def test_state_beyond_the_cone_does_not_matter(n_t):
    net = _net(4)
    a0 = _state(2)
    ref = _ref(a0, n_t)
    loss, g = nn_train.loss_and_grad([(a0, ref)], net, CFG)
    # this outlet reads the streamed column L-1 (columns L-2..L of the state
    # before), so A_{n_t} over the last n_t columns depends on A_0 from
    # column NX - 2 n_t on; the trainer's strip of 2 n_t + 3 columns holds it
    b0 = a0.copy()
    cut = NX - 2 * n_t
    rng = np.random.default_rng(5)
    b0[:, :, :cut] *= 1.0 + 1e-3 * rng.standard_normal(b0[:, :, :cut].shape)
    loss_b, g_b = nn_train.loss_and_grad([(b0, ref)], net, CFG)
    assert loss_b == loss
    for k in nn_train.PARAMS:
        np.testing.assert_array_equal(g_b[k], g[k])
    # and the first column of the cone does matter
    c0 = a0.copy()
    c0[:, :, cut] *= 1.0 + 1e-3
    assert nn_train.loss_only([(c0, ref)], net, CFG) != loss


def test_loss_only_and_final_state_agree_with_the_rollout():
    net = _net(6)
    a0 = _state(3)
    ref = _ref(a0, 4)
    loss, _ = nn_train.loss_and_grad([(a0, ref)], net, CFG)
    assert nn_train.loss_only([(a0, ref)], net, CFG) == pytest.approx(loss, rel=1e-14)
    fin = nn_train.final_state(a0, net, CFG, 4)
    rho, u, v = d2q9.moments(fin[:, :, -4:])
    direct = np.mean((rho - ref[0]) ** 2) + np.mean((u - ref[1]) ** 2 + (v - ref[2]) ** 2)
    assert direct == pytest.approx(loss, rel=1e-12)
