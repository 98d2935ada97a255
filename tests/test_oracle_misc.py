"""Pins of the oracle's MLP, optimiser, random generator, observables and
of the geometry input generators."""
import math

import numpy as np
import pytest
import torch
from scipy import integrate

from oracle import mlp, observables, splitmix64
from oracle.solver import Lattice
from paper_2506_05293_amd import geometry


def _params(rng, scale=0.3):
    return {"w1": scale * rng.standard_normal((64, 27)), "b1": 0.1 * rng.standard_normal(64),
            "w2": scale * rng.standard_normal((64, 64)), "b2": 0.1 * rng.standard_normal(64),
            "w3": scale * rng.standard_normal((3, 64)), "b3": 0.1 * rng.standard_normal(3)}


def _torch_net(P):
    net = torch.nn.Sequential(torch.nn.Linear(27, 64), torch.nn.Tanh(),
                              torch.nn.Linear(64, 64), torch.nn.Tanh(),
                              torch.nn.Linear(64, 3)).double()
    with torch.no_grad():
        for lin, (w, b) in zip([net[0], net[2], net[4]], [("w1", "b1"), ("w2", "b2"), ("w3", "b3")]):
            lin.weight.copy_(torch.from_numpy(np.asarray(P[w], np.float64)))
            lin.bias.copy_(torch.from_numpy(np.asarray(P[b], np.float64)))
    return net


def test_bf16_rounding():
    # exactly representable values are kept; halfway cases go to even
    assert mlp.bf16_round(1.0) == 1.0
    assert mlp.bf16_round(1.0 + 2.0**-8) == 1.0            # tie -> even (down)
    assert mlp.bf16_round(1.0 + 3 * 2.0**-8) == 1.0 + 2.0**-6   # tie -> even (up)
    assert mlp.bf16_round(1.0 + 2.0**-8 + 2.0**-20) == 1.0 + 2.0**-7
    x = np.random.default_rng(0).standard_normal(1000)
    r = mlp.bf16_round(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0**-8 * (1 + 1e-6))
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).double().numpy()
    np.testing.assert_array_equal(r, ref)


def test_forward_f64_matches_library_layers():
    rng = np.random.default_rng(1)
    P = _params(rng)
    z = rng.standard_normal((50, 27))
    _, o = mlp.forward_f64(z, P)
    ref = _torch_net(P)(torch.from_numpy(z)).detach().numpy()
    np.testing.assert_allclose(o, ref, rtol=1e-13, atol=1e-14)


def test_forward_bf16_close_to_library_layers():
    rng = np.random.default_rng(2)
    P = _params(rng)
    P.update(mu_in=0.01 * rng.standard_normal(27), sd_in=0.02 + 0.01 * rng.random(27),
             mu_out=0.001 * rng.standard_normal(3), sd_out=0.003 + 0.001 * rng.random(3))
    x = 0.02 * rng.standard_normal((200, 27))
    s = mlp.forward_bf16(x, P)
    z = (x - P["mu_in"]) / P["sd_in"]
    o = _torch_net(P)(torch.from_numpy(z)).detach().numpy()
    ref = o * P["sd_out"] + P["mu_out"]
    # BF16 rounding of inputs, weights and activations: a few 2^-8 relative
    scale = np.abs(o).max() * P["sd_out"].max()
    assert np.max(np.abs(s - ref)) < 0.05 * scale
    assert np.max(np.abs(s - ref)) > 0           # the roundings are really there


def test_gradients_match_finite_differences_and_autograd():
    rng = np.random.default_rng(3)
    P = _params(rng)
    z = rng.standard_normal((16, 27))
    y = rng.standard_normal((16, 3))
    cache, o = mlp.forward_f64(z, P)
    g = mlp.backward_f64(cache, o, y, P)
    h = 1e-6
    for k in mlp.PARAM_NAMES:
        flat = P[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(8, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.mse_loss(mlp.forward_f64(z, P)[1], y)
            flat[idx] = old - h
            lm = mlp.mse_loss(mlp.forward_f64(z, P)[1], y)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[idx]) < 1e-7 * max(1.0, abs(fd))
    net = _torch_net(P)
    loss = torch.nn.functional.mse_loss(net(torch.from_numpy(z)), torch.from_numpy(y))
    loss.backward()
    for lin, (w, b) in zip([net[0], net[2], net[4]], [("w1", "b1"), ("w2", "b2"), ("w3", "b3")]):
        np.testing.assert_allclose(g[w], lin.weight.grad.numpy(), rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(g[b], lin.bias.grad.numpy(), rtol=1e-12, atol=1e-15)


def test_adam_first_step_closed_form_and_library():
    rng = np.random.default_rng(4)
    P = _params(rng)
    g = {k: rng.standard_normal(P[k].shape) for k in mlp.PARAM_NAMES}
    P0 = {k: P[k].copy() for k in mlp.PARAM_NAMES}
    opt = mlp.Adam(P, lr=1e-3)
    opt.step(P, g)
    for k in mlp.PARAM_NAMES:
        np.testing.assert_allclose(P[k] - P0[k], -1e-3 * g[k] / (np.abs(g[k]) + 1e-8),
                                   rtol=1e-12, atol=1e-18)
    # several steps against the library optimiser
    tp = {k: torch.tensor(P0[k], requires_grad=True) for k in mlp.PARAM_NAMES}
    topt = torch.optim.Adam(tp.values(), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    P = {k: P0[k].copy() for k in mlp.PARAM_NAMES}
    opt = mlp.Adam(P, lr=1e-3)
    for it in range(5):
        gi = {k: rng.standard_normal(P[k].shape) for k in mlp.PARAM_NAMES}
        opt.step(P, gi)
        for k in mlp.PARAM_NAMES:
            tp[k].grad = torch.from_numpy(gi[k])
        topt.step()
    for k in mlp.PARAM_NAMES:
        np.testing.assert_allclose(P[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-15)


def test_training_reaches_least_squares_limit():
    # Training only the output layer is a linear least-squares problem in
    # (w3, b3): Adam on the MSE of Eq. 17 must reach the loss of the library
    # least-squares solution.
    rng = np.random.default_rng(5)
    P = _params(rng, 0.2)
    z = rng.standard_normal((256, 27))
    y = rng.standard_normal((256, 3))
    h2 = mlp.forward_f64(z, P)[0][2]
    A = np.hstack([h2, np.ones((256, 1))])
    sol = np.linalg.lstsq(A, y, rcond=None)[0]
    best = mlp.mse_loss(A @ sol, y)
    opt = mlp.Adam(P, lr=1e-2)
    for it in range(4000):
        if it == 3000:
            opt.lr = 1e-3
        cache, o = mlp.forward_f64(z, P)
        g = mlp.backward_f64(cache, o, y, P)
        for k in ("w1", "b1", "w2", "b2"):
            g[k] = np.zeros_like(g[k])
        opt.step(P, g)
    loss = mlp.mse_loss(mlp.forward_f64(z, P)[1], y)
    assert best <= loss < best * (1 + 1e-6)


def test_splitmix64_published_vectors():
    g = splitmix64.SplitMix64(0)
    assert [g.next() for _ in range(4)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                            0x06C45D188009454F, 0xF88BB8A8724C81EC]
    g = splitmix64.SplitMix64(12345)
    seq = [g.next() for _ in range(100)]
    np.testing.assert_array_equal(splitmix64.sequence(12345, 100), np.array(seq, np.uint64))


def test_velocity_noise_layout():
    nx, ny, seed, amp = 7, 5, 99, 1e-4
    nux, nuy = splitmix64.velocity_noise(seed, nx, ny, amp)
    g = splitmix64.SplitMix64(seed)
    for y in range(ny):
        for x in range(nx):
            ox, oy = g.next(), g.next()
            assert nux[y, x] == amp * (2 * ((ox >> 11) * 2.0**-53) - 1)
            assert nuy[y, x] == amp * (2 * ((oy >> 11) * 2.0**-53) - 1)
    assert np.abs(nux).max() <= amp


def test_strouhal_of_synthetic_signal():
    rng = np.random.default_rng(6)
    f0, D, U = 0.00123, 80.0, 0.05
    t = np.arange(20000)
    cl = 0.7 * np.sin(2 * np.pi * f0 * t + 0.3) + 0.05 + 0.01 * rng.standard_normal(t.size)
    st = observables.strouhal(cl, D, U)
    assert abs(st / (f0 * D / U) - 1) < 1e-3
    assert abs(observables.zero_crossing_frequency(cl) / f0 - 1) < 1e-2


def test_force_coefficients_eq13():
    cd, cl = observables.force_coefficients(0.01, -0.002, 1.0, 0.05, 20.0)
    assert abs(cd - 2 * 0.01 / (0.05**2 * 20)) < 1e-15 and abs(cl + 0.4 * 0.2) < 1e-15


def test_cylinder_mask():
    m = geometry.cylinder(101, 101, 50, 50, 20.0)
    assert m.sum() == 317                    # lattice points with r^2 <= 100
    assert np.array_equal(m, m[::-1, :]) and np.array_equal(m, m[:, ::-1])
    m80 = geometry.cylinder(200, 200, 100, 100, 80.0)
    assert abs(m80.sum() - math.pi * 40**2) < 2 * math.pi * 40 * 0.1


def test_naca0012_mask():
    yt = geometry.naca0012_half_thickness
    assert abs(yt(1.0)) < 1e-15              # closed trailing edge
    s = np.linspace(0, 1, 200001)
    k = np.argmax(yt(s))
    # the closed-edge coefficients give 0.11897 c, "12%" in the appendix
    assert abs(2 * yt(s[k]) - 0.12) < 1.5e-3 and 0.28 < s[k] < 0.32
    area = integrate.quad(lambda x: 2 * yt(x), 0, 1, limit=200)[0]
    c = 256
    for aoa in (0.0, 4.0, 8.0):
        m = geometry.naca0012(1400, 600, c, aoa, (600.0, 300.0))
        perim = 2.05 * c
        assert abs(m.sum() - area * c * c) < 0.1 * perim, (aoa, m.sum(), area * c * c)
    m0 = geometry.naca0012(1400, 601, c, 0.0, (600.0, 300.0))
    assert np.array_equal(m0, m0[::-1, :])   # symmetric section at zero incidence
    # positive incidence lifts the nose: leading edge above the pivot line
    m8 = geometry.naca0012(1400, 600, c, 8.0, (600.0, 300.0))
    ys, xs = np.nonzero(m8)
    assert ys[np.argmin(xs)] > 300 and ys[np.argmax(xs)] < 300


def test_oracle_default_init_uses_the_noise():
    mask = geometry.cylinder(20, 10, 6, 5, 4.0)
    lat = Lattice(mask, 0.6, u_in=0.05, noise_amp=1e-4, seed=3)
    rho, ux, uy = lat.macroscopic()
    nux, nuy = splitmix64.velocity_noise(3, 20, 10, 1e-4)
    fl = mask == 0
    np.testing.assert_allclose(rho[fl], 1.0, rtol=1e-15)
    np.testing.assert_allclose(ux[fl], 0.05 + nux[fl], atol=1e-16)
    np.testing.assert_allclose(uy[fl], nuy[fl], atol=1e-16)
    assert np.all(ux[~fl] == 0)


def test_bf16_gradient_reduces_to_chain_rule(monkeypatch):
    # with the roundings taken out, the MFMA-emulating gradient is the plain
    # FP64 chain rule (itself pinned to autograd above); with them it stays
    # within BF16 accuracy of it
    rng = np.random.default_rng(8)
    P = _params(rng, 0.3)
    P.update(mu_in=0.01 * rng.standard_normal(27), sd_in=0.02 + 0.01 * rng.random(27),
             mu_out=1e-4 * rng.standard_normal(3), sd_out=1e-3 * (1 + rng.random(3)))
    x = 0.02 * rng.standard_normal((128, 27))
    t = 1e-3 * rng.standard_normal((128, 3))
    loss_b, gb = mlp.grad_bf16(x, t, P)
    z = (x - P["mu_in"]) / P["sd_in"]
    y = (t - P["mu_out"]) / P["sd_out"]
    cache, o = mlp.forward_f64(z, P)
    ref = mlp.backward_f64(cache, o, y, P)
    for k in mlp.PARAM_NAMES:
        assert np.linalg.norm(gb[k] - ref[k]) < 0.03 * np.linalg.norm(ref[k]), k
    monkeypatch.setattr(mlp, "bf16_round", lambda v: np.asarray(v, np.float64))
    monkeypatch.setattr(mlp, "standardise_f32",
                        lambda v, mu, sd: (np.asarray(v, np.float64) - mu) / sd)
    loss_e, ge = mlp.grad_bf16(x, t, P)
    assert abs(loss_e - mlp.mse_loss(o, y)) < 1e-12 * loss_e
    for k in mlp.PARAM_NAMES:
        np.testing.assert_allclose(ge[k], ref[k], rtol=1e-10, atol=1e-14)


def test_product_observables_agree_with_oracle():
    # the library's host-side observables (a different peak refinement) and
    # the oracle's recover the same synthetic Strouhal number and coefficients
    from paper_2506_05293_amd import observables as pobs
    rng = np.random.default_rng(9)
    f0, D, U = 0.000911, 80.0, 0.05
    t = np.arange(30000)
    cl = 0.4 * np.sin(2 * np.pi * f0 * t) + 0.02 * rng.standard_normal(t.size)
    fx = np.full(t.size, 0.3) * 0.5 * U * U * D
    fy = cl * 0.5 * U * U * D
    s = pobs.summarize(fx, fy, U, D, window=1.0)
    assert abs(s["st"] / (f0 * D / U) - 1) < 1e-3
    assert abs(s["st"] / observables.strouhal(cl, D, U) - 1) < 1e-3
    assert abs(s["cd_mean"] - 0.3) < 1e-12
    assert abs(s["cl_rms"] - 0.4 / np.sqrt(2)) < 5e-3
    cd, cl2 = observables.force_coefficients(fx, fy, 1.0, U, D)
    np.testing.assert_allclose(cl2, cl, rtol=1e-12)


def test_naca_coefficients_are_the_printed_ones():
    # the mask generator uses the coefficients of Eq. A.1 as printed, and the
    # printed law has the properties of a closed-trailing-edge NACA0012:
    # zero thickness at x = 1 (to the 9 printed digits) and a maximum
    # thickness of nominally 12 % of the chord near 30 % chord (the printed
    # closed-edge form gives 11.897 %)
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "naca0012_eq_a1.json")) as fh:
        g = json.load(fh)
    printed = tuple(g[k] for k in ("a0", "a1", "a2", "a3", "a4", "a5"))
    assert geometry.NACA0012_COEF == printed
    a0, a1, a2, a3, a4, a5 = printed
    s = np.linspace(0.0, 1.0, 1000001)
    y = a0 * (a1 * np.sqrt(s) + a2 * s + a3 * s**2 + a4 * s**3 + a5 * s**4)
    assert abs(y[-1]) < 1e-9
    k = np.argmax(y)
    assert abs(2 * y[k] - 0.12) < 1.5e-3
    assert 0.28 < s[k] < 0.32
