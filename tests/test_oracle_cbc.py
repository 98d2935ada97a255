"""Pins of the oracle's characteristic outflow (Sec. 4, Eqs. 18-29).

Each test fixes a part by something other than the code itself: exactness of
the difference stencils on quadratics, the equilibrium fixed point, the
closed-form relaxation of a uniform state towards the far-field pressure
(Eqs. 18-19 and 27-28 with every gradient zero), the exact moments of the
reconstructed node, the defining property of the method (a plane acoustic
pulse leaves without reflection, where the Zou & He pressure outlet reflects
it), and the reduction of the tuning network to fixed parameters."""
import numpy as np
import pytest

from oracle import cbc, d2q9
from oracle.d2q9 import C, CS2
from oracle.solver import Lattice

CS = np.sqrt(CS2)


def test_difference_stencils_exact_on_quadratics():
    x = np.array([7.0, 8.0, 9.0])                     # columns L-2, L-1, L
    phi = 0.3 * x**2 - 1.1 * x + 2.0
    assert cbc.x_derivative(*phi) == pytest.approx(0.6 * 9.0 - 1.1, abs=1e-12)
    y = np.arange(12.0)
    q = 0.2 * y**2 + 0.5 * y - 1.0
    np.testing.assert_allclose(cbc.y_derivative(q, periodic=False), 0.4 * y + 0.5, atol=1e-12)
    s = np.sin(2 * np.pi * y / 12)
    d = cbc.y_derivative(s, periodic=True)
    np.testing.assert_allclose(d, np.sin(2 * np.pi / 12) * np.cos(2 * np.pi * y / 12), atol=1e-12)


def _uniform_col(rho, u, v, n):
    return d2q9.equilibrium(np.full(n, rho), np.full(n, u), np.full(n, v))


def test_uniform_far_field_state_is_a_fixed_point():
    nx, ny, u0 = 40, 12, 0.08
    lat = Lattice(np.zeros((ny, nx), np.uint8), 0.6, lateral="periodic", u_in=u0)
    lat.set_outflow_cbc(sigma=0.7, kappa2=0.3, mach=u0 / CS, length=nx)
    f0 = lat.f.copy()
    lat.step(60)
    np.testing.assert_allclose(lat.f, f0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("sigma,kappa2", [(0.0, 0.0), (0.4, 0.2), (1.0, 0.3)])
def test_uniform_state_relaxes_towards_far_field_in_closed_form(sigma, kappa2):
    # every gradient zero: L_5 = L_3 = T = 0 and L_1 = kappa_1 c_s^2 (rho - rho_inf),
    # so rho' = rho - kappa_1 (rho - rho_inf) / 2 and
    # u' = u + kappa_1 c_s (rho - rho_inf) / (2 rho), v' = v
    ny, rho, u, v, mach, length, rho_inf = 6, 1.02, 0.06, 0.01, 0.2, 50.0, 1.0
    col = _uniform_col(rho, u, v, ny)
    rho3 = np.full((3, ny), rho)
    u3 = np.full((3, ny), u)
    v3 = np.full((3, ny), v)
    params = dict(sigma=sigma, kappa2=kappa2, mach=mach, length=length, rho_inf=rho_inf)
    g, dt = cbc.outlet(col, rho3, u3, v3, np.zeros((ny, 3)), params, periodic=True)
    k1 = sigma * (1 - mach**2) * CS / length
    rho1 = rho - k1 * (rho - rho_inf) / 2
    u1 = u + k1 * CS * (rho - rho_inf) / (2 * rho)
    # the reconstructed node carries exactly the prescribed state
    np.testing.assert_allclose(g.sum(0), rho1, rtol=1e-15)
    np.testing.assert_allclose((C[:, 0, None] * g).sum(0), rho1 * u1, rtol=1e-14)
    np.testing.assert_allclose((C[:, 1, None] * g).sum(0), rho1 * v, rtol=1e-13)
    # only f_0 and the unknowns change
    for q in (1, 2, 4, 5, 8):
        np.testing.assert_array_equal(g[q], col[q])
    np.testing.assert_allclose(dt[:, 0], -CS2 * k1 * (rho - rho_inf) / 2, rtol=1e-12, atol=1e-20)


def test_reconstruction_moments_for_random_states():
    rng = np.random.default_rng(4)
    ny = 16
    rho3 = 1 + 0.01 * rng.standard_normal((3, ny))
    u3 = 0.1 + 0.01 * rng.standard_normal((3, ny))
    v3 = 0.01 * rng.standard_normal((3, ny))
    col = d2q9.equilibrium(rho3[2], u3[2], v3[2]) + 1e-4 * rng.standard_normal((9, ny))
    params = dict(sigma=0.3, kappa2=0.25, mach=0.3, length=200.0, rho_inf=1.0)
    g, dt = cbc.outlet(col, rho3, u3, v3, np.zeros((ny, 3)), params, periodic=False)
    rho1 = rho3[2] + dt[:, 0] / CS2
    u1 = u3[2] + dt[:, 1]
    v1 = v3[2] + dt[:, 2]
    np.testing.assert_allclose(g.sum(0), rho1, rtol=1e-14)
    np.testing.assert_allclose((C[:, 0, None] * g).sum(0), rho1 * u1, rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose((C[:, 1, None] * g).sum(0), rho1 * v1, rtol=1e-12, atol=1e-16)


def _pulse(outflow):
    """A right-going plane acoustic pulse in a y-periodic channel at rest."""
    nx, ny, amp, x0, w = 160, 4, 2e-3, 80.0, 6.0
    lat = Lattice(np.zeros((ny, nx), np.uint8), 0.52, lateral="periodic", u_in=0.0)
    x = np.arange(nx)[None, :].repeat(ny, 0).astype(float)
    drho = amp * np.exp(-0.5 * ((x - x0) / w) ** 2)
    lat.set_equilibrium(1 + drho, CS * drho, np.zeros_like(drho))   # Riemann invariant: right-going
    if outflow == "cbc":
        lat.set_outflow_cbc(sigma=0.0, kappa2=0.0, mach=0.0, length=nx)
    steps = int((nx - x0 + 4 * w) / CS) + 20
    lat.step(steps)
    rho, _, _ = lat.macroscopic()
    return np.abs(rho - 1).max() / amp


def test_plane_pulse_leaves_without_reflection():
    # L_1 = 0 for a plane wave leaving through the outlet: no incoming wave;
    # the Zou & He pressure outlet (rho fixed) sends it back inverted
    r_cbc, r_zh = _pulse("cbc"), _pulse("zouhe")
    assert r_cbc < 0.05, r_cbc
    assert r_zh > 0.5, r_zh


def _net(seed=0, zero=False):
    rng = np.random.default_rng(seed)
    s = 0.0 if zero else 1.0
    return {"w1": s * rng.standard_normal((20, 9)), "b1": s * rng.standard_normal(20),
            "w2": s * rng.standard_normal((20, 20)) / 4, "b2": s * rng.standard_normal(20),
            "w3": s * rng.standard_normal((2, 20)) / 4, "b3": np.zeros(2),
            "mu_in": np.zeros(9), "sd_in": np.full(9, 1e-3), "leaky_slope": 0.01,
            "sigma_scale": 1.0, "sigma_shift": 0.0, "kappa_scale": 0.5, "kappa_shift": 0.1}


def _vortex_lattice(nx=60, ny=40, u0=0.1):
    lat = Lattice(np.zeros((ny, nx), np.uint8), 0.6, lateral="periodic", u_in=u0)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    r2 = (x - 45) ** 2 + (y - 20) ** 2
    e = np.exp(-r2 / (2 * 6.0**2))
    ux = u0 - 0.3 * u0 * (y - 20) / 6.0 * e
    uy = 0.3 * u0 * (x - 45) / 6.0 * e
    rho = np.exp(-(0.3 * u0) ** 2 / (2 * CS2) * np.exp(-r2 / 6.0**2))
    lat.set_equilibrium(rho, ux, uy)
    return lat


def test_constant_network_equals_fixed_parameters():
    # zero weights: sigma = sigma_scale * sigmoid(b3_0) + shift, likewise kappa_2
    net = _net(zero=True)
    net["b3"] = np.array([np.log(0.3 / 0.7), np.log(0.6 / 0.4)])     # sigmoid -> 0.3, 0.6
    a = _vortex_lattice()
    b = _vortex_lattice()
    a.set_outflow_cbc(net=net, mach=0.1 / CS, length=60)
    b.set_outflow_cbc(sigma=0.3, kappa2=0.5 * 0.6 + 0.1, mach=0.1 / CS, length=60)
    a.step(40)
    b.step(40)
    np.testing.assert_allclose(a.f, b.f, rtol=0, atol=1e-14)


def test_network_reads_features_in_stated_order():
    # a network that passes feature k through both LeakyReLU layers to s_0:
    # sigma = sigmoid(leaky(leaky(z_k))) with sigma_scale 1, shift 0
    rng = np.random.default_rng(1)
    feats = rng.standard_normal((50, 9)) * 1e-3
    for k in range(9):
        net = _net(zero=True)
        net["w1"][3, k] = 1.0
        net["w2"][7, 3] = 1.0
        net["w3"][0, 7] = 1.0
        sigma, kappa2 = cbc.network(feats, net)
        z = feats[:, k] / 1e-3
        h = np.where(z > 0, z, 0.01 * z)
        h = np.where(h > 0, h, 0.01 * h)
        np.testing.assert_allclose(sigma, 1 / (1 + np.exp(-h)), rtol=1e-14)
        np.testing.assert_allclose(kappa2, 0.5 * 0.5 + 0.1, rtol=1e-14)


def test_network_features_are_gradients_and_previous_time_derivatives():
    # the CBC hands the network (p_x, u_x, v_x, p_y, u_y, v_y, p_t, u_t, v_t)
    # with the time derivatives of the previous step
    lat = _vortex_lattice()
    seen = []
    orig = cbc.network

    def spy(features, P):
        seen.append(np.array(features))
        return orig(features, P)
    cbc.network = spy
    try:
        lat.set_outflow_cbc(net=_net(3), mach=0.1 / CS, length=60)
        lat.step(1)
        prev = lat.cbc_prev.copy()
        fstar = lat.collide()
        rho, ux, uy = d2q9.moments(fstar[:, :, -3:])
        lat.step(1)
    finally:
        cbc.network = orig
    g = cbc.gradients(rho.T, ux.T, uy.T, True)
    np.testing.assert_allclose(seen[1][:, :6], np.stack(g, axis=1), rtol=1e-12, atol=1e-18)
    np.testing.assert_array_equal(seen[1][:, 6:], prev)
    np.testing.assert_array_equal(seen[0][:, 6:], 0.0)


def test_walls_are_rejected():
    lat = Lattice(np.zeros((10, 30), np.uint8), 0.6, lateral="walls", u_in=0.05)
    with pytest.raises(ValueError):
        lat.set_outflow_cbc(sigma=0.2, kappa2=0.1, mach=0.1, length=30)
