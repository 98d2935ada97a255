"""Pins of the oracle's lattice core, collision and Zou & He columns against
closed forms and identities that the paper and the mathematics fix."""
import numpy as np
import pytest

from oracle import d2q9, zouhe
from oracle.d2q9 import C, OPP, W


def _rand_state(rng, shape, amp=0.02):
    rho = 1.0 + 0.05 * rng.standard_normal(shape)
    ux = 0.08 * rng.standard_normal(shape)
    uy = 0.08 * rng.standard_normal(shape)
    f = d2q9.equilibrium(rho, ux, uy)
    f = f * (1.0 + amp * rng.standard_normal(f.shape))   # non-equilibrium part
    return f


def test_lattice_symmetries():
    # weights: zeroth, second and fourth order isotropy of D2Q9 (cs^2 = 1/3)
    assert abs(W.sum() - 1.0) < 1e-16
    cx, cy = C[:, 0].astype(float), C[:, 1].astype(float)
    assert abs((W * cx).sum()) < 1e-16 and abs((W * cy).sum()) < 1e-16
    assert abs((W * cx * cx).sum() - 1 / 3) < 1e-16
    assert abs((W * cx * cy).sum()) < 1e-16
    assert abs((W * cx**4).sum() - 1 / 3) < 1e-16
    assert abs((W * cx**2 * cy**2).sum() - 1 / 9) < 1e-16
    assert np.all(C[OPP] == -C)
    # unknowns at a right boundary are the directions with c_x = -1 (Sec. 2.2)
    assert set(np.nonzero(C[:, 0] == -1)[0]) == {3, 6, 7}
    assert set(np.nonzero(C[:, 0] == 1)[0]) == {1, 5, 8}


def test_equilibrium_closed_moments():
    rng = np.random.default_rng(0)
    rho = 1 + 0.1 * rng.random(50)
    ux, uy = 0.1 * rng.standard_normal(50), 0.1 * rng.standard_normal(50)
    feq = d2q9.equilibrium(rho, ux, uy)
    cx, cy = C[:, 0, None].astype(float), C[:, 1, None].astype(float)
    np.testing.assert_allclose(feq.sum(0), rho, rtol=1e-15)
    np.testing.assert_allclose((cx * feq).sum(0), rho * ux, atol=1e-16)
    np.testing.assert_allclose((cy * feq).sum(0), rho * uy, atol=1e-16)
    # second moment: rho cs^2 delta_ab + rho u_a u_b
    np.testing.assert_allclose((cx * cx * feq).sum(0), rho / 3 + rho * ux * ux, rtol=1e-15)
    np.testing.assert_allclose((cy * cy * feq).sum(0), rho / 3 + rho * uy * uy, rtol=1e-15)
    np.testing.assert_allclose((cx * cy * feq).sum(0), rho * ux * uy, atol=1e-16)
    # at rest it is the weights times rho
    np.testing.assert_allclose(d2q9.equilibrium(2.0, 0.0, 0.0), 2 * W, rtol=1e-16)


@pytest.mark.parametrize("kind", ["bgk", "mrt"])
def test_collision_conserves_mass_momentum(kind):
    rng = np.random.default_rng(1)
    f = _rand_state(rng, (8, 8))
    fs = d2q9.bgk_collide(f, 0.56) if kind == "bgk" else d2q9.mrt_collide(f, 0.56)
    cx, cy = C[:, 0, None, None].astype(float), C[:, 1, None, None].astype(float)
    np.testing.assert_allclose(fs.sum(0), f.sum(0), rtol=1e-13, atol=0)
    assert np.max(np.abs((cx * fs).sum(0) - (cx * f).sum(0))) < 1e-13
    assert np.max(np.abs((cy * fs).sum(0) - (cy * f).sum(0))) < 1e-13
    assert not np.allclose(fs, f)        # it does relax something


def test_bgk_tau_one_is_equilibrium():
    rng = np.random.default_rng(2)
    f = _rand_state(rng, (5, 7))
    np.testing.assert_allclose(d2q9.bgk_collide(f, 1.0),
                               d2q9.equilibrium(*d2q9.moments(f)), rtol=1e-14)


def test_mrt_equal_rates_is_bgk():
    rng = np.random.default_rng(3)
    f = _rand_state(rng, (6, 5))
    tau = 0.61
    s = 1.0 / tau
    np.testing.assert_allclose(d2q9.mrt_collide(f, tau, s, s, s),
                               d2q9.bgk_collide(f, tau), rtol=1e-13, atol=1e-16)


def test_mrt_basis_and_equilibrium_moments():
    M = d2q9.MRT_M
    np.testing.assert_array_equal(M @ M.T, np.diag([9, 36, 36, 6, 12, 6, 12, 4, 4]))
    # rows are polynomials in c: rho=1, e=3|c|^2-4, jx=cx, qx=(3|c|^2-5)cx,
    # pxx=cx^2-cy^2, pxy=cx cy
    cx, cy = C[:, 0].astype(float), C[:, 1].astype(float)
    c2 = cx * cx + cy * cy
    np.testing.assert_array_equal(M[1], 3 * c2 - 4)
    np.testing.assert_array_equal(M[2], 4.5 * c2 * c2 - 10.5 * c2 + 4)
    np.testing.assert_array_equal(M[4], (3 * c2 - 5) * cx)
    np.testing.assert_array_equal(M[6], (3 * c2 - 5) * cy)
    np.testing.assert_array_equal(M[7], cx * cx - cy * cy)
    np.testing.assert_array_equal(M[8], cx * cy)
    rng = np.random.default_rng(4)
    rho = 1 + 0.1 * rng.random(20)
    ux, uy = 0.1 * rng.standard_normal(20), 0.1 * rng.standard_normal(20)
    m = M @ d2q9.equilibrium(rho, ux, uy)
    u2 = ux * ux + uy * uy
    closed = np.stack([rho, -2 * rho + 3 * rho * u2, rho - 3 * rho * u2,
                       rho * ux, -rho * ux, rho * uy, -rho * uy,
                       rho * (ux * ux - uy * uy), rho * ux * uy])
    np.testing.assert_allclose(m, closed, atol=1e-15)


def test_mrt_magic_rate():
    for tau in (0.5075, 0.53, 0.6, 1.0, 2.0):
        sq = d2q9.mrt_magic_sq(tau)
        assert abs((tau - 0.5) * (1 / sq - 0.5) - 3 / 16) < 1e-15


def test_mrt_relaxes_each_moment_at_its_rate():
    rng = np.random.default_rng(5)
    f = _rand_state(rng, (4, 4))
    tau = 0.7
    rates = d2q9.mrt_rates(tau, 1.2, 1.4, 1.6)
    M = d2q9.MRT_M
    meq = np.tensordot(M, d2q9.equilibrium(*d2q9.moments(f)), axes=(1, 0))
    m0 = np.tensordot(M, f, axes=(1, 0))
    m1 = np.tensordot(M, d2q9.mrt_collide(f, tau, 1.2, 1.4, 1.6), axes=(1, 0))
    for k in range(9):
        np.testing.assert_allclose(m1[k] - meq[k], (1 - rates[k]) * (m0[k] - meq[k]),
                                   atol=1e-14)


# --- Zou & He ------------------------------------------------------------------

def test_outlet_moments_and_unchanged_knowns():
    rng = np.random.default_rng(6)
    f = _rand_state(rng, (40,))
    g, u = zouhe.outlet_pressure(f, 1.02)
    cx, cy = C[:, 0, None].astype(float), C[:, 1, None].astype(float)
    np.testing.assert_allclose(g.sum(0), 1.02, rtol=1e-15)        # prescribed rho
    np.testing.assert_allclose((cy * g).sum(0), 0.0, atol=1e-16)  # v = 0
    np.testing.assert_allclose((cx * g).sum(0), 1.02 * u, atol=1e-15)
    for q in (0, 1, 2, 4, 5, 8):                                   # Eq. 11
        np.testing.assert_array_equal(g[q], f[q])
    # non-equilibrium bounce-back of the normal pair
    feq = d2q9.equilibrium(1.02, u, 0 * u)
    np.testing.assert_allclose(g[3] - feq[3], f[1] - feq[1], atol=1e-16)


def test_inlet_moments_and_unchanged_knowns():
    rng = np.random.default_rng(7)
    f = _rand_state(rng, (40,))
    prof = 0.05 + 0.01 * rng.random(40)
    g, rho = zouhe.inlet_velocity(f, prof, 0.0)
    cx, cy = C[:, 0, None].astype(float), C[:, 1, None].astype(float)
    np.testing.assert_allclose(g.sum(0), rho, rtol=1e-15)
    np.testing.assert_allclose((cx * g).sum(0), rho * prof, rtol=1e-14)
    np.testing.assert_allclose((cy * g).sum(0), 0.0, atol=1e-16)
    for q in (0, 2, 3, 4, 6, 7):
        np.testing.assert_array_equal(g[q], f[q])
    feq = d2q9.equilibrium(rho, prof, 0 * prof)
    np.testing.assert_allclose(g[1] - feq[1], f[3] - feq[3], atol=1e-16)


def test_zouhe_keeps_equilibrium():
    # an equilibrium column with the prescribed macros is reproduced exactly
    feq = d2q9.equilibrium(np.full(5, 1.0), np.full(5, 0.05), np.zeros(5))
    g, u = zouhe.outlet_pressure(feq, 1.0)
    np.testing.assert_allclose(u, 0.05, rtol=1e-14)
    np.testing.assert_allclose(g, feq, rtol=1e-14)
    feq2 = d2q9.equilibrium(np.full(5, 1.03), np.full(5, 0.04), np.zeros(5))
    g2, rho = zouhe.inlet_velocity(feq2, 0.04)
    np.testing.assert_allclose(rho, 1.03, rtol=1e-14)
    np.testing.assert_allclose(g2, feq2, rtol=1e-14)
