"""Pins of the D3Q19 oracle: lattice isotropy and equilibrium moments in
closed form, conservation by BGK, streaming against a brute-force neighbour
loop, exact moments of the inlet and outlet faces, the free stream as a
fixed point, the decay rate of a shear wave (viscosity cs^2 (tau - 1/2)),
the momentum balance with a body, and the reduction to the two-dimensional
step for flows uniform in z."""
import itertools

import numpy as np
import pytest

from oracle import d2q9, d3q19
from oracle.d3q19 import C, CS2, OPP, W
from oracle.solver import Lattice as Lattice2


def test_lattice_isotropy():
    assert W.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose((W[:, None] * C).sum(0), 0, atol=1e-15)
    second = np.einsum("i,ia,ib->ab", W, C, C)
    np.testing.assert_allclose(second, CS2 * np.eye(3), atol=1e-15)
    fourth = np.einsum("i,ia,ib,ic,id->abcd", W, C, C, C, C)
    d = np.eye(3)
    iso = CS2**2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) +
                    np.einsum("ad,bc->abcd", d, d))
    np.testing.assert_allclose(fourth, iso, atol=1e-15)
    assert all((C[OPP] == -C).ravel())
    assert sorted(map(tuple, C.tolist())) == sorted(
        [(0, 0, 0)] + [v for v in itertools.product((-1, 0, 1), repeat=3)
                       if sum(map(abs, v)) in (1, 2)])


def test_equilibrium_moments():
    rng = np.random.default_rng(0)
    rho = 1 + 0.05 * rng.standard_normal(50)
    u = 0.08 * rng.standard_normal((3, 50))
    feq = d3q19.equilibrium(rho, u)
    np.testing.assert_allclose(feq.sum(0), rho, rtol=1e-14)
    np.testing.assert_allclose(np.tensordot(C.T.astype(float), feq, axes=(1, 0)), rho * u,
                               rtol=1e-13, atol=1e-16)
    pi = np.einsum("ia,ib,in->abn", C, C, feq)
    want = rho * (CS2 * np.eye(3)[:, :, None] + u[:, None] * u[None, :])
    np.testing.assert_allclose(pi, want, rtol=1e-13, atol=1e-16)


def test_bgk_conserves_mass_and_momentum():
    rng = np.random.default_rng(1)
    f = d3q19.equilibrium(np.ones(40), np.zeros((3, 40))) * (1 + 0.1 * rng.random((19, 40)))
    g = d3q19.bgk_collide(f, 0.7)
    np.testing.assert_allclose(g.sum(0), f.sum(0), rtol=1e-14)
    np.testing.assert_allclose(np.tensordot(C.T.astype(float), g, axes=(1, 0)),
                               np.tensordot(C.T.astype(float), f, axes=(1, 0)), atol=1e-15)


@pytest.mark.parametrize("lateral", ["walls", "periodic"])
def test_streaming_matches_neighbour_loop(lateral):
    rng = np.random.default_rng(2)
    nz, ny, nx = 4, 5, 6
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[1:3, 2, 2:4] = 1
    lat = d3q19.Lattice3(mask, 0.7, lateral=lateral)
    fs = rng.random((19, nz, ny, nx))
    got = lat.stream(fs)
    for i, z, y, x in itertools.product(range(19), range(nz), range(ny), range(nx)):
        if mask[z, y, x]:
            continue
        sx, sy, sz = x - C[i, 0], y - C[i, 1], z - C[i, 2]
        if not 0 <= sx < nx:
            assert np.isnan(got[i, z, y, x])
            continue
        if lateral == "periodic":
            sy, sz = sy % ny, sz % nz
        elif not (0 <= sy < ny and 0 <= sz < nz):
            assert got[i, z, y, x] == fs[OPP[i], z, y, x]
            continue
        want = fs[OPP[i], z, y, x] if mask[sz, sy, sx] else fs[i, sz, sy, sx]
        assert got[i, z, y, x] == want


@pytest.mark.parametrize("side", ["in", "out"])
def test_face_carries_prescribed_moments(side):
    rng = np.random.default_rng(3)
    n = 30
    rho = 1 + 0.02 * rng.standard_normal(n)
    u = np.stack([0.05 + 0.01 * rng.standard_normal(n), 0.01 * rng.standard_normal(n),
                  0.01 * rng.standard_normal(n)])
    f = d3q19.equilibrium(rho, u) + 1e-3 * rng.standard_normal((19, n))
    # the face's own rule fixes the free quantity (Eq. 7): the inlet density,
    # the outlet normal velocity
    if side == "in":
        rho = d3q19.inlet_density(f, u[0])
    else:
        u[0] = d3q19.outlet_velocity(f, rho)
    g = d3q19.face_unknowns(f, rho, u, side)
    np.testing.assert_allclose(g.sum(0), rho, rtol=1e-14)
    np.testing.assert_allclose(np.tensordot(C.T.astype(float), g, axes=(1, 0)), rho * u,
                               rtol=1e-12, atol=1e-16)
    sgn = 1 if side == "in" else -1
    for i in range(19):
        if C[i, 0] != sgn:
            assert np.array_equal(g[i], f[i])            # known populations stay
    # an equilibrium face is a fixed point
    feq = d3q19.equilibrium(rho, u)
    np.testing.assert_allclose(d3q19.face_unknowns(feq, rho, u, side), feq, atol=1e-16)


def test_density_and_velocity_rules_on_an_equilibrium_face():
    rho, ux = 1.013, 0.061
    feq = d3q19.equilibrium(np.array([rho]), np.array([[ux], [0.0], [0.0]]))
    assert d3q19.inlet_density(feq, ux)[0] == pytest.approx(rho, rel=1e-14)
    assert d3q19.outlet_velocity(feq, rho)[0] == pytest.approx(ux, rel=1e-13)


@pytest.mark.parametrize("lateral", ["walls", "periodic"])
def test_free_stream_is_a_fixed_point(lateral):
    # with walls only the rest state is (no-slip); periodic keeps u_in
    u_in = 0.0 if lateral == "walls" else 0.06
    lat = d3q19.Lattice3(np.zeros((4, 5, 12), np.uint8), 0.65, lateral=lateral, u_in=u_in)
    f0 = lat.f.copy()
    lat.step(20)
    np.testing.assert_allclose(lat.f, f0, rtol=0, atol=1e-15)


def _shear_wave_viscosity(nz, tau, steps, amp=1e-4):
    """Effective viscosity of a decaying shear wave u_x = A sin(2 pi z / nz)."""
    lat = d3q19.Lattice3(np.zeros((nz, 2, 2), np.uint8), tau, lateral="periodic",
                         xbc="periodic", u_in=0.0)
    z = np.arange(nz)[:, None, None] * np.ones((nz, 2, 2))
    k = 2 * np.pi / nz
    u = np.zeros((3, nz, 2, 2))
    u[0] = amp * np.sin(k * z)
    lat.set_fields(np.ones((nz, 2, 2)), u)
    lat.step(steps)
    _, uu = d3q19.moments(lat.f)
    a = 2 * np.mean(uu[0] * np.sin(k * z))
    return -np.log(a / amp) / (k * k * steps)


def test_shear_wave_decays_at_the_lattice_viscosity_to_second_order():
    # nu = cs^2 (tau - 1/2); the discrete decay rate approaches it as (k dx)^2
    tau = 0.8
    nu = CS2 * (tau - 0.5)
    e32 = abs(_shear_wave_viscosity(32, tau, 400) / nu - 1)
    e64 = abs(_shear_wave_viscosity(64, tau, 1600) / nu - 1)
    assert e32 < 5e-3
    assert 3.0 < e32 / e64 < 5.0


def test_momentum_balance_with_a_body():
    rng = np.random.default_rng(4)
    nz, ny, nx = 6, 7, 8
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[2:4, 2:5, 3:5] = 1
    lat = d3q19.Lattice3(mask, 0.7, lateral="periodic", xbc="periodic", u_in=0.0)
    u = 0.02 * rng.standard_normal((3, nz, ny, nx))
    lat.set_fields(1 + 0.01 * rng.standard_normal((nz, ny, nx)), u)
    for _ in range(5):
        p0 = lat.momentum()
        lat.step(1)
        F = np.array([lat.fx_hist[-1], lat.fy_hist[-1], lat.fz_hist[-1]])
        np.testing.assert_allclose(lat.momentum() - p0, -F, atol=1e-13)
    assert np.abs(F).max() > 1e-6


def test_flow_uniform_in_z_projects_exactly_onto_the_two_dimensional_step():
    # summing the D3Q19 populations over c_z gives the D2Q9 weights; BGK,
    # streaming, bounce-back and the face construction commute with that
    # projection, so a flow uniform in z (periodic z) is the D2Q9 step of
    # the two-dimensional oracle, faces and forces included
    ny, nx, u_in, nz = 10, 24, 0.05, 3
    mask2 = np.zeros((ny, nx), np.uint8)
    mask2[4:6, 8:10] = 1
    rng = np.random.default_rng(5)
    rho = 1 + 0.01 * rng.standard_normal((ny, nx))
    ux = u_in + 0.01 * rng.standard_normal((ny, nx))
    uy = 0.01 * rng.standard_normal((ny, nx))
    l2 = Lattice2(mask2, 0.8, lateral="walls", u_in=u_in)
    l2.set_equilibrium(rho, ux, uy)
    l3 = d3q19.Lattice3(np.repeat(mask2[None], nz, axis=0), 0.8, lateral=("walls", "periodic"),
                        u_in=u_in)
    l3.set_fields(np.repeat(rho[None], nz, 0),
                  np.stack([np.repeat(a[None], nz, 0) for a in (ux, uy, np.zeros_like(ux))]))
    l2.step(40)
    l3.step(40)
    proj = np.zeros((9, nz, ny, nx))
    for i in range(19):
        k = [q for q in range(9) if tuple(d2q9.C[q]) == tuple(C[i, :2])][0]
        proj[k] += l3.f[i]
    fl = mask2 == 0
    for z in range(nz):
        np.testing.assert_allclose(proj[:, z][:, fl], l2.f[:, fl], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(np.array(l3.fx_hist), nz * np.array(l2.fx_hist), rtol=1e-10,
                               atol=1e-15)
    np.testing.assert_allclose(np.array(l3.fy_hist), nz * np.array(l2.fy_hist), rtol=1e-10,
                               atol=1e-15)
    np.testing.assert_allclose(np.array(l3.fz_hist), 0, atol=1e-15)
