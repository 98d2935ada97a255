"""GPU parity of the D3Q19 step through the C ABI (lbm3d_*) against the
FP64 oracle (oracle/d3q19.py).

FP64: the same arithmetic up to summation order, so populations agree to
1e-12 relative after hundreds of steps and the force history to 1e-11 of
its scale.  FP32 offsets: density within 1e-5 and velocity within 1e-4 (as
for the D2Q9 step: offsets of order 1e-2 stored with a 24-bit significand).
"""
import numpy as np
import pytest

from oracle import d3q19
from oracle.d3q19 import C
from paper_2506_05293_amd import lbm, workloads

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu case]", *a, flush=True)


def _sphere(nz, ny, nx, xc, r):
    Z, Y, X = np.mgrid[0:nz, 0:ny, 0:nx]
    return (((X - xc) ** 2 + (Y - (ny - 1) / 2) ** 2 + (Z - (nz - 1) / 2) ** 2) <= r * r
            ).astype(np.uint8)


def _fields(shape, u0, seed):
    rng = np.random.default_rng(seed)
    rho = 1 + 0.01 * rng.standard_normal(shape)
    u = np.stack([u0 + 0.01 * rng.standard_normal(shape), 0.01 * rng.standard_normal(shape),
                  0.01 * rng.standard_normal(shape)])
    return rho, u


CASES = [
    ((10, 12, 37), ("walls", "periodic"), "inout"),
    ((9, 11, 29), ("walls", "walls"), "inout"),
    ((8, 10, 21), ("periodic", "periodic"), "inout"),
    ((6, 8, 300), ("periodic", "walls"), "inout"),        # two x-tiles, ragged
    ((8, 9, 16), ("periodic", "periodic"), "periodic"),
]


@pytest.mark.parametrize("shape,lateral,xbc", CASES)
def test_fp64_parity_with_a_body(shape, lateral, xbc):
    nz, ny, nx = shape
    _say("d3q19 fp64", shape, lateral, xbc)
    mask = _sphere(nz, ny, nx, nx // 3, 2.6)
    tau, u0, steps = 0.62, 0.05, 120
    g = lbm.Lattice3D(mask, tau, precision="fp64", lateral=lateral, xbc=xbc, u_in=u0,
                      history_cap=steps)
    o = d3q19.Lattice3(mask, tau, lateral=lateral, xbc=xbc, u_in=u0)
    rho, u = _fields(shape, u0, 1)
    g.init_fields(rho, u)
    o.set_fields(rho, u)
    g.step(steps)
    o.step(steps)
    f, ref = g.populations(), o.post_collision()
    err = np.max(np.abs(f - ref) / np.abs(ref))
    print("max rel error", err, flush=True)
    assert err < 1e-12
    fx, fy, fz = g.force_history()
    scale = max(np.max(np.abs(o.fx_hist)), 1e-12)
    for got, want in ((fx, o.fx_hist), (fy, o.fy_hist), (fz, o.fz_hist)):
        assert len(got) == steps
        assert np.max(np.abs(got - np.array(want))) < 1e-11 * scale
    fo = g.forces()
    assert fo.step == steps and fo.nonfinite == 0
    dm = (o.f.sum(axis=0) - 1)[mask == 0].sum()
    assert abs(fo.dmass - dm) < 1e-9


@pytest.mark.parametrize("lateral", [("walls", "periodic"), ("periodic", "periodic")])
def test_fp32_offsets(lateral):
    shape = (10, 12, 40)
    _say("d3q19 fp32", lateral)
    mask = _sphere(*shape, 12, 2.6)
    g = lbm.Lattice3D(mask, 0.6, precision="fp32", lateral=lateral, u_in=0.05)
    o = d3q19.Lattice3(mask, 0.6, lateral=lateral, u_in=0.05)
    rho, u = _fields(shape, 0.05, 2)
    g.init_fields(rho, u)
    o.set_fields(rho, u)
    g.step(200)
    o.step(200)
    rg, ug = d3q19.moments(g.populations())
    ro, uo = d3q19.moments(o.post_collision())
    fl = mask == 0
    assert np.max(np.abs(rg - ro)[fl]) < 1e-5
    assert np.max(np.abs(ug - uo)[:, fl]) < 1e-4


def test_init_and_read_write_round_trip():
    shape = (5, 6, 70)
    _say("d3q19 init / read / write")
    mask = _sphere(*shape, 20, 1.5)
    g = lbm.Lattice3D(mask, 0.7, precision="fp64", lateral="periodic", u_in=0.03)
    # the geometry's initial state is f^eq(1, (u_in, 0, 0)) on fluid, f^eq(1, 0) on solid
    u = np.zeros((3,) + shape)
    u[0] = np.where(mask == 0, 0.03, 0.0)
    np.testing.assert_allclose(g.populations(), d3q19.equilibrium(np.ones(shape), u), atol=1e-16)
    rho, u = _fields(shape, 0.03, 3)
    g.init_fields(rho, u)
    want = d3q19.equilibrium(np.where(mask == 0, rho, 1.0), np.where(mask == 0, u, 0.0))
    np.testing.assert_allclose(g.populations(), want, rtol=0, atol=1e-16)
    f = want * (1 + 1e-3 * np.random.default_rng(4).standard_normal(want.shape))
    g.write_populations(f)
    np.testing.assert_array_equal(g.populations(), f)


def test_momentum_balance_in_a_periodic_box():
    # P(t+1) - P(t) = -F(t) with the GPU's own populations and force
    shape = (12, 12, 16)
    _say("d3q19 momentum balance")
    mask = _sphere(*shape, 8, 3.0)
    g = lbm.Lattice3D(mask, 0.7, precision="fp64", lateral="periodic", xbc="periodic",
                      u_in=0.0, history_cap=4)
    rho, u = _fields(shape, 0.02, 5)
    g.init_fields(rho, u)
    fl = mask == 0

    def momentum():
        # the pre-collision momentum equals the post-collision one at fluid nodes
        f = g.populations()[:, fl]
        return np.array([(C[:, a, None] * f).sum() for a in range(3)])
    for _ in range(3):
        p0 = momentum()
        g.step(1)
        fo = g.forces()
        np.testing.assert_allclose(momentum() - p0, -np.array([fo.fx, fo.fy, fo.fz]), atol=1e-12)
    assert abs(fo.fx) > 1e-6


def test_full_size_steps_fp32():
    # the 256 x 128 x 128 channel with a sphere of diameter 32 (the bench
    # lattice), FP32 offsets: both sides start from the same seeded smooth
    # fields and take two steps
    nz, ny, nx = 128, 128, 256
    _say("d3q19 full size 256x128x128 fp32")
    mask = _sphere(nz, ny, nx, 64, 16.0)
    tau = 0.5 + 3 * 0.05 * 32 / 100
    rho, u = workloads.smooth_fields(mask.shape, 0.05, amp=0.02, seed=15)
    g = lbm.Lattice3D(mask, tau, precision="fp32", lateral="walls", u_in=0.05, history_cap=2)
    g.init_fields(rho, u)
    g.step(2)
    o = d3q19.Lattice3(mask, tau, lateral="walls", u_in=0.05)
    o.set_fields(rho, u)
    o.step(2)
    fl = mask == 0
    err = np.max(np.abs(g.populations() - o.post_collision())[:, fl])
    print("d3q19 full-size two-step error", err, flush=True)
    assert err < 2e-7
    fx, fy, fz = g.force_history()
    np.testing.assert_allclose(fx, o.fx_hist, rtol=1e-5, atol=1e-8)
