"""GPU parity of the characteristic outflow (Sec. 4, Eqs. 18-29) fused into
the step, against the oracle, through the C ABI (lbm_set_outflow_cbc).

FP64: both sides take the same arithmetic in the same order up to
summation order (gradients, LODI terms, forward Euler, reconstruction), so
populations agree to 1e-12 relative after hundreds of steps; the tuning
network is evaluated in FP64 on both sides from the same FP32 weights.
FP32 offsets: the density and velocity tolerances of the plain step."""
import numpy as np
import pytest

from oracle.d2q9 import CS2, moments
from oracle.solver import Lattice as Oracle
from paper_2506_05293_amd import geometry, lbm, workloads

pytestmark = pytest.mark.gpu
CS = np.sqrt(CS2)


def _say(*a):
    print("[gpu case]", *a, flush=True)


def vortex_fields(nx, ny, u0, xc, yc, rc=6.0, beta=0.3):
    """Lamb-Oseen vortex in a uniform stream (isothermal density)."""
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    r2 = (x - xc) ** 2 + (y - yc) ** 2
    e = np.exp(-r2 / (2 * rc**2))
    ux = u0 - beta * u0 * (y - yc) / rc * e
    uy = beta * u0 * (x - xc) / rc * e
    rho = np.exp(-(beta * u0) ** 2 / (2 * CS2) * np.exp(-r2 / rc**2))
    return rho, ux, uy


def random_net(seed):
    rng = np.random.default_rng(seed)
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    return {"w1": f32(0.5 * rng.standard_normal((20, 9))), "b1": f32(0.2 * rng.standard_normal(20)),
            "w2": f32(0.3 * rng.standard_normal((20, 20))), "b2": f32(0.2 * rng.standard_normal(20)),
            "w3": f32(0.3 * rng.standard_normal((2, 20))), "b3": f32(0.2 * rng.standard_normal(2)),
            "mu_in": f32(1e-5 * rng.standard_normal(9)), "sd_in": f32(np.full(9, 2e-4)),
            "leaky_slope": 0.01, "sigma_scale": 1.0, "sigma_shift": 0.0,
            "kappa_scale": 0.6, "kappa_shift": 0.0}


def _pair(nx, ny, lateral, collision, precision, cbc, tau=0.58, u0=0.1, mask=None):
    mask = np.zeros((ny, nx), np.uint8) if mask is None else mask
    rho, ux, uy = vortex_fields(nx, ny, u0, nx - 14.5, ny / 2 - 0.3)
    g = lbm.Lattice(mask, tau, precision=precision, collision=collision, lateral=lateral,
                    u_in=u0, noise_amp=0.0, seed=1)
    g.init_fields(rho, ux, uy)
    g.set_outflow_cbc(**cbc)
    o = Oracle(mask, tau, collision=collision, lateral=lateral, u_in=u0)
    o.set_equilibrium(rho, ux, uy)
    o.set_outflow_cbc(**{**cbc, "length": cbc.get("length", nx)})
    return g, o


FIXED = dict(sigma=0.4, kappa2=0.3, mach=0.1 / CS, length=61.0, rho_inf=1.0)


@pytest.mark.parametrize("collision,body", [("bgk", False), ("mrt", False), ("mrt", True)])
def test_cbc_fp64_parity(collision, body, schedule):
    lateral = "periodic"
    _say("cbc fp64", collision, "body" if body else "")
    mask = geometry.cylinder(61, 43, 14.3, 20.6, 9.0) if body else None
    g, o = _pair(61, 43, lateral, collision, "fp64", FIXED, mask=mask)
    g.step(150)
    o.step(150)
    f, ref = g.populations(), o.post_collision()
    err = np.max(np.abs(f - ref) / np.abs(ref))
    print("cbc fp64 max rel error", err, flush=True)
    assert err < 1e-12
    # the characteristic outlet is not the Zou & He one
    mask = np.zeros((43, 61), np.uint8) if mask is None else mask
    z = Oracle(mask, 0.58, collision=collision, lateral=lateral, u_in=0.1)
    z.set_equilibrium(*vortex_fields(61, 43, 0.1, 61 - 14.5, 43 / 2 - 0.3))
    z.step(150)
    assert np.max(np.abs(z.post_collision()[:, :, -1] - ref[:, :, -1])) > 1e-6
    fo = g.forces()
    assert abs(fo.mass - o.mass_hist[-1]) < 1e-10 * o.mass_hist[-1]


def test_cbc_network_fp64_parity(schedule):
    _say("cbc network fp64")
    cbc = dict(FIXED, net=random_net(3))
    g, o = _pair(61, 43, "periodic", "bgk", "fp64", cbc)
    g.step(120)
    o.step(120)
    f, ref = g.populations(), o.post_collision()
    err = np.max(np.abs(f - ref) / np.abs(ref))
    print("cbc network fp64 max rel error", err, flush=True)
    assert err < 1e-11
    # the network is not a constant map here: sigma, kappa_2 vary over the column
    fs = o.collide(o.f)[:, :, -3:]
    rho, ux, uy = moments(fs)
    from oracle import cbc as ocbc
    grads = ocbc.gradients(rho.T, ux.T, uy.T, True)
    feats = np.stack([*grads, *o.cbc_prev.T], axis=1)
    sig, kap = ocbc.network(feats, cbc["net"])
    assert np.ptp(sig) > 1e-3 and np.ptp(kap) > 1e-3


@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_cbc_fp32_offsets(collision, schedule):
    _say("cbc fp32", collision)
    g, o = _pair(61, 43, "periodic", collision, "fp32", FIXED)
    g.step(300)
    o.step(300)
    rg, ug, vg = moments(g.populations())
    ro, uo, vo = o.macroscopic()
    assert np.max(np.abs(rg - ro)) < 1e-5
    assert max(np.max(np.abs(ug - uo)), np.max(np.abs(vg - vo))) < 1e-4


def test_cbc_uniform_flow_is_a_fixed_point():
    _say("cbc uniform fixed point")
    nx, ny, u0 = 70, 24, 0.08
    g = lbm.Lattice(np.zeros((ny, nx), np.uint8), 0.6, precision="fp64", collision="mrt",
                    lateral="periodic", u_in=u0, noise_amp=0.0)
    f0 = g.populations()
    g.set_outflow_cbc(sigma=0.5, kappa2=0.2, mach=u0 / CS)
    g.step(200)
    np.testing.assert_allclose(g.populations(), f0, rtol=0, atol=1e-14)


def test_cbc_plane_pulse_leaves_without_reflection():
    # the method's defining property on the GPU (FP32 offsets): a right-going
    # plane pulse leaves through the characteristic outlet and is sent back by
    # the Zou & He pressure outlet
    _say("cbc plane pulse")
    nx, ny, amp, x0, w = 160, 8, 2e-3, 80.0, 6.0
    x = np.arange(nx)[None, :].repeat(ny, 0).astype(float)
    drho = amp * np.exp(-0.5 * ((x - x0) / w) ** 2)
    out = {}
    for kind in ("cbc", "zouhe"):
        g = lbm.Lattice(np.zeros((ny, nx), np.uint8), 0.52, precision="fp32", collision="bgk",
                        lateral="periodic", u_in=0.0, noise_amp=0.0)
        g.init_fields(1 + drho, CS * drho, np.zeros_like(drho))
        if kind == "cbc":
            g.set_outflow_cbc(sigma=0.0, kappa2=0.0, mach=0.0)
        g.step(int((nx - x0 + 4 * w) / CS) + 20)
        rho, _, _ = moments(g.populations())
        out[kind] = np.abs(rho - 1).max() / amp
    print("pulse residual", out, flush=True)
    assert out["cbc"] < 0.05 and out["zouhe"] > 0.5


def test_cbc_full_size_steps(schedule):
    # the 4096 x 1024 cylinder lattice with periodic laterals, FP32,
    # characteristic outlet: both sides start from the same seeded smooth
    # fields and take three steps; every fluid node is compared
    nx, ny = 4096, 1024
    mask = geometry.cylinder(nx, ny, 800, ny // 2, 80)
    tau = 3 * 0.05 * 80 / 200 + 0.5
    _say("cbc full size 4096x1024 fp32")
    rho, u = workloads.smooth_fields(mask.shape, 0.05, amp=0.02, seed=14)
    g = lbm.Lattice(mask, tau, precision="fp32", collision="mrt", lateral="periodic",
                    u_in=0.05, noise_amp=0.0)
    g.init_fields(rho, u[0], u[1])
    g.set_outflow_cbc(sigma=0.25, kappa2=0.05 / CS, mach=0.05 / CS)
    g.step(3)
    o = Oracle(mask, tau, collision="mrt", lateral="periodic", u_in=0.05)
    o.set_equilibrium(rho, u[0], u[1])
    o.set_outflow_cbc(sigma=0.25, kappa2=0.05 / CS, mach=0.05 / CS, length=nx)
    o.step(3)
    fl = mask == 0
    ref = o.post_collision()
    err = np.max(np.abs(g.populations()[:, fl] - ref[:, fl]))
    print("cbc full-size three-step error", err, flush=True)
    assert err < 2e-6


@pytest.mark.parametrize("net", [False, True])
def test_cbc_pairs_equal_single_steps(net):
    # two steps per launch at the characteristic outlet: the outlet blocks run
    # the single-step arithmetic (LODI update, Eq. 29 reconstruction, the
    # network in FP64) and carry the time derivatives of the first step to
    # the second in LDS, so both schedules agree to 1e-12 relative in FP64,
    # over odd counts, read-outs and a lattice shorter than one outlet block
    _say("cbc pairs vs single steps", "network" if net else "fixed")
    cbc = dict(FIXED, net=random_net(3)) if net else FIXED
    mask = geometry.cylinder(61, 43, 14.3, 20.6, 9.0)
    out = {}
    for launch in ("pairs", "pairs_held", "single"):
        g = lbm.Lattice(mask, 0.58, precision="fp64", collision="mrt", lateral="periodic",
                        u_in=0.1, noise_amp=0.0, seed=1, launch=launch, history_cap=81)
        g.init_fields(*vortex_fields(61, 43, 0.1, 61 - 14.5, 43 / 2 - 0.3))
        g.set_outflow_cbc(**cbc)
        for n in (40, 7, 34):
            g.step(n)
        out[launch] = (g.populations(), g.force_history()[0])
    (f1, fx1), (f0, fx0) = out["pairs"], out["single"]
    print("cbc pairs vs single: populations that differ", np.count_nonzero(f1 != f0), flush=True)
    np.testing.assert_array_equal(f1, f0)
    # the strips' other walk (stores held back one row): the same bits
    np.testing.assert_array_equal(out["pairs_held"][0], f1)
    np.testing.assert_array_equal(out["pairs_held"][1], fx1)
    np.testing.assert_allclose(fx1, fx0, rtol=0, atol=1e-12 * np.max(np.abs(fx0)))


def test_cbc_pairs_full_size():
    # the 4096 x 1024 cylinder lattice with periodic laterals and the
    # characteristic outlet, FP32, four steps in two launches, against the
    # oracle from the same seeded smooth fields
    nx, ny = 4096, 1024
    mask = geometry.cylinder(nx, ny, 800, ny // 2, 80)
    tau = 3 * 0.05 * 80 / 200 + 0.5
    _say("cbc pairs full size 4096x1024 fp32")
    rho, u = workloads.smooth_fields(mask.shape, 0.05, amp=0.02, seed=14)
    g = lbm.Lattice(mask, tau, precision="fp32", collision="mrt", lateral="periodic",
                    u_in=0.05, noise_amp=0.0, launch="pairs")
    g.init_fields(rho, u[0], u[1])
    g.set_outflow_cbc(sigma=0.25, kappa2=0.05 / CS, mach=0.05 / CS)
    g.step(4)
    o = Oracle(mask, tau, collision="mrt", lateral="periodic", u_in=0.05)
    o.set_equilibrium(rho, u[0], u[1])
    o.set_outflow_cbc(sigma=0.25, kappa2=0.05 / CS, mach=0.05 / CS, length=nx)
    o.step(4)
    fl = mask == 0
    err = np.max(np.abs(g.populations()[:, fl] - o.post_collision()[:, fl]))
    print("cbc pairs full-size four-step error", err, flush=True)
    assert err < 2e-6
