"""GPU parity of the configurations of the diffusive-scaling sweep (Sec. 3.1:
the relaxation time stays at 0.6 and u_in = Re nu / D, so the inflow speed
grows with Re: 0.0052 at Re 10, 0.104 at Re 200) on the sweep's own lattice,
the 8 D truncated cylinder (4096 x 512, D = 64, periodic laterals, MRT with
the sweep's rates, FP32 offsets), with the Zou & He and with the neural
outflow, against the oracle.  Both sides start from the same seeded smooth
fields around the configuration's inflow and take three steps; the bound is
that of the other full-size FP32 step tests (offsets stored with a 24-bit
significand)."""
import numpy as np
import pytest

import cases
from oracle.solver import Lattice as Oracle
from paper_2506_05293_amd import experiments, lbm, workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("outflow", ["zouhe", "nn"])
@pytest.mark.parametrize("re", [10.0, 200.0])
def test_diffusive_scaling_configuration(re, outflow):
    case = workloads.truncated_cylinder(8, re=re, tau=0.6)
    mask, tau, u_in = case["mask"], case["tau"], case["u_in"]
    assert mask.shape == (512, 4096)
    assert u_in == pytest.approx(re * (0.6 - 0.5) / 3.0 / 64)
    print("[gpu case] diffusive scaling Re", re, outflow, "u_in", u_in, flush=True)
    rho, u = workloads.smooth_fields(mask.shape, u_in, amp=0.02, seed=21)
    g = lbm.Lattice(mask, tau, precision="fp32", collision="mrt", lateral="periodic",
                    u_in=u_in, noise_amp=0.0, history_cap=3, **experiments.RATES)
    g.init_fields(rho, u[0], u[1])
    o = Oracle(mask, tau, collision="mrt", lateral="periodic", u_in=u_in, **experiments.RATES)
    o.set_equilibrium(rho, u[0], u[1])
    if outflow == "nn":
        P = cases.f32_values(cases.random_params(5, w_scale=0.5, out_sd=2e-4))
        g.set_outflow_nn(P, mass_bound=1e9)
        o.set_outflow_nn(P, mass_bound=1e9)
    g.step(3)
    o.step(3)
    fl = mask == 0
    got, want = g.populations(), o.post_collision()
    err = np.max(np.abs(got[:, fl] - want[:, fl]))
    print("three-step error", err, flush=True)
    assert err < 1e-6
    fx, fy = g.force_history()
    np.testing.assert_allclose(fx, o.fx_hist, rtol=1e-5, atol=1e-8)
    np.testing.assert_allclose(fy, o.fy_hist, rtol=1e-5, atol=1e-8)
