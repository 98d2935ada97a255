"""GPU parity of three steps per launch (params.launch = LBM_LAUNCH_TRIPLES
or the default; Zou & He, neural and characteristic outflows; FP32 and FP16
offsets).  Every node takes the
single-step node code, and the states after the first two steps of a
launch are rounded to the storage precision as a store and reload would
round them, so the populations equal those of one launch per step bit for
bit, over step counts that leave one or two steps for two-step and single
launches and over read-outs in between.  The force and mass terms are
summed in other groups (strips of the three-step kernel, tiles of the
one-step kernel, which adds a wave's terms in FP32 first): the force
history agrees to 1e-5 of its scale.  Against the oracle as the other
schedules: the full-size bench lattice from the same smooth fields."""
import numpy as np
import pytest

import cases
from oracle.solver import Lattice as Oracle
from paper_2506_05293_amd import lbm, workloads

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu case]", *a, flush=True)


def _gpu(case, precision, history_cap, launch):
    return lbm.Lattice(case["mask"], case["tau"], precision=precision,
                       collision=case["collision"], lateral=case["lateral"],
                       u_in=case["u_in"], noise_amp=case["noise_amp"], seed=case["seed"],
                       history_cap=history_cap, launch=launch)


@pytest.mark.parametrize("name,precision", [("c1_bgk", "fp32"), ("ragged_mrt_periodic", "fp32"),
                                            ("ragged_mrt_walls", "fp16"), ("c1_mrt", "fp32"),
                                            ("c1_mrt", "fp16")])
def test_triples_equal_single_steps(name, precision):
    case = {"c1_bgk": cases.c1(75.0), "ragged_mrt_periodic": cases.ragged("mrt", "periodic"),
            "ragged_mrt_walls": cases.ragged("mrt", "walls"), "c1_mrt": cases.c1(100.0, "mrt")}[name]
    _say("triples vs single steps", name, precision)
    chunks = (40, 7, 34, 2, 3)          # remainders of one and two steps, read-outs between
    out = {}
    for launch in ("triples", "single"):
        g = _gpu(case, precision, 86, launch)
        for n in chunks:
            g.step(n)
        out[launch] = (g.populations(), g.force_history())
    (f1, (fx1, fy1)), (f0, (fx0, fy0)) = out["triples"], out["single"]
    print("triples vs single: populations that differ", np.count_nonzero(f1 != f0), flush=True)
    np.testing.assert_array_equal(f1, f0)
    assert len(fx1) == 86
    scale = max(np.max(np.abs(fx0)), 1e-9)
    print("force history: max difference / scale", np.max(np.abs(fx1 - fx0)) / scale, flush=True)
    np.testing.assert_allclose(fx1, fx0, rtol=0, atol=1e-5 * scale)
    np.testing.assert_allclose(fy1, fy0, rtol=0, atol=1e-5 * scale)


def test_triples_full_size_c2_against_oracle():
    # the bench lattice, FP32 offsets, MRT: six steps (two launches) from the
    # same smooth fields as the oracle
    case = cases.c2()
    _say("triples c2 full size fp32")
    rho, u = workloads.smooth_fields(case["mask"].shape, case["u_in"], amp=0.02, seed=17)
    g = _gpu(case, "fp32", 6, "triples")
    g.init_fields(rho, u[0], u[1])
    g.step(6)
    o = Oracle(case["mask"], **cases.oracle_kwargs(case))
    o.set_equilibrium(rho, u[0], u[1])
    o.step(6)
    fl = case["mask"] == 0
    err = np.max(np.abs(g.populations()[:, fl] - o.post_collision()[:, fl]))
    print("c2 six-step max abs error", err, flush=True)
    assert err < 5e-8
    fx, fy = g.force_history()
    np.testing.assert_allclose(fx, o.fx_hist, rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(fy, o.fy_hist, rtol=1e-5, atol=1e-7)


@pytest.mark.parametrize("precision,mass_bound", [("fp32", 1e9), ("fp32", 3e-4), ("fp16", 3e-4)])
def test_triples_with_the_neural_outflow_equal_single_steps(precision, mass_bound):
    # the three-step outlet blocks run the single-step node code and Eq. 16
    # with its fallback on the same network tiles: the same populations bit
    # for bit and the same fallback counts, over counts that leave one or
    # two steps for other launches
    case = cases.ragged("mrt", "periodic")
    P = {k: np.asarray(v, np.float32).astype(np.float64)
         for k, v in cases.random_params(3, w_scale=0.5, out_sd=2e-4).items()}
    _say("nn triples vs single steps", precision, mass_bound)
    out = {}
    for launch in ("triples", "single"):
        g = _gpu(case, precision, 86, launch)
        g.set_outflow_nn(P, mass_bound=mass_bound)
        for n in (40, 7, 34, 2, 3):
            g.step(n)
        out[launch] = (g.populations(), g.forces().n_fallback, g.force_history())
    (f1, n1, (fx1, _)), (f0, n0, (fx0, _)) = out["triples"], out["single"]
    print("nn triples vs single: populations that differ", np.count_nonzero(f1 != f0),
          "fallbacks", n1, n0, flush=True)
    np.testing.assert_array_equal(f1, f0)
    assert n1 == n0
    if mass_bound < 1:
        assert 0.1 * 86 * 77 < n0 < 0.9 * 86 * 77      # partial fallback
    np.testing.assert_allclose(fx1, fx0, rtol=0, atol=1e-5 * np.max(np.abs(fx0)) + 1e-15)


def test_triples_with_the_neural_outflow_on_a_tall_lattice():
    # several outlet blocks of 56 rows and a ragged last one, walls
    case = cases.c1(100.0, "mrt")
    mask = np.pad(case["mask"], ((0, 131 - case["mask"].shape[0]), (0, 0)))
    case = dict(case, mask=mask)
    P = {k: np.asarray(v, np.float32).astype(np.float64)
         for k, v in cases.random_params(4, w_scale=0.5, out_sd=2e-4).items()}
    _say("nn triples, 131 rows")
    out = {}
    for launch in ("triples", "single"):
        g = _gpu(case, "fp32", 30, launch)
        g.set_outflow_nn(P, mass_bound=1e-2)
        g.step(30)
        out[launch] = g.populations()
    np.testing.assert_array_equal(out["triples"], out["single"])


@pytest.mark.parametrize("net", [False, True])
def test_triples_with_the_characteristic_outflow_equal_single_steps(net):
    # the three-step outlet blocks of the characteristic outflow run the
    # single-step arithmetic (LODI update, Eq. 29 reconstruction, the
    # tuning network) and carry the time derivatives of each step to the
    # next in LDS: the same populations bit for bit in FP32, over counts that
    # leave one or two steps for other launches and a lattice taller than
    # one outlet block
    from test_gpu_cbc import FIXED, random_net, vortex_fields
    from paper_2506_05293_amd import geometry
    _say("cbc triples vs single steps", "network" if net else "fixed")
    cbc = dict(FIXED, net=random_net(3)) if net else FIXED
    nx, ny = 61, 107
    mask = geometry.cylinder(nx, ny, 14.3, 50.6, 9.0)
    out = {}
    for launch in ("triples", "single"):
        g = lbm.Lattice(mask, 0.58, precision="fp32", collision="mrt", lateral="periodic",
                        u_in=0.1, noise_amp=0.0, seed=1, launch=launch, history_cap=86)
        g.init_fields(*vortex_fields(nx, ny, 0.1, nx - 14.5, ny / 2 - 0.3))
        g.set_outflow_cbc(**cbc)
        for n in (40, 7, 34, 2, 3):
            g.step(n)
        out[launch] = (g.populations(), g.force_history()[0])
    (f1, fx1), (f0, fx0) = out["triples"], out["single"]
    print("cbc triples vs single: populations that differ", np.count_nonzero(f1 != f0), flush=True)
    np.testing.assert_array_equal(f1, f0)
    np.testing.assert_allclose(fx1, fx0, rtol=0, atol=1e-5 * np.max(np.abs(fx0)))


@pytest.mark.parametrize("outflow", ["nn", "cbc"])
def test_triples_on_a_lattice_shorter_than_an_outlet_block(outflow):
    # 60 x 16 with periodic laterals: an outlet block's staged rows wrap round
    # the lattice about four times; three-step and single launches agree bit
    # for bit
    from test_gpu_cbc import FIXED
    from paper_2506_05293_amd import geometry
    nx, ny = 60, 16
    mask = geometry.cylinder(nx, ny, 15, 7.5, 5.0)
    _say("triples on 60 x 16 periodic,", outflow)
    out = {}
    for launch in ("triples", "single"):
        g = lbm.Lattice(mask, 0.6, precision="fp32", collision="bgk", lateral="periodic",
                        u_in=0.05, noise_amp=1e-3, seed=3, launch=launch)
        if outflow == "nn":
            P = {k: np.asarray(v, np.float32).astype(np.float64)
                 for k, v in cases.random_params(8, w_scale=0.5, out_sd=2e-4).items()}
            g.set_outflow_nn(P, mass_bound=1e9)
        else:
            g.set_outflow_cbc(**dict(FIXED, length=60.0))
        g.step(31)
        out[launch] = g.populations()
    np.testing.assert_array_equal(out["triples"], out["single"])


@pytest.mark.parametrize("outflow", ["zouhe", "nn", "cbc"])
def test_held_triple_walk_equals_plain_walk(outflow):
    # the two walks of the three-step strips differ only in when a row's
    # stores are issued and how the link flags are read: the same
    # populations and force partials bit for bit
    from test_gpu_cbc import FIXED
    case = cases.ragged("mrt", "periodic")
    _say("held vs plain three-step walk,", outflow)
    out = {}
    for launch in ("triples_held", "triples_plain"):
        g = _gpu(case, "fp32", 86, launch)
        if outflow == "nn":
            P = {k: np.asarray(v, np.float32).astype(np.float64)
                 for k, v in cases.random_params(3, w_scale=0.5, out_sd=2e-4).items()}
            g.set_outflow_nn(P, mass_bound=3e-4)
        elif outflow == "cbc":
            g.set_outflow_cbc(**dict(FIXED, length=float(case["mask"].shape[1])))
        for n in (40, 7, 34, 2, 3):
            g.step(n)
        out[launch] = (g.populations(), g.force_history())
    (f1, (fx1, fy1)), (f0, (fx0, fy0)) = out["triples_held"], out["triples_plain"]
    np.testing.assert_array_equal(f1, f0)
    np.testing.assert_array_equal(fx1, fx0)
    np.testing.assert_array_equal(fy1, fy0)
