"""GPU parity of the neural outflow (Eq. 16) fused into the step, and of the
MFMA network evaluation, against the oracle's BF16-emulating forward pass.

Tolerance of the network output: both sides round the same standardised
inputs and the same weights to BF16; the GPU accumulates in FP32 and the
oracle in FP64, so a hidden activation can land on the other side of a BF16
rounding boundary.  The bound below lets every hidden unit move by one BF16
unit in the last place (2^-8 relative) plus FP32 accumulation error (1e-5 of
the absolute sum), propagated through |W|; most outputs must agree to
within the FP32 part alone."""
import numpy as np
import pytest
import torch

import cases
import nn_bounds
from oracle import mlp as omlp
from oracle.solver import Lattice as Oracle
from paper_2506_05293_amd import geometry, lbm, workloads

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu case]", *a, flush=True)


random_params = cases.random_params
_f32 = cases.f32_values


output_bound = nn_bounds.output_bound


def _lattice_with_net(P, mass_bound=1e9, **kw):
    case = cases.c1(75.0)
    args = dict(tau=case["tau"], precision="fp32", collision="bgk", lateral="walls")
    args.update(kw)
    g = lbm.Lattice(case["mask"], **args)
    g.set_outflow_nn(P, mass_bound)
    return g


@pytest.mark.parametrize("n", [1, 63, 64, 1000, 4097])
def test_mlp_forward_matches_oracle(n):
    P = _f32(random_params(1))
    rng = np.random.default_rng(n)
    x = (0.01 * rng.standard_normal((n, 27))).astype(np.float32)
    _say("mlp forward", n)
    g = _lattice_with_net(P)
    xd = torch.from_numpy(x).cuda()
    sd = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    lbm.lbm_mlp_forward(g.ctx, xd.data_ptr(), sd.data_ptr(), n)
    torch.cuda.synchronize()
    s = sd.cpu().numpy().astype(np.float64)
    ref = omlp.forward_bf16(x.astype(np.float64), P)
    bound, tight = output_bound(x.astype(np.float64), P)
    err = np.abs(s - ref)
    assert np.all(err <= bound + 1e-12), np.max(err / (bound + 1e-30))
    assert np.mean(err <= tight + 1e-12) > 0.9


def test_zero_network_is_copy_outflow_fp64():
    case = cases.c1(100.0, "mrt")
    P = {"w1": np.zeros((64, 27)), "b1": np.zeros(64), "w2": np.zeros((64, 64)),
         "b2": np.zeros(64), "w3": np.zeros((3, 64)), "b3": np.zeros(3),
         "mu_in": np.zeros(27), "sd_in": np.ones(27), "mu_out": np.zeros(3), "sd_out": np.ones(3)}
    _say("zero network fp64 c1")
    g = lbm.Lattice(case["mask"], case["tau"], precision="fp64", collision="mrt",
                    lateral="walls", u_in=0.05, noise_amp=1e-4, seed=1, history_cap=500)
    g.set_outflow_nn(P, mass_bound=1e9)
    g.step(500)
    o = Oracle(case["mask"], **cases.oracle_kwargs(case))
    o.set_outflow_nn(P, mass_bound=1e9)
    o.step(500)
    fl = case["mask"] == 0
    f = g.populations()
    ref = o.post_collision()
    assert np.max(np.abs(f[:, fl] - ref[:, fl]) / np.abs(ref[:, fl])) < 1e-12
    assert g.forces().n_fallback == 0 == o.n_fallback


@pytest.mark.parametrize("how", ["mass_bound_zero", "nan_weights"])
def test_forced_fallback_equals_zouhe_bitwise(how, schedule, monkeypatch):
    # the neural kernel's fallback runs the single-step node code: compare
    # with one launch per step on the Zou & He side too
    monkeypatch.setitem(lbm.LATTICE_DEFAULTS, "launch", "single")
    case = cases.ragged("mrt", "periodic")
    P = _f32(random_params(2))
    bound = 0.0
    if how == "nan_weights":
        P["w2"] = P["w2"].copy()
        P["w2"][5, 7] = np.nan
        bound = 1e9
    _say("forced fallback", how)
    a = lbm.Lattice(case["mask"], case["tau"], precision="fp32", collision="mrt",
                    lateral="periodic", u_in=case["u_in"], noise_amp=case["noise_amp"],
                    seed=case["seed"])
    b = lbm.Lattice(case["mask"], case["tau"], precision="fp32", collision="mrt",
                    lateral="periodic", u_in=case["u_in"], noise_amp=case["noise_amp"],
                    seed=case["seed"])
    b.set_outflow_nn(P, mass_bound=bound)
    a.step(120)
    b.step(120)
    np.testing.assert_array_equal(a.populations(), b.populations())
    ny = case["mask"].shape[0]
    assert b.forces().n_fallback == 120 * ny


def test_nn_outflow_run_matches_oracle(schedule):
    case = cases.ragged("bgk", "periodic")
    P = _f32(random_params(3, w_scale=0.5, out_sd=2e-4))
    _say("nn outflow run fp64 vs oracle")
    g = lbm.Lattice(case["mask"], case["tau"], precision="fp64", collision="bgk",
                    lateral="periodic", u_in=case["u_in"], noise_amp=case["noise_amp"],
                    seed=case["seed"], history_cap=40)
    g.set_outflow_nn(P, mass_bound=1e9)
    g.step(40)
    o = Oracle(case["mask"], **cases.oracle_kwargs(case))
    o.set_outflow_nn(P, mass_bound=1e9)
    o.step(40)
    fl = case["mask"] == 0
    f = g.populations()
    ref = o.post_collision()
    err = np.max(np.abs(f[:, fl] - ref[:, fl]))
    print("nn run max abs error", err, flush=True)
    # corrections are ~1e-4; a BF16 flip moves one by <= 2^-8 of that
    assert err < 5e-6
    assert g.forces().n_fallback == 0 == o.n_fallback
    # the outlet really differs from Zou & He
    z = Oracle(case["mask"], **cases.oracle_kwargs(case))
    z.step(40)
    assert np.max(np.abs(z.post_collision()[:, :, -1] - ref[:, :, -1])) > 1e-5


def test_nn_outflow_full_size_steps(schedule):
    # truncated cylinder lattice 4096 x 512 (D = 64, periodic laterals, MRT,
    # FP32) with the neural outflow: both sides start from the same seeded
    # smooth fields and take three steps
    nx, ny, D = 4096, 512, 64
    mask = geometry.cylinder(nx, ny, nx - 1 - 8 * D, ny // 2, D)
    tau = 3 * 0.05 * D / 200 + 0.5
    P = _f32(random_params(4, w_scale=0.5, out_sd=2e-4))
    _say("nn full size 4096x512 fp32")
    rho, u = workloads.smooth_fields(mask.shape, 0.05, amp=0.02, seed=12)
    g = lbm.Lattice(mask, tau, precision="fp32", collision="mrt", lateral="periodic",
                    u_in=0.05, noise_amp=0.0)
    g.init_fields(rho, u[0], u[1])
    g.set_outflow_nn(P, mass_bound=1e9)
    g.step(3)
    o = Oracle(mask, tau, collision="mrt", lateral="periodic", u_in=0.05)
    o.set_equilibrium(rho, u[0], u[1])
    o.set_outflow_nn(P, mass_bound=1e9)
    o.step(3)
    fl = mask == 0
    err = np.max(np.abs(g.populations()[:, fl] - o.post_collision()[:, fl]))
    print("nn full-size three-step error", err, flush=True)
    assert err < 1e-6
    assert np.max(np.abs(o.post_collision()[:, :, -1] - o.post_collision()[:, :, -2])) > 1e-4


@pytest.mark.parametrize("precision,tol", [("fp32", 5e-6), ("fp16", 2e-4)])
def test_naca_full_size_with_neural_outflow(precision, tol, schedule):
    if schedule == "pairs_held" and precision == "fp16":
        pytest.skip("the held walk has no FP16 form (LBM_LAUNCH_PAIRS_HELD rejects FP16)")
    # the NACA0012 lattice of the airfoil study (chord 256, AoA 4 deg, 3 chords
    # behind the trailing edge: 3072 x 1024, MRT, Re 1000) with a network of the
    # paper's shape at the outlet, FP32 and FP16 offsets: three steps from the
    # same seeded smooth fields on both sides.  FP32: corrections here reach
    # ~5e-4 and a hidden activation that lands on the other side of a BF16
    # rounding boundary moves one by up to 2^-8 of that; FP16 offsets: an
    # 11-bit significand on offsets of ~1e-2 per store
    case = workloads.naca_case(4.0)
    mask, tau = case["mask"], case["tau"]
    P = _f32(padded(paper_params(6)))
    _say("naca full size", mask.shape, precision)
    rho, u = workloads.smooth_fields(mask.shape, 0.05, amp=0.02, seed=13)
    g = lbm.Lattice(mask, tau, precision=precision, collision="mrt", lateral="periodic",
                    u_in=0.05, noise_amp=0.0)
    g.init_fields(rho, u[0], u[1])
    g.set_outflow_nn(P, mass_bound=1e9)
    g.step(3)
    o = Oracle(mask, tau, collision="mrt", lateral="periodic", u_in=0.05)
    o.set_equilibrium(rho, u[0], u[1])
    o.set_outflow_nn(P, mass_bound=1e9)
    o.step(3)
    fl = mask == 0
    err = np.max(np.abs(g.populations()[:, fl] - o.post_collision()[:, fl]))
    print("naca", precision, "three-step error", err, flush=True)
    assert err < tol


def paper_params(seed):
    """A random network of the paper's shape, 9 -> 20 -> 20 -> 3 (Sec. 3.1)."""
    rng = np.random.default_rng(seed)
    return {"w1": 0.4 * rng.standard_normal((20, 9)), "b1": 0.1 * rng.standard_normal(20),
            "w2": 0.3 * rng.standard_normal((20, 20)), "b2": 0.1 * rng.standard_normal(20),
            "w3": 0.3 * rng.standard_normal((3, 20)), "b3": 0.1 * rng.standard_normal(3),
            "mu_in": 0.002 * rng.standard_normal(9), "sd_in": 0.01 + 0.01 * rng.random(9),
            "mu_out": 1e-5 * rng.standard_normal(3), "sd_out": 2e-4 * (1 + rng.random(3))}


def padded(P):
    h1, n_in = P["w1"].shape
    h2 = P["w2"].shape[0]
    Q = {"w1": np.zeros((64, 27)), "b1": np.zeros(64), "w2": np.zeros((64, 64)),
         "b2": np.zeros(64), "w3": np.zeros((3, 64)), "b3": np.array(P["b3"], float),
         "mu_in": np.zeros(27), "sd_in": np.ones(27), "mu_out": np.array(P["mu_out"], float),
         "sd_out": np.array(P["sd_out"], float)}
    Q["w1"][:h1, :n_in] = P["w1"]
    Q["b1"][:h1] = P["b1"]
    Q["w2"][:h2, :h1] = P["w2"]
    Q["b2"][:h2] = P["b2"]
    Q["w3"][:, :h2] = P["w3"]
    Q["mu_in"][:n_in] = P["mu_in"]
    Q["sd_in"][:n_in] = P["sd_in"]
    return Q


def test_paper_network_run_matches_oracle(schedule):
    case = cases.ragged("bgk", "periodic")
    P = _f32(paper_params(5))
    _say("paper-shape network run fp64 vs oracle")
    g = lbm.Lattice(case["mask"], case["tau"], precision="fp64", collision="bgk",
                    lateral="periodic", u_in=case["u_in"], noise_amp=case["noise_amp"],
                    seed=case["seed"])
    g.set_outflow_nn(P, mass_bound=1e9)
    g.step(40)
    o = Oracle(case["mask"], **cases.oracle_kwargs(case))
    o.set_outflow_nn(P, mass_bound=1e9)
    o.step(40)
    fl = case["mask"] == 0
    err = np.max(np.abs(g.populations()[:, fl] - o.post_collision()[:, fl]))
    print("paper network run max abs error", err, flush=True)
    assert err < 5e-6
    assert g.forces().n_fallback == 0 == o.n_fallback


def test_paper_network_equals_its_padded_embedding():
    P = _f32(paper_params(6))
    _say("paper-shape network vs padded 27-64-64-3, fp32")
    a = _lattice_with_net(P)
    b = _lattice_with_net(padded(P))
    a.step(60)
    b.step(60)
    np.testing.assert_array_equal(a.populations(), b.populations())
    with pytest.raises(lbm.LbmError) as e:
        bad = dict(P)
        bad["w1"] = np.zeros((20, 28))
        bad["mu_in"], bad["sd_in"] = np.zeros(28), np.ones(28)
        _lattice_with_net(bad)
    assert e.value.status == lbm.LBM_EINVAL


# ---- two steps per launch with the neural outlet ------------------------------

@pytest.mark.parametrize("precision,mass_bound", [("fp64", 1e9), ("fp64", 3e-4), ("fp32", 3e-4)])
def test_nn_pairs_equal_single_steps(precision, mass_bound):
    # the outlet blocks of the two-step kernel run the single-step node code
    # and Eq. 16 with its fallback on the same network tiles, so both
    # schedules give the same populations bit for bit and the same fallback
    # counts, over odd counts and read-outs
    case = cases.ragged("mrt", "periodic")
    P = _f32(random_params(3, w_scale=0.5, out_sd=2e-4))
    _say("nn pairs vs single steps", precision, mass_bound)
    out = {}
    for launch in ("pairs", "pairs_held", "single"):
        g = lbm.Lattice(case["mask"], case["tau"], precision=precision, collision="mrt",
                        lateral="periodic", u_in=case["u_in"], noise_amp=case["noise_amp"],
                        seed=case["seed"], history_cap=81, launch=launch)
        g.set_outflow_nn(P, mass_bound=mass_bound)
        for n in (40, 7, 34):
            g.step(n)
        out[launch] = (g.populations(), g.forces().n_fallback, g.force_history())
    f1, n1, (fx1, _) = out["pairs"]
    f0, n0, (fx0, _) = out["single"]
    print("nn pairs vs single: populations that differ", np.count_nonzero(f1 != f0),
          "fallbacks", n1, n0, flush=True)
    np.testing.assert_array_equal(f1, f0)
    assert n1 == n0
    # the strips' other walk (stores held back one row): the same bits
    fh, nh, (fxh, _) = out["pairs_held"]
    np.testing.assert_array_equal(fh, f1)
    assert nh == n1
    np.testing.assert_array_equal(fxh, fx1)
    if mass_bound < 1:
        assert 0.1 * 81 * 77 < n0 < 0.9 * 81 * 77      # partial fallback
    # force partials are summed in another grouping (FP32: the one-step kernel
    # sums a wave's nodes in FP32 before the FP64 reduction)
    tol = 1e-12 if precision == "fp64" else 1e-5
    np.testing.assert_allclose(fx1, fx0, rtol=0, atol=tol * np.max(np.abs(fx0)) + 1e-15)


def test_nn_pairs_fp64_300_steps_against_oracle():
    case = cases.ragged("bgk", "periodic")
    P = _f32(random_params(3, w_scale=0.5, out_sd=2e-4))
    _say("nn pairs fp64 vs oracle, 300 steps")
    g = lbm.Lattice(case["mask"], case["tau"], precision="fp64", collision="bgk",
                    lateral="periodic", u_in=case["u_in"], noise_amp=case["noise_amp"],
                    seed=case["seed"], history_cap=300, launch="pairs")
    g.set_outflow_nn(P, mass_bound=1e9)
    g.step(300)
    o = Oracle(case["mask"], **cases.oracle_kwargs(case))
    o.set_outflow_nn(P, mass_bound=1e9)
    o.step(300)
    fl = case["mask"] == 0
    err = np.max(np.abs(g.populations()[:, fl] - o.post_collision()[:, fl]))
    print("nn pairs 300-step max abs error", err, flush=True)
    # corrections are ~2e-4; a BF16 flip moves one by <= 2^-8 of that
    assert err < 5e-6
    # the force moves with the populations near the body: 1e-6 of its scale
    fx, _ = g.force_history()
    np.testing.assert_allclose(fx, o.fx_hist, rtol=0, atol=1e-6 * np.max(np.abs(o.fx_hist)))


def test_nn_pairs_full_size():
    # the truncated-domain lattice 4096 x 512 (D = 64, periodic laterals,
    # MRT, FP32) with the neural outflow: four steps in two launches from the
    # same seeded smooth fields as the oracle
    nx, ny, D = 4096, 512, 64
    mask = geometry.cylinder(nx, ny, nx - 1 - 8 * D, ny // 2, D)
    tau = 3 * 0.05 * D / 200 + 0.5
    P = _f32(random_params(4, w_scale=0.5, out_sd=2e-4))
    _say("nn pairs full size 4096x512 fp32")
    rho, u = workloads.smooth_fields(mask.shape, 0.05, amp=0.02, seed=12)
    g = lbm.Lattice(mask, tau, precision="fp32", collision="mrt", lateral="periodic",
                    u_in=0.05, noise_amp=0.0, launch="pairs", history_cap=4)
    g.init_fields(rho, u[0], u[1])
    g.set_outflow_nn(P, mass_bound=1e9)
    g.step(4)
    o = Oracle(mask, tau, collision="mrt", lateral="periodic", u_in=0.05)
    o.set_equilibrium(rho, u[0], u[1])
    o.set_outflow_nn(P, mass_bound=1e9)
    o.step(4)
    fl = mask == 0
    err = np.max(np.abs(g.populations()[:, fl] - o.post_collision()[:, fl]))
    print("nn pairs full-size four-step error", err, flush=True)
    assert err < 1e-6
    fx, fy = g.force_history()
    np.testing.assert_allclose(fx, o.fx_hist, rtol=1e-5, atol=1e-9)


def test_nn_pairs_on_a_lattice_shorter_than_a_third_of_an_outlet_block():
    # 60 x 20 with periodic laterals: an outlet block's 64 rows wrap round
    # the lattice more than three times; pairs and single steps agree
    nx, ny = 60, 20
    mask = geometry.cylinder(nx, ny, 15, 9.5, 6.0)
    P = _f32(random_params(8, w_scale=0.5, out_sd=2e-4))
    _say("nn pairs, 60 x 20 periodic")
    out = {}
    for launch in ("pairs", "single"):
        g = lbm.Lattice(mask, 0.6, precision="fp64", collision="bgk", lateral="periodic",
                        u_in=0.05, noise_amp=1e-3, seed=3, launch=launch)
        g.set_outflow_nn(P, mass_bound=1e9)
        g.step(30)
        out[launch] = g.populations()
    fl = mask == 0
    err = np.max(np.abs(out["pairs"][:, fl] - out["single"][:, fl]) / np.abs(out["single"][:, fl]))
    assert err < 1e-12, err
