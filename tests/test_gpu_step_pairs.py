"""GPU parity of the two-steps-per-launch path of the step
(params.launch = LBM_LAUNCH_PAIRS, and the default for the outflows and
precisions without a three-step form; LBM_LAUNCH_SINGLE gives one launch
per step).  Every node takes the single-step node code in registers with the
same explicit fused multiply-adds, and the state between the two steps is
rounded to the storage precision as a store and reload would round it, so
the populations equal those of one launch per step bit for bit in FP64,
FP32 and FP16 over odd step counts and read-outs.  The force and mass
partials are summed in another grouping: the force history agrees to 1e-12
of its scale in FP64 and 1e-5 in FP32 and FP16 (the one-step kernel adds a
wave's node terms in FP32 first).  The two walks of the strips (the stores
of a row held back one row, or not; LBM_LAUNCH_PAIRS_HELD and
LBM_LAUNCH_PAIRS_PLAIN force one) give the same populations and the same
force history bit for bit.  Against the oracle as the single-step path."""
import numpy as np
import pytest

import cases
from oracle.solver import Lattice as Oracle
from paper_2506_05293_amd import lbm, workloads

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu case]", *a, flush=True)


def _gpu(case, precision, history_cap, launch="pairs"):
    return lbm.Lattice(case["mask"], case["tau"], precision=precision,
                       collision=case["collision"], lateral=case["lateral"],
                       u_in=case["u_in"], noise_amp=case["noise_amp"], seed=case["seed"],
                       history_cap=history_cap, launch=launch)


def _run(case, precision, steps, pairs, chunks=(None,)):
    g = _gpu(case, precision, steps, "pairs" if pairs else "single")
    for n in chunks:
        g.step(n if n is not None else steps)
    return g.populations(), g.force_history()


@pytest.mark.parametrize("name,precision", [("c1_bgk", "fp64"), ("ragged_mrt_periodic", "fp64"),
                                            ("ragged_mrt_walls", "fp32"), ("c1_mrt", "fp16")])
def test_pairs_equal_single_steps(name, precision):
    case = {"c1_bgk": cases.c1(75.0), "ragged_mrt_periodic": cases.ragged("mrt", "periodic"),
            "ragged_mrt_walls": cases.ragged("mrt", "walls"), "c1_mrt": cases.c1(100.0, "mrt")}[name]
    _say("pairs vs single steps", name, precision)
    # odd counts and read-outs in between: pairs, a single step, pairs again
    chunks = (40, 7, 34)
    f1, (fx1, fy1) = _run(case, precision, 81, True, chunks)
    f0, (fx0, fy0) = _run(case, precision, 81, False, chunks)
    # every kernel runs the same node arithmetic (explicit fused multiply-adds,
    # no contraction, FP16 rounding of the state between the two steps of a
    # launch), so the populations are equal bit for bit in every precision
    diff = np.count_nonzero(f1 != f0)
    print("pairs vs single steps: populations that differ", diff, flush=True)
    np.testing.assert_array_equal(f1, f0)
    assert len(fx1) == 81
    # the forces: the same node terms summed in other groups (strips of the
    # two-step kernel, tiles of the one-step kernel); in FP32 and FP16 the
    # one-step kernel adds a wave's node terms in FP32 before its FP64
    # reduction (measured 5e-6 of the largest |F_x| at FP32, 3e-7 at FP16)
    tol = 1e-12 if precision == "fp64" else 1e-5
    scale = max(np.max(np.abs(fx0)), 1e-9)
    print("force history: max difference / scale", np.max(np.abs(fx1 - fx0)) / scale, flush=True)
    np.testing.assert_allclose(fx1, fx0, rtol=0, atol=tol * scale)
    np.testing.assert_allclose(fy1, fy0, rtol=0, atol=tol * scale)


@pytest.mark.parametrize("name,precision", [("c1_bgk", "fp64"), ("ragged_mrt_periodic", "fp32"),
                                            ("ragged_mrt_walls", "fp64"), ("c1_mrt", "fp32")])
def test_held_walk_equals_plain_walk(name, precision):
    # the two walks of the two-step kernel differ only in when a row's
    # stores are issued and how the link flags are read: the same
    # populations and the same force partials, bit for bit
    case = {"c1_bgk": cases.c1(75.0), "ragged_mrt_periodic": cases.ragged("mrt", "periodic"),
            "ragged_mrt_walls": cases.ragged("mrt", "walls"), "c1_mrt": cases.c1(100.0, "mrt")}[name]
    _say("held vs plain walk", name, precision)
    out = {}
    for launch in ("pairs_held", "pairs_plain"):
        g = _gpu(case, precision, 81, launch)
        for n in (40, 7, 34):
            g.step(n)
        out[launch] = (g.populations(), g.force_history())
    (f1, (fx1, fy1)), (f0, (fx0, fy0)) = out["pairs_held"], out["pairs_plain"]
    print("held vs plain: populations that differ", np.count_nonzero(f1 != f0), flush=True)
    np.testing.assert_array_equal(f1, f0)
    np.testing.assert_array_equal(fx1, fx0)
    np.testing.assert_array_equal(fy1, fy0)


def test_held_walk_full_size_by_default():
    # 4096 x 1536 FP32 holds 226 MB per population buffer, past the size
    # from which the default two-step launch holds its stores: four steps
    # equal four single-step launches bit for bit
    case = cases.c2(4096, 1536)
    _say("held walk by default, 4096 x 1536 fp32")
    rho, u = workloads.smooth_fields(case["mask"].shape, case["u_in"], amp=0.02, seed=17)
    out = {}
    for launch in ("pairs", "single"):
        g = _gpu(case, "fp32", 4, launch)
        g.init_fields(rho, u[0], u[1])
        g.step(4)
        out[launch] = g.populations()
        del g
    print("populations that differ", np.count_nonzero(out["pairs"] != out["single"]), flush=True)
    np.testing.assert_array_equal(out["pairs"], out["single"])


def test_pairs_fp64_against_oracle():
    case = cases.c1(75.0)
    _say("pairs c1 fp64 vs oracle, 300 steps")
    f, (fx, fy) = _run(case, "fp64", 300, True)
    o = Oracle(case["mask"], **cases.oracle_kwargs(case))
    o.step(300)
    fl = case["mask"] == 0
    ref = o.post_collision()
    err = np.max(np.abs(f[:, fl] - ref[:, fl]) / np.abs(ref[:, fl]))
    print("max rel error", err, flush=True)
    assert err < 1e-12
    np.testing.assert_allclose(fx, o.fx_hist, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(fy, o.fy_hist, rtol=1e-10, atol=1e-12)


def test_pairs_full_size_c2():
    # the bench lattice, FP32 offsets, MRT: four steps (two launches) from
    # the same smooth fields as the oracle
    case = cases.c2()
    _say("pairs c2 full size fp32")
    rho, u = workloads.smooth_fields(case["mask"].shape, case["u_in"], amp=0.02, seed=17)
    g = _gpu(case, "fp32", 4)
    g.init_fields(rho, u[0], u[1])
    g.step(4)
    o = Oracle(case["mask"], **cases.oracle_kwargs(case))
    o.set_equilibrium(rho, u[0], u[1])
    o.step(4)
    fl = case["mask"] == 0
    err = np.max(np.abs(g.populations()[:, fl] - o.post_collision()[:, fl]))
    print("c2 four-step max abs error", err, flush=True)
    assert err < 5e-8
    fx, fy = g.force_history()
    np.testing.assert_allclose(fx, o.fx_hist, rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(fy, o.fy_hist, rtol=1e-5, atol=1e-7)
