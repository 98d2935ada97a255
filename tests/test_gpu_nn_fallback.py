"""GPU parity of the neural outflow (Sec. 3.1, Eq. 16) when only some outlet
rows keep the reconstruction and the rest fall back to Zou & He (reading
R17: positivity of g_3, g_6, g_7 and the density jump |rho_g - rho(L-1)|
against the bound delta_m).

Decisions.  Both sides take the decision in the kernel's precision (FP32
positivity, FP32 difference of the density offsets), but their inputs differ
slightly: the GPU accumulates the network in FP32 (the oracle in FP64) and an
FP32 lattice rounds the populations it stores.  A row may therefore decide
differently only when its jump lies within that difference of the bound (or
a reconstructed population within it of zero).  ``band`` gives that width
per row: the difference of the corrections s, measured by evaluating the
library's network (lbm_mlp_forward, the same MFMA tiles and roundings as the
fused outlet) on the oracle's features and itself checked against the
network's error bound (tests/nn_bounds.py), plus the FP32 rounding of the
two density offsets and of their difference, plus the storage rounding of
the 18 populations involved.  Every test counts the rows in the band and
requires the decisions outside it to agree exactly.

Single-step cases write the oracle's own state (never a GPU state) into the
library, take one step, and identify each outlet row's choice from its
post-collision populations: the row must match one of the oracle's two
candidates (reconstruction kept, Zou & He fallback) within the step's
tolerance, and the two must be farther apart than twice that tolerance."""
import numpy as np
import pytest

import cases
import nn_bounds
from oracle.d2q9 import W
from oracle.solver import Lattice as Oracle
from paper_2506_05293_amd import geometry, lbm, workloads

pytestmark = pytest.mark.gpu

BOUND = 3e-4          # delta_m of the truncated-domain studies
ULP32 = 2.0**-24      # unit roundoff of FP32


def _say(*a):
    print("[gpu case]", *a, flush=True)


def _net(seed=3, out_sd=2e-4):
    return cases.f32_values(cases.random_params(seed, w_scale=0.5, out_sd=out_sd))


def _features(o, fstar):
    fnew = o.stream(np.asarray(fstar, np.float64))
    L = o.nx - 1
    return fnew, np.concatenate([(fnew[:, :, L - 1 - j] - W[:, None]).T for j in range(3)], axis=1)


def gpu_corrections(g, feats):
    """The library's network on the given feature rows (FP32 in, FP32 out)."""
    import torch
    x = torch.from_numpy(np.ascontiguousarray(feats, np.float32)).cuda()
    s = torch.zeros((feats.shape[0], 3), dtype=torch.float32, device="cuda")
    lbm.lbm_mlp_forward(g.ctx, x.data_ptr(), s.data_ptr(), feats.shape[0])
    torch.cuda.synchronize()
    return s.cpu().numpy().astype(np.float64)


def band(o, fstar, P, precision, s_gpu):
    """Per-row width around the bound (density test) and around zero
    (positivity) within which GPU and oracle may decide differently."""
    fnew, feats = _features(o, fstar)
    L = o.nx - 1
    from oracle.mlp import forward_bf16
    s_or = forward_bf16(feats, P)
    bound, _ = nn_bounds.output_bound(feats, P)
    ds = np.abs(s_gpu - s_or)
    assert np.all(ds <= bound + 1e-12), np.max(ds / (bound + 1e-30))
    r = o.nn_outlet(fnew)
    dg = np.abs((r["nn"] - W[:, None]).sum(0))
    dp = np.abs((fnew[:, :, L - 1] - W[:, None]).sum(0))
    store = 0.0
    if precision != "fp64":
        # the populations the GPU pulled into columns L-1 and L are the
        # written state rounded to the storage precision: 2^-24 (FP32) or
        # 2^-11 (FP16) of each offset (the unknowns at L are NaN here)
        u = ULP32 if precision == "fp32" else 2.0**-11
        off = np.abs(fnew[:, :, L - 1:L + 1] - W[:, None, None])
        store = 2 * u * np.nansum(off, axis=(0, 2))
    dens = ds.sum(1) + 2 * ULP32 * (dg + dp + r["jump"]) + store + 1e-15
    pos = ds.max(1) + 2 * ULP32 * np.max(np.abs(r["nn"][[3, 6, 7]]), axis=0) + store + 1e-15
    return r, dens, pos


def in_band(r, dens, pos, mass_bound):
    g = r["nn"][[3, 6, 7]]
    near_zero = np.any(np.abs(g) <= pos[None], axis=0)
    return (np.abs(r["jump"] - np.float32(mass_bound)) <= dens) | near_zero


def gpu_choices(col, cand, tol):
    """Per row: 1 the GPU kept the reconstruction, 0 it fell back, -1 it
    matches neither candidate within tol, -2 the candidates are too close
    to tell apart."""
    d_nn = np.max(np.abs(col - cand["post_nn"]), axis=0)
    d_zh = np.max(np.abs(col - cand["post_zh"]), axis=0)
    sep = np.max(np.abs(cand["post_nn"] - cand["post_zh"]), axis=0)
    out = np.where(d_nn <= tol, 1, np.where(d_zh <= tol, 0, -1))
    return np.where(sep <= 2 * tol, -2, out), d_nn, d_zh


def _check_step(o, fstar, P, precision, mass_bound, g, tol, label):
    """One GPU step from the oracle's post-collision state fstar; compares
    every row's decision and the whole post-collision state."""
    cand = o.nn_outlet_candidates(fstar)
    _, feats = _features(o, fstar)
    r, dens, pos = band(o, fstar, P, precision, gpu_corrections(g, feats))
    g.write_populations(fstar)
    n0 = g.forces().n_fallback
    g.step(1)
    f = g.populations()
    choice, d_nn, d_zh = gpu_choices(f[:, :, -1], cand, tol)
    fluid = o.fluid[:, -1]
    ok = cand["ok"]
    near = in_band(r, dens, pos, mass_bound)
    known = fluid & (choice >= 0)
    mism = known & (choice != ok.astype(int))
    frac = 1.0 - ok[fluid].mean()
    print(f"{label}: fallback fraction {frac:.2f}, rows in the band {int(near[fluid].sum())}, "
          f"mismatches {int(mism.sum())} (in band {int((mism & near).sum())}), "
          f"unidentified {int((fluid & (choice == -1)).sum())}, "
          f"too close {int((fluid & (choice == -2)).sum())}", flush=True)
    assert not np.any(fluid & (choice == -1)), (np.flatnonzero(fluid & (choice == -1)),
                                               d_nn[choice == -1], d_zh[choice == -1])
    assert not np.any(mism & ~near), np.flatnonzero(mism & ~near)
    # the fallback count of the step
    n_gpu = g.forces().n_fallback - n0
    n_or = int((~ok & fluid).sum())
    assert abs(n_gpu - n_or) <= int((mism & near).sum()), (n_gpu, n_or)
    # every node away from the outlet, and the outlet rows that decided alike
    ref, _ = o.advance_post(fstar)
    fl = o.fluid.copy()
    fl[:, -1] &= ~mism
    err = np.max(np.abs(f[:, fl] - ref[:, fl]))
    assert err < tol, err
    return frac, int(near[fluid].sum()), int(mism.sum())


def _ragged_gpu(case, precision, P, mass_bound):
    g = lbm.Lattice(case["mask"], case["tau"], precision=precision, collision=case["collision"],
                    lateral=case["lateral"], u_in=case["u_in"])
    g.set_outflow_nn(P, mass_bound=mass_bound)
    return g


@pytest.mark.parametrize("precision,tol", [("fp64", 5e-6), ("fp32", 5e-6)])
def test_partial_fallback_decisions_ragged(precision, tol):
    # the ragged 203 x 77 lattice (BGK, periodic laterals, a body touching the
    # edges) with a random 27-64-64-3 network at delta_m = 3e-4: the oracle
    # runs 150 steps and every 30th state is handed to the GPU for one step
    case = cases.ragged("bgk", "periodic")
    P = _net()
    o = Oracle(case["mask"], **cases.oracle_kwargs(case))
    o.set_outflow_nn(P, mass_bound=BOUND)
    _say("partial fallback decisions, ragged", precision)
    g = _ragged_gpu(case, precision, P, BOUND)
    fracs, nears, mis = [], 0, 0
    for k in range(5):
        o.step(30)
        fr, nr, m = _check_step(o, o.post_collision(), P, precision, BOUND, g, tol,
                                f"ragged {precision} step {o.t}")
        fracs.append(fr)
        nears += nr
        mis += m
    print("fallback fractions", np.round(fracs, 2), "rows in band", nears, "mismatches", mis)
    assert 0.2 <= np.mean(fracs) <= 0.8
    if precision == "fp64":
        assert mis == 0


def test_partial_fallback_positivity_only():
    # the density test switched off (delta_m = 1e9); a network whose first
    # correction takes g_3 = f_3(L-1) + s_3 through zero in about half of the
    # rows (mu_out[0] near -f_3), FP64
    case = cases.ragged("bgk", "periodic")
    P = cases.f32_values(cases.random_params(5, w_scale=0.5, out_sd=5e-4))
    P["mu_out"] = np.array([-0.09235, 0.0, 0.0])
    o = Oracle(case["mask"], **cases.oracle_kwargs(case))
    o.step(60)
    o.set_outflow_nn(P, mass_bound=1e9)
    _say("partial fallback, positivity only")
    g = _ragged_gpu(case, "fp64", P, 1e9)
    fr, _, m = _check_step(o, o.post_collision(), P, "fp64", 1e9, g, 5e-6, "positivity only")
    assert 0.2 <= fr <= 0.8 and m == 0


def test_partial_fallback_run_fp64():
    # 100 steps of the ragged lattice with delta_m = 3e-4, both sides from the
    # same seeded noise: the fallback counts agree exactly and the state to
    # the neural outflow's tolerance (corrections ~2e-4; a BF16 flip moves
    # one by <= 2^-8 of that)
    case = cases.ragged("bgk", "periodic")
    P = _net()
    _say("partial fallback run fp64, 100 steps")
    g = lbm.Lattice(case["mask"], case["tau"], precision="fp64", collision="bgk",
                    lateral="periodic", u_in=case["u_in"], noise_amp=case["noise_amp"],
                    seed=case["seed"], history_cap=100)
    g.set_outflow_nn(P, mass_bound=BOUND)
    g.step(100)
    o = Oracle(case["mask"], **cases.oracle_kwargs(case))
    o.set_outflow_nn(P, mass_bound=BOUND)
    o.step(100)
    ny = case["mask"].shape[0]
    n_gpu = g.forces().n_fallback
    print("fallbacks gpu", n_gpu, "oracle", o.n_fallback, "of", 100 * ny, flush=True)
    assert 0.2 * 100 * ny <= o.n_fallback <= 0.8 * 100 * ny
    assert n_gpu == o.n_fallback
    fl = case["mask"] == 0
    err = np.max(np.abs(g.populations()[:, fl] - o.post_collision()[:, fl]))
    print("max abs error", err, flush=True)
    assert err < 5e-6
    fx, _ = g.force_history()
    np.testing.assert_allclose(fx, o.fx_hist, rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-6), ("fp64", 1e-6)])
def test_partial_fallback_full_size(precision, tol, mass_bound=BOUND):
    # the truncated-domain lattice of the outflow study, 4096 x 512 (D = 64,
    # periodic laterals, MRT), from seeded smooth fields, one step; with
    # corrections of ~1e-3 the jumps spread around delta_m = 3e-4 (quartiles
    # 2.1e-4 and 3.5e-4), so part of the 512 rows falls back
    nx, ny, D = 4096, 512, 64
    mask = geometry.cylinder(nx, ny, nx - 1 - 8 * D, ny // 2, D)
    tau = 3 * 0.05 * D / 200 + 0.5
    P = _net(4, out_sd=1e-3)
    rho, u = workloads.smooth_fields(mask.shape, 0.05, amp=0.02, seed=12)
    o = Oracle(mask, tau, collision="mrt", lateral="periodic", u_in=0.05)
    o.set_equilibrium(rho, u[0], u[1])
    o.set_outflow_nn(P, mass_bound=mass_bound)
    _say("partial fallback full size 4096x512", precision)
    g = lbm.Lattice(mask, tau, precision=precision, collision="mrt", lateral="periodic", u_in=0.05)
    g.set_outflow_nn(P, mass_bound=mass_bound)
    fr, _, _ = _check_step(o, o.post_collision(), P, precision, mass_bound, g, tol,
                           "4096x512 " + precision)
    assert 0.2 <= fr <= 0.8
