"""GPU tests of the batched persistent launch (include/lbm_batch.h).

A lattice of a batch must evolve bit for bit like the same lattice stepped
alone (FP32 offsets, vector tile: the same node code), whatever the other
lattices do; its force history agrees to FP32 summation order.  Logged
samples are the pulled populations of the logging step: bit for bit the
permutation of the state read back just before it (a copy, checked by
index), and within FP32 rounding the oracle's own run from the same seeded
start."""
import numpy as np
import pytest

from oracle.d2q9 import W
from oracle.solver import Lattice as Oracle
from paper_2506_05293_amd import geometry, lbm

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu case]", *a, flush=True)


def _lattices():
    return [
        dict(mask=geometry.cylinder(203, 77, 51.3, 37.6, 17.0), tau=0.56, u_in=0.06, seed=7),
        dict(mask=geometry.cylinder(300, 64, 60, 31.5, 16.0), tau=0.6, u_in=0.05, seed=8),
        dict(mask=np.zeros((96, 150), np.uint8), tau=0.7, u_in=0.04, seed=9),
        dict(mask=geometry.cylinder(520, 160, 80, 80, 40.0), tau=0.55, u_in=0.05, seed=10),
    ]


LAUNCHES = ["persistent", "per_step"]


@pytest.mark.parametrize("launch", LAUNCHES)
@pytest.mark.parametrize("collision,lateral", [("mrt", "periodic"), ("bgk", "walls")])
def test_batch_equals_single_lattices(collision, lateral, launch, monkeypatch):
    # the batch kernel runs the single-step node code: single lattices
    # with one launch per step are its bitwise reference
    monkeypatch.setitem(lbm.LATTICE_DEFAULTS, "schedule", "vector")
    monkeypatch.setitem(lbm.LATTICE_DEFAULTS, "launch", "single")
    lats = _lattices()
    _say("batch vs single", collision, lateral, launch)
    b = lbm.Batch(lats, collision=collision, lateral=lateral, noise_amp=1e-3, history_cap=200,
                  launch=launch)
    b.step(70)
    b.step(130)
    for i, L in enumerate(lats):
        g = lbm.Lattice(L["mask"], L["tau"], precision="fp32", collision=collision, lateral=lateral,
                        u_in=L["u_in"], noise_amp=1e-3, seed=L["seed"], history_cap=200)
        g.step(200)
        np.testing.assert_array_equal(b.populations(i), g.populations())
        bx, by = b.force_history(i)
        gx, gy = g.force_history()
        assert len(bx) == 200
        scale = np.max(np.abs(gx)) + 1e-30
        assert np.max(np.abs(bx - gx)) < 1e-5 * scale and np.max(np.abs(by - gy)) < 1e-5 * scale
        fb, fg = b.forces(i), g.forces()
        assert abs(fb.mass - fg.mass) < 1e-9 * fg.mass and fb.step == 200
    assert not b.retired().any()


@pytest.mark.parametrize("launch", LAUNCHES)
def test_logging_matches_pull_of_read_state(launch):
    # a source lattice (logged at an interior cut column) and its truncated
    # twin (logged at its outlet), rows aligned
    D = 16
    ny = 8 * D
    x_cut = 4 * D + 10 * D
    long_mask = geometry.cylinder(4 * D + 20 * D, ny, 4 * D, ny // 2, D)
    short_mask = geometry.cylinder(x_cut + 1, ny, 4 * D, ny // 2, D)
    lats = [dict(mask=long_mask, tau=0.56, seed=3, log_role=1, log_x=x_cut, log_row0=0),
            dict(mask=short_mask, tau=0.56, seed=3, log_role=2, log_x=x_cut, log_row0=0)]
    _say("batch logging", launch)
    b = lbm.Batch(lats, collision="mrt", lateral="periodic", noise_amp=1e-3,
                  log_start=5, log_every=3, log_slots=2, log_rows=ny, launch=launch)

    cx = [0, 1, 0, -1, 0, 1, -1, -1, 1]
    cy = [0, 0, 1, 0, -1, 1, 1, -1, -1]

    def pull(f):
        # the logged columns are interior and free of solids, the rows
        # periodic: population q of node (x, y) is f_q(x - c_x, y - c_y)
        return np.stack([np.roll(np.roll(f[q], cy[q], axis=0), cx[q], axis=1)
                         for q in range(9)]) - W[:, None, None]                   # offsets
    oracles = [Oracle(L["mask"], L["tau"], collision="mrt", lateral="periodic", u_in=0.05,
                      noise_amp=1e-3, seed=L["seed"]) for L in lats]
    expect, indep = [], []
    b.step(5)                     # the next step (5 taken before it) logs slot 0
    expect.append([pull(b.populations(i)) for i in range(2)])
    for o in oracles:
        o.step(5)
    indep.append([pull(o.post_collision()) for o in oracles])
    b.step(3)                     # ... and the step after 8 logs slot 1
    expect.append([pull(b.populations(i)) for i in range(2)])
    for o in oracles:
        o.step(3)
    indep.append([pull(o.post_collision()) for o in oracles])
    b.step(21)                    # two slots only: nothing more is logged
    x, xa, t = (v.cpu().numpy() for v in b.dataset())
    assert x.shape == (2 * ny, 27) and t.shape == (2 * ny, 3)
    for k, (pl, ps) in enumerate(expect):
        rows = slice(k * ny, (k + 1) * ny)
        for j in range(3):
            col = x_cut - 1 - j
            np.testing.assert_array_equal(x[rows, 9 * j:9 * j + 9], pl[:, :, col].T.astype(np.float32))
            np.testing.assert_array_equal(xa[rows, 9 * j:9 * j + 9], ps[:, :, col].T.astype(np.float32))
        want = (pl[[3, 6, 7], :, x_cut].T.astype(np.float32) -
                pl[[3, 6, 7], :, x_cut - 1].T.astype(np.float32))
        np.testing.assert_array_equal(t[rows], want)
        # the same samples from the oracle's own runs (FP64 against FP32 offsets)
        ol, os_ = indep[k]
        for j in range(3):
            col = x_cut - 1 - j
            np.testing.assert_allclose(x[rows, 9 * j:9 * j + 9], ol[:, :, col].T, rtol=0, atol=2e-7)
            np.testing.assert_allclose(xa[rows, 9 * j:9 * j + 9], os_[:, :, col].T, rtol=0,
                                       atol=2e-7)


@pytest.mark.parametrize("launch", LAUNCHES)
def test_unstable_lattice_is_retired_alone(launch, monkeypatch):
    # the batch kernel runs the single-step node code: single lattices
    # with one launch per step are its bitwise reference
    monkeypatch.setitem(lbm.LATTICE_DEFAULTS, "schedule", "vector")
    monkeypatch.setitem(lbm.LATTICE_DEFAULTS, "launch", "single")
    lats = _lattices()[:2]
    bad = dict(mask=geometry.cylinder(200, 60, 40, 30, 20.0), tau=0.5005, u_in=0.3, seed=1)
    _say("batch retirement", launch)
    b = lbm.Batch(lats + [bad], collision="bgk", lateral="walls", noise_amp=1e-2, history_cap=400,
                  launch=launch)
    b.step(400)
    flags = b.retired()
    assert list(flags) == [0, 0, 1]
    with pytest.raises(lbm.LbmError) as e:
        b.forces(2)
    assert e.value.status == lbm.LBM_EUNSTABLE
    for i, L in enumerate(lats):
        g = lbm.Lattice(L["mask"], L["tau"], precision="fp32", collision="bgk", lateral="walls",
                        u_in=L["u_in"], noise_amp=1e-2, seed=L["seed"])
        g.step(400)
        np.testing.assert_array_equal(b.populations(i), g.populations())


def test_barrier_wait_bound_is_reported():
    # a one-poll wait bound makes the grid barrier give up; every workgroup
    # leaves and the next synchronising call reports the failure
    _say("batch barrier bound")
    b = lbm.Batch(_lattices(), collision="mrt", lateral="periodic", spin_limit=1,
                  launch="persistent")
    b.step(50)
    with pytest.raises(lbm.LbmError) as e:
        b.forces(0)
    assert e.value.status == lbm.LBM_EHIP


def test_persistent_grid_beyond_residency_is_rejected():
    # the persistent grid must be co-resident: asking for more workgroups per
    # CU than the kernel's registers and LDS let a CU hold is an argument
    # error at creation, not a barrier that never completes
    _say("batch groups_per_cu beyond residency")
    with pytest.raises(lbm.LbmError) as e:
        lbm.Batch(_lattices(), collision="mrt", lateral="periodic", launch="persistent",
                  groups_per_cu=64)
    assert e.value.status == lbm.LBM_EINVAL
    b = lbm.Batch(_lattices(), collision="mrt", lateral="periodic", launch="persistent",
                  groups_per_cu=2)
    b.step(4)
    assert b.forces(0).step == 4


def test_batch_solid_nodes_survive_read_out():
    lats = _lattices()
    _say("batch solid nodes after read-out")
    b = lbm.Batch(lats, collision="mrt", lateral="periodic", noise_amp=1e-3)
    f0 = [b.populations(i) for i in range(len(lats))]
    for _ in range(3):
        b.step(1)
        for i, L in enumerate(lats):
            f = b.populations(i)
            solid = L["mask"] != 0
            np.testing.assert_array_equal(f[:, solid], f0[i][:, solid])
            assert np.isfinite(f).all()


@pytest.mark.parametrize("launch", LAUNCHES)
def test_full_training_batch_against_oracle(launch):
    # the data-generation batch itself: 64 cylinder pairs (128 lattices,
    # 33.4M nodes) in one persistent launch, FP32, MRT with the study rates;
    # three steps, then the first pair and the largest lattice against the
    # oracle's own runs from the same seeded start
    from paper_2506_05293_amd import workloads
    lats, _, _ = workloads.training_pairs(64, 3)
    lats = [dict(L, log_role=0) for L in lats]             # no logging here
    _say("batch full size", len(lats), "lattices", launch)
    rates = dict(s_e=1.0, s_eps=1.0, s_q=1.0)
    b = lbm.Batch(lats, collision="mrt", lateral="periodic", noise_amp=1e-4, launch=launch, **rates)
    b.step(3)
    big = int(np.argmax([L["mask"].size for L in lats]))
    for i in (0, 1, big):
        L = lats[i]
        o = Oracle(L["mask"], L["tau"], collision="mrt", lateral="periodic", u_in=L["u_in"],
                   noise_amp=1e-4, seed=L["seed"], **rates)
        o.step(3)
        fl = L["mask"] == 0
        err = np.max(np.abs(b.populations(i)[:, fl] - o.post_collision()[:, fl]))
        print("lattice", i, L["mask"].shape, "three-step error", err, flush=True)
        assert err < 5e-8
    assert not np.any(b.retired())
