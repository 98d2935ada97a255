"""Pins of the oracle's closed-loop training of the tuning network (Sec. 4.2).

The torch re-expression of the step is fixed to the numpy solver (itself
pinned on its own); its reverse-mode gradient to central finite differences
of the numpy solver's loss; the loss normalisation and the loss region to
closed forms; the free stream to a zero loss and a zero gradient; and the
dependence cone that lets a segment be advanced on a strip of 2 n_t + 3
columns to exact invariance under changes further upstream."""
import numpy as np
import pytest
import torch

from oracle import cbc_train, d2q9
from oracle.d2q9 import CS2
from oracle.solver import Lattice

CS = np.sqrt(CS2)
NX, NY, TAU, U0 = 40, 22, 0.6, 0.1
CFG = dict(tau=TAU, u_in=U0, mach=U0 / CS, length=float(NX), rho_inf=1.0)


def _net(seed):
    rng = np.random.default_rng(seed)
    return {"w1": 0.5 * rng.standard_normal((20, 9)), "b1": 0.3 * rng.standard_normal(20),
            "w2": 0.3 * rng.standard_normal((20, 20)), "b2": 0.3 * rng.standard_normal(20),
            "w3": 0.5 * rng.standard_normal((2, 20)), "b3": 0.3 * rng.standard_normal(2),
            "mu_in": 1e-5 * rng.standard_normal(9), "sd_in": np.full(9, 3e-4),
            "leaky_slope": 0.01, "sigma_scale": 1.0, "sigma_shift": 0.0,
            "kappa_scale": 0.8, "kappa_shift": 0.1}


def _oracle(net, cbc=True):
    lat = Lattice(np.zeros((NY, NX), np.uint8), TAU, lateral="periodic", u_in=U0)
    if cbc:
        lat.set_outflow_cbc(net=net, mach=CFG["mach"], length=NX)
    return lat


def _state(seed=0, steps=6):
    """A post-collision state with a vortex at the outlet (numpy solver)."""
    y, x = np.mgrid[0:NY, 0:NX].astype(float)
    xc, yc, rc, b = NX - 6.5 + 0.3 * seed, NY / 2 - 0.4, 4.0, 0.4
    r2 = (x - xc) ** 2 + (y - yc) ** 2
    e = np.exp(-r2 / (2 * rc**2))
    lat = _oracle(None, cbc=False)
    lat.set_outflow_cbc(sigma=0.3, kappa2=0.2, mach=CFG["mach"], length=NX)
    lat.set_equilibrium(np.exp(-(b * U0) ** 2 / (2 * CS2) * np.exp(-r2 / rc**2)),
                        U0 - b * U0 * (y - yc) / rc * e, b * U0 * (x - xc) / rc * e)
    lat.step(steps)
    return lat.post_collision()


def _ref(a0, n_t):
    """Reference moments: the same state advanced by the Zou & He outlet."""
    lat = _oracle(None, cbc=False)
    a = a0
    for _ in range(n_t):
        a, _ = lat.advance_post(a)
    return np.stack(d2q9.moments(a[:, :, -n_t:]))


def _np_loss(segments, net):
    """The segment loss evaluated with the numpy solver."""
    tot = 0.0
    for a0, ref in segments:
        n_t = ref.shape[2]
        lat = _oracle(net)
        a = a0
        for _ in range(n_t):
            a, _ = lat.advance_post(a)
        rho, u, v = d2q9.moments(a[:, :, -n_t:])
        tot += np.mean((rho - ref[0]) ** 2) + np.mean((u - ref[1]) ** 2 + (v - ref[2]) ** 2)
    return tot / len(segments)


@pytest.mark.parametrize("n_t", [1, 4, 7])
def test_rollout_matches_numpy_solver(n_t):
    net = _net(1)
    a0 = _state()
    states = cbc_train.rollout(a0, cbc_train._theta(net, False), net, CFG, n_t)
    lat = _oracle(net)
    a = a0
    for k in range(n_t):
        a, _ = lat.advance_post(a)
        np.testing.assert_allclose(states[k + 1].numpy(), a, rtol=0, atol=2e-15)
    np.testing.assert_allclose(states[-1].numpy(), a, rtol=0, atol=2e-15)


def test_gradient_matches_finite_differences():
    net = _net(2)
    segs = [(_state(0), _ref(_state(0), 3)), (_state(1, 8), _ref(_state(1, 8), 5))]
    loss, g = cbc_train.loss_and_grad(segs, net, CFG)
    assert loss == pytest.approx(_np_loss(segs, net), rel=1e-12)
    rng = np.random.default_rng(7)
    h = 1e-6
    for trial in range(3):
        d = {k: rng.standard_normal(np.shape(net[k])) for k in cbc_train.PARAMS}
        plus = dict(net, **{k: net[k] + h * d[k] for k in cbc_train.PARAMS})
        minus = dict(net, **{k: net[k] - h * d[k] for k in cbc_train.PARAMS})
        fd = (_np_loss(segs, plus) - _np_loss(segs, minus)) / (2 * h)
        ad = sum(float(np.sum(g[k] * d[k])) for k in cbc_train.PARAMS)
        assert ad == pytest.approx(fd, rel=1e-6), (trial, ad, fd)
    # single output-layer entries (smooth: no LeakyReLU after them, so a
    # wide step keeps the rounding of the loss out of the difference, and
    # Richardson extrapolation over H and H/2 removes the O(H^2) term; the
    # sigma output's derivative is 2000 times smaller than kappa_2's here)
    def central(k, e, H):
        return (_np_loss(segs, dict(net, **{k: net[k] + H * e})) -
                _np_loss(segs, dict(net, **{k: net[k] - H * e}))) / (2 * H)
    H = 1e-3
    for k, idx in (("b3", (0,)), ("b3", (1,)), ("w3", (1, 4)), ("w3", (0, 7))):
        e = np.zeros(np.shape(net[k]))
        e[idx] = 1.0
        fd = (4 * central(k, e, H / 2) - central(k, e, H)) / 3
        assert g[k][idx] == pytest.approx(fd, rel=1e-6), (k, idx)
    assert abs(g["b3"][0]) > 0 and abs(g["b3"][1]) > 0


def test_segments_with_their_own_relaxation_and_mach():
    # a segment may carry its own configuration (tau, inflow, Mach number):
    # the mixed set's loss is the numpy solver's with each segment on a
    # lattice of its own parameters, and its gradient the mean of the
    # segments' own gradients
    net = _net(4)
    u1 = 0.06
    cfg1 = dict(CFG, tau=0.72, u_in=u1, mach=u1 / CS)
    a, b = _state(0), _state(1, 8)
    ref_a, ref_b = _ref(a, 4), _ref(b, 3)
    loss, g = cbc_train.loss_and_grad([(a, ref_a), (b, ref_b, cfg1)], net, CFG)

    def np_seg(a0, ref, tau, u_in, mach):
        lat = Lattice(np.zeros((NY, NX), np.uint8), tau, lateral="periodic", u_in=u_in)
        lat.set_outflow_cbc(net=net, mach=mach, length=NX)
        st = a0
        for _ in range(ref.shape[2]):
            st, _ = lat.advance_post(st)
        rho, u, v = d2q9.moments(st[:, :, -ref.shape[2]:])
        return np.mean((rho - ref[0]) ** 2) + np.mean((u - ref[1]) ** 2 + (v - ref[2]) ** 2)
    want = 0.5 * (np_seg(a, ref_a, TAU, U0, CFG["mach"]) + np_seg(b, ref_b, 0.72, u1, u1 / CS))
    assert loss == pytest.approx(want, rel=1e-12)
    la, ga = cbc_train.loss_and_grad([(a, ref_a)], net, CFG)
    lb, gb = cbc_train.loss_and_grad([(b, ref_b)], net, cfg1)
    assert loss == pytest.approx(0.5 * (la + lb), rel=1e-14)
    for k in cbc_train.PARAMS:
        np.testing.assert_allclose(g[k], 0.5 * (ga[k] + gb[k]), rtol=1e-12,
                                   atol=1e-12 * np.max(np.abs(g[k])))
    # the segment's own parameters matter
    assert abs(cbc_train.loss_only([(b, ref_b)], net, CFG) - lb) > 1e-3 * lb


def test_free_stream_has_zero_loss_and_gradient():
    a0 = d2q9.equilibrium(np.ones((NY, NX)), np.full((NY, NX), U0), np.zeros((NY, NX)))
    ref = np.stack([np.ones((NY, 5)), np.full((NY, 5), U0), np.zeros((NY, 5))])
    loss, g = cbc_train.loss_and_grad([(a0, ref)], _net(3), CFG)
    assert loss < 1e-28
    for k in cbc_train.PARAMS:
        assert np.max(np.abs(g[k])) < 1e-18


def test_loss_normalisation_and_region():
    # the reference equal to the segment's own final moments on the last n_t
    # columns gives zero; a defect delta at one node of Omega_s adds
    # delta^2 / (n_t ny), once per velocity component
    net, n_t, delta = _net(4), 4, 3e-3
    a0 = _state()
    fin = cbc_train.final_state(a0, net, CFG, n_t)
    ref = np.stack(d2q9.moments(fin[:, :, NX - n_t:]))
    assert cbc_train.loss_only([(a0, ref)], net, CFG) < 1e-30
    for comp, y, x in ((0, 3, 0), (1, 17, n_t - 1), (2, 0, 2)):
        r = ref.copy()
        r[comp, y, x] += delta
        assert cbc_train.loss_only([(a0, r)], net, CFG) == pytest.approx(
            delta**2 / (n_t * NY), rel=1e-9)
    r = ref.copy()
    r[1, 5, 1] += delta
    r[2, 5, 1] += delta
    assert cbc_train.loss_only([(a0, r)], net, CFG) == pytest.approx(
        2 * delta**2 / (n_t * NY), rel=1e-9)
    # the batch loss is the mean of the segment losses
    r = ref.copy()
    r[0, 0, 0] += delta
    assert cbc_train.loss_only([(a0, ref), (a0, r)], net, CFG) == pytest.approx(
        0.5 * delta**2 / (n_t * NY), rel=1e-9)


@pytest.mark.parametrize("n_t", [2, 5])
def test_segment_depends_only_on_the_last_2nt_plus_3_columns(n_t):
    net = _net(5)
    a0 = _state()
    ref = _ref(a0, n_t)
    loss, g = cbc_train.loss_and_grad([(a0, ref)], net, CFG)
    w = 2 * n_t + 3
    rng = np.random.default_rng(n_t)
    b0 = a0.copy()
    b0[:, :, :NX - w] *= 1 + 1e-2 * rng.standard_normal(b0[:, :, :NX - w].shape)
    loss_b, g_b = cbc_train.loss_and_grad([(b0, ref)], net, CFG)
    assert loss_b == loss
    for k in cbc_train.PARAMS:
        np.testing.assert_array_equal(g_b[k], g[k])
    # the cone is not empty: a change inside the strip reaches the loss
    c0 = a0.copy()
    c0[:, :, NX - 2 * n_t + 1] *= 1 + 1e-3
    assert cbc_train.loss_only([(c0, ref)], net, CFG) != loss


def test_torch_is_float64():
    st = cbc_train.rollout(_state(), cbc_train._theta(_net(0), False), _net(0), CFG, 1)
    assert st[-1].dtype == torch.float64
