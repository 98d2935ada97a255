"""Closed-loop training of the tuning network of the characteristic outflow,
FP64 on the CPU (test infrastructure; see ``oracle/__init__``).

Sec. 4.2: a training segment starts from a state of the reflection-free
reference run, advances n_t steps on the truncated lattice with sigma and
kappa_2 set per outlet node by the network, and is scored by the mean
squared error of density and velocity against the reference at step n_t,
over the columns next to the outlet that a reflection can reach in n_t
steps.  The gradient of that loss with respect to the network parameters is
the derivative of the whole rollout; here it is taken by reverse-mode
automatic differentiation (a library primitive) through a plain
re-expression of the oracle's step in torch operations: BGK collision
(Eq. 2), pull streaming (Eq. 1) with periodic laterals, the Zou & He
velocity inlet (Eqs. 5-11 mirrored) and the characteristic outlet of
``oracle/cbc.py`` (Eqs. 18-29, same readings).  The re-expression is pinned
to the numpy solver step by step, and its gradient to finite differences of
the numpy solver's loss.

Readings where the section is silent or at odds with itself:
  * the loss region Omega_s: the section bounds it by L - n_t < x < L and
    also calls it the n_t layers closest to the outlet; the strict upper
    bound would leave n_t - 1 layers, so the n_t columns
    L - n_t < x <= L are used (the outlet column's state is part of the
    simulated field);
  * the velocity MSE sums the squared components per node before the mean
    over Omega_s, so a segment's loss is
        mean_Omega (rho - rho_ref)^2 + mean_Omega |U - U_ref|^2;
  * a segment is a fresh run from the reference state: the time derivatives
    of the previous step (network features 7-9) start at zero;
  * a batch of segments is scored by the mean of their losses;
  * the lattice of a segment is free of solid nodes (the vortex benchmark).
"""
import numpy as np
import torch

from .d2q9 import C, CS2, W

CS = float(np.sqrt(CS2))
PARAMS = ("w1", "b1", "w2", "b2", "w3", "b3")
_CX = [int(c) for c in C[:, 0]]
_CY = [int(c) for c in C[:, 1]]
_W = [float(w) for w in W]


def _feq(rho, ux, uy):
    """Eq. 3 in torch: (9, ...) from rho, u."""
    usq = ux * ux + uy * uy
    out = []
    for i in range(9):
        cu = _CX[i] * ux + _CY[i] * uy
        out.append(_W[i] * rho * (1.0 + cu / CS2 + cu * cu / (2 * CS2 * CS2) - usq / (2 * CS2)))
    return torch.stack(out)


def moments(f):
    """Eq. 4 in torch: rho, u, v of f (9, ...)."""
    rho = f.sum(0)
    jx = sum(_CX[i] * f[i] for i in range(9) if _CX[i])
    jy = sum(_CY[i] * f[i] for i in range(9) if _CY[i])
    return rho, jx / rho, jy / rho


def collide(f, tau):
    """BGK, Eq. 2."""
    rho, ux, uy = moments(f)
    return f - (f - _feq(rho, ux, uy)) / tau


def stream(a):
    """Pull streaming f_i(x) = a_i(x - c_i) with periodic rows; entries whose
    source lies outside the columns are zero placeholders (the unknowns of
    the inlet and outlet columns)."""
    out = []
    for i in range(9):
        g = torch.roll(a[i], shifts=_CY[i], dims=0)
        z = torch.zeros_like(g[:, :1])
        if _CX[i] == 1:
            g = torch.cat([z, g[:, :-1]], dim=1)
        elif _CX[i] == -1:
            g = torch.cat([g[:, 1:], z], dim=1)
        out.append(g)
    return torch.stack(out)


def inlet(fc, u_in):
    """Zou & He velocity inlet at x = 0 (mirror of Eqs. 7-10), v = 0:
    fills 1, 5, 8 of the column fc (9, ny)."""
    rho = (fc[0] + fc[2] + fc[4] + 2.0 * (fc[3] + fc[6] + fc[7])) / (1.0 - u_in)
    ux = torch.full_like(rho, u_in)
    uy = torch.zeros_like(rho)
    eq = _feq(rho, ux, uy)
    ne = fc - eq
    g = list(fc)
    g[1] = eq[1] + ne[3]
    g[5] = eq[5] + ne[7] + 0.5 * (ne[4] - ne[2])
    g[8] = eq[8] + ne[6] - 0.5 * (ne[4] - ne[2])
    return torch.stack(g)


def _dx(p2, p1, p0):
    return 0.5 * (3.0 * p0 - 4.0 * p1 + p2)


def _dy(p):
    return 0.5 * (torch.roll(p, -1, 0) - torch.roll(p, 1, 0))


def network(feats, theta, net):
    """The tuning network (Sec. 4.2): (ny, 9) features -> sigma, kappa_2."""
    z = (feats - torch.as_tensor(net["mu_in"], dtype=torch.float64)) / \
        torch.as_tensor(net["sd_in"], dtype=torch.float64)
    a = float(net.get("leaky_slope", 0.01))

    def leaky(x):
        return torch.where(x > 0, x, a * x)
    h1 = leaky(z @ theta["w1"].T + theta["b1"])
    h2 = leaky(h1 @ theta["w2"].T + theta["b2"])
    s = torch.sigmoid(h2 @ theta["w3"].T + theta["b3"])
    return (net["sigma_scale"] * s[:, 0] + net["sigma_shift"],
            net["kappa_scale"] * s[:, 1] + net["kappa_shift"])


def outlet(fc, a3, prev, theta, net, cfg):
    """Characteristic outlet (Eqs. 18-29, readings of ``oracle/cbc.py``) from
    the streamed column fc (9, ny), the post-collision state a3 (9, ny, 3)
    of the last three columns and the previous time derivatives prev
    (ny, 3).  Returns the completed column and the new time derivatives."""
    rho3, u3, v3 = moments(a3)
    rho, u, v = rho3[:, 2], u3[:, 2], v3[:, 2]
    px = CS2 * _dx(rho3[:, 0], rho3[:, 1], rho3[:, 2])
    ux = _dx(u3[:, 0], u3[:, 1], u3[:, 2])
    vx = _dx(v3[:, 0], v3[:, 1], v3[:, 2])
    py, uy, vy = CS2 * _dy(rho), _dy(u), _dy(v)
    feats = torch.stack([px, ux, vx, py, uy, vy, prev[:, 0], prev[:, 1], prev[:, 2]], dim=1)
    sigma, kappa2 = network(feats, theta, net)
    p = CS2 * rho
    L3 = u * vx
    L5 = (u + CS) * (px + rho * CS * ux)
    T1 = -(v * py + p * vy - rho * CS * v * uy)
    T3 = -(v * vy + py / rho)
    T5 = -(v * py + p * vy + rho * CS * v * uy)
    kappa1 = sigma * (1.0 - cfg["mach"] ** 2) * CS / cfg["length"]
    L1 = kappa1 * CS2 * (rho - cfg["rho_inf"]) - kappa2 * T1 + T1
    rho_t = (-(L5 + L1) + (T5 + T1)) / (2.0 * CS2)
    u_t = (-(L5 - L1) + (T5 - T1)) / (2.0 * rho * CS)
    v_t = -L3 + T3
    r1, u1, v1 = rho + rho_t, u + u_t, v + v_t
    known = fc[0] + fc[2] + fc[4] + 2.0 * (fc[1] + fc[5] + fc[8])
    g = list(fc)
    g[0] = fc[0] + r1 * (1.0 + u1) - known                     # Eq. 29 (reading)
    eq = _feq(r1, u1, v1)
    ne = [fc[q] - eq[q] for q in range(9)]
    g[3] = eq[3] + ne[1]                                        # Eq. 9
    g[6] = eq[6] + ne[8] + 0.5 * (ne[4] - ne[2])                # Eq. 8
    g[7] = eq[7] + ne[5] - 0.5 * (ne[4] - ne[2])                # Eq. 10
    return torch.stack(g), torch.stack([CS2 * rho_t, u_t, v_t], dim=1)


def rollout(a0, theta, net, cfg, n_t):
    """Post-collision states A_0 .. A_{n_t} of the truncated lattice (no
    solids, periodic rows), starting from a0 (9, ny, nx) with zero previous
    time derivatives."""
    a = torch.as_tensor(a0, dtype=torch.float64)
    prev = torch.zeros((a.shape[1], 3), dtype=torch.float64)
    states = [a]
    for _ in range(n_t):
        f = stream(a)
        fin = inlet(f[:, :, 0], cfg["u_in"])
        fout, prev = outlet(f[:, :, -1], a[:, :, -3:], prev, theta, net, cfg)
        f = torch.cat([fin[:, :, None], f[:, :, 1:-1], fout[:, :, None]], dim=2)
        a = collide(f, cfg["tau"])
        states.append(a)
    return states


def segment_loss(a_nt, ref):
    """Loss of one segment from its final state a_nt (9, ny, nx) and the
    reference moments ref (3, ny, n_t) over the last n_t columns."""
    n_t = ref.shape[2]
    rho, u, v = moments(a_nt[:, :, -n_t:])
    ref = torch.as_tensor(ref, dtype=torch.float64)
    return ((rho - ref[0]) ** 2).mean() + ((u - ref[1]) ** 2 + (v - ref[2]) ** 2).mean()


def _theta(net, requires_grad):
    return {k: torch.tensor(np.asarray(net[k], dtype=np.float64), requires_grad=requires_grad)
            for k in PARAMS}


def _seg(segment, cfg):
    """(a0, ref, cfg) of a segment given as (a0, ref) or (a0, ref, own cfg)."""
    return (segment[0], segment[1], segment[2] if len(segment) > 2 else cfg)


def loss_and_grad(segments, net, cfg):
    """Mean loss over segments [(a0, ref), ...] (n_t of each = ref.shape[2];
    a segment may carry its own cfg as a third element) and its gradient
    with respect to w1, b1, w2, b2, w3, b3 (numpy dict)."""
    theta = _theta(net, True)
    total = 0.0
    for seg in segments:
        a0, ref, c = _seg(seg, cfg)
        states = rollout(a0, theta, net, c, ref.shape[2])
        total = total + segment_loss(states[-1], ref)
    loss = total / len(segments)
    loss.backward()
    return float(loss.detach()), {k: theta[k].grad.numpy().copy() for k in PARAMS}


def loss_only(segments, net, cfg):
    theta = _theta(net, False)
    with torch.no_grad():
        total = 0.0
        for seg in segments:
            a0, ref, c = _seg(seg, cfg)
            total += float(segment_loss(rollout(a0, theta, net, c, ref.shape[2])[-1], ref))
    return total / len(segments)


def final_state(a0, net, cfg, n_t):
    """A_{n_t} as a numpy array (forward only)."""
    with torch.no_grad():
        return rollout(a0, _theta(net, False), net, cfg, n_t)[-1].numpy()
