"""Closed-loop training of the outflow reconstruction network of Eq. 16,
FP64 on the CPU (test infrastructure; see ``oracle/__init__``).

The training procedure of Sec. 4.2 (segments started from states of the
long reference run, advanced n_t steps with the network in the loop, scored
against the reference at step n_t over the n_t columns next to the outlet,
the gradient taken through the whole rollout) applied to the network of
Sec. 3.1 instead of the tuning network: at every outlet row the unknown
populations are g_i = f_i(L-1) + s_i for i = 3, 6, 7 (Eq. 16), with
s = o * sd_out + mu_out and o the 9-20-20-3 network (tanh hidden layers,
linear output) of the standardised pre-collision offsets f - w of column
L - 1.  No fallback inside a segment (the fallback is a selection the
training does not differentiate).

The step is the one of ``oracle/cbc_train`` (BGK, pull streaming with
periodic rows, the Zou & He velocity inlet, a lattice without solid nodes)
with this outlet; the loss, its region Omega_s and the batch mean are the
readings stated there.  The gradient is taken by reverse-mode automatic
differentiation (a library primitive).
"""
import numpy as np
import torch

from .cbc_train import _seg, collide, inlet, moments, segment_loss, stream  # noqa: F401
from .d2q9 import W

PARAMS = ("w1", "b1", "w2", "b2", "w3", "b3")
_W = torch.tensor(W, dtype=torch.float64)


def network(feats, theta, net):
    """Eq. 16's corrections s (ny, 3) from the pre-collision offsets of
    column L-1 (ny, 9)."""
    f64 = lambda k: torch.as_tensor(np.asarray(net[k], np.float64))
    z = (feats - f64("mu_in")) / f64("sd_in")
    h1 = torch.tanh(z @ theta["w1"].T + theta["b1"])
    h2 = torch.tanh(h1 @ theta["w2"].T + theta["b2"])
    o = h2 @ theta["w3"].T + theta["b3"]
    return o * f64("sd_out") + f64("mu_out")


def outlet(fc, fl1, theta, net):
    """The outlet column (9, ny) from its streamed populations fc (the
    unknowns 3, 6, 7 are placeholders) and the streamed column L-1, fl1."""
    s = network((fl1 - _W[:, None]).T, theta, net)
    g = list(fc)
    for k, q in enumerate((3, 6, 7)):
        g[q] = fl1[q] + s[:, k]
    return torch.stack(g)


def rollout(a0, theta, net, cfg, n_t):
    """Post-collision states A_0 .. A_{n_t} of the lattice (no solids,
    periodic rows) from a0 (9, ny, nx)."""
    a = torch.as_tensor(a0, dtype=torch.float64)
    states = [a]
    for _ in range(n_t):
        f = stream(a)
        fin = inlet(f[:, :, 0], cfg["u_in"])
        fout = outlet(f[:, :, -1], f[:, :, -2], theta, net)
        f = torch.cat([fin[:, :, None], f[:, :, 1:-1], fout[:, :, None]], dim=2)
        a = collide(f, cfg["tau"])
        states.append(a)
    return states


def _theta(net, requires_grad):
    return {k: torch.tensor(np.asarray(net[k], dtype=np.float64), requires_grad=requires_grad)
            for k in PARAMS}


def loss_and_grad(segments, net, cfg):
    """Mean loss over segments [(a0, ref), ...] (n_t of each = ref.shape[2];
    a segment may carry its own cfg) and its gradient with respect to
    w1, b1, w2, b2, w3, b3 (numpy dict)."""
    theta = _theta(net, True)
    total = 0.0
    for seg in segments:
        a0, ref, c = _seg(seg, cfg)
        total = total + segment_loss(rollout(a0, theta, net, c, ref.shape[2])[-1], ref)
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


__all__ = ["network", "outlet", "rollout", "loss_and_grad", "loss_only", "final_state",
           "moments"]
