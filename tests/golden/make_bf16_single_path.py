"""Writes bf16_single_path.json: a hand-checkable worked example that fixes
where the BF16 roundings of the outflow network's MFMA path go (Sec. 3.1,
Eq. 16 forward; Eq. 17 loss and its gradient).

The network is a single path through the 1-1-1-3 form of the outflow MLP
(one input feature, one unit per hidden layer, output 0 connected; outputs 1
and 2 carry only their biases).  Every intermediate value is derived here in
scalar Python: IEEE FP32 operations through numpy.float32, BF16 rounding
through torch's float32 -> bfloat16 conversion (round to nearest, ties to
even), tanh from the math module.  Nothing here imports the oracle or the
library: the oracle's forward_bf16 and grad_bf16 are tested against the
values written here.

Rounding points of the path (the specification the kernels implement):
  forward   z = (x - mu_in) * (1 / sd_in) in FP32, rounded to BF16; weights
            rounded to BF16; a = W z + b with b in FP32 (not rounded);
            h = tanh(a) rounded to BF16 before the next product; the output
            o = W3 h2 + b3 is not rounded, s = o sd_out + mu_out.
  gradient  standardised targets y = (t - mu_out) * (1 / sd_out) in FP32;
            d_o = 2 (o - y) / (3 n); dW3 = bf16(d_o) h2; the hidden error
            dz2 = (d_o W3) (1 - h2^2) takes W3 unrounded and h2 unrounded;
            dW2 = bf16(dz2) h1; dz1 = (bf16(dz2) W2) (1 - h1^2) with the BF16
            W2 and h1 unrounded; dW1 = bf16(dz1) z; bias gradients sum the
            unrounded d_o, dz2, dz1.

The parameters were picked so that moving any one rounding point (dropping
one, adding one, taking a standardisation in FP64) changes some output or
gradient entry: by 5.9e-8 relative for the FP64 standardisation of the
targets (it moves the loss only), by at least 9.6e-6 for every other one;
the fixture lists the values each such mistake would give.  The first sample puts the FP32 standardisation
exactly on a BF16 tie that rounds up, where the FP64 standardisation rounds
down.

    python tests/golden/make_bf16_single_path.py
"""
import json
import math
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))

P = {"mu_in": 0.0, "sd_in": 3.0, "w1": 0.2328948974609375, "w2": 2.132568359375,
     "w3": 1.5819091796875, "b1": 0.06468963623046875, "b2": 0.1274261474609375,
     "b3": [0.268524169921875, -0.02, 0.013], "mu_out": [1e-05, 2e-06, -3e-06],
     "sd_out": [0.001, 0.002, 0.0005]}
X = [3.035156011581421, 2.526848077774048, 4.393764495849609, 4.326937198638916,
     3.810360908508301, 3.37967848777771, 2.7330164909362793, 2.297926425933838,
     3.082693576812744, 2.234828472137451, 3.3983118534088135, 3.577960252761841,
     4.012757778167725, 2.9490034580230713, 3.101569414138794, 4.0055623054504395]
T_SEED = 11

FORWARD_MISTAKES = ["std_f64", "z_unrounded", "w1_unrounded", "w2_unrounded", "w3_unrounded",
                    "b1_rounded", "b2_rounded", "b3_rounded", "a1_rounded", "a2_rounded",
                    "h1_unrounded", "h2_unrounded", "o_rounded"]
GRADIENT_MISTAKES = FORWARD_MISTAKES + [
    "do_unrounded_in_gw3", "w3_rounded_in_dz2", "h2b_in_tanh_prime2", "dz2_unrounded_in_gw2",
    "dz2_unrounded_in_dz1", "w2_unrounded_in_dz1", "h1b_in_tanh_prime1", "dz1_unrounded_in_gw1",
    "y_f64"]


def bf16(v):
    return float(torch.tensor(np.float32(v)).to(torch.bfloat16).float())


def f32(v):
    return float(np.float32(v))


def std_f32(v, mu, sd):
    return float((np.float32(v) - np.float32(mu)) * (np.float32(1.0) / np.float32(sd)))


def sample(x, t, m=()):
    """Forward chain of one sample; ``m`` names mistakes to make."""
    z32 = f32((x - P["mu_in"]) / P["sd_in"]) if "std_f64" in m else std_f32(x, P["mu_in"], P["sd_in"])
    zb = z32 if "z_unrounded" in m else bf16(z32)
    W1 = P["w1"] if "w1_unrounded" in m else bf16(P["w1"])
    W2 = P["w2"] if "w2_unrounded" in m else bf16(P["w2"])
    W3 = P["w3"] if "w3_unrounded" in m else bf16(P["w3"])
    b1 = bf16(P["b1"]) if "b1_rounded" in m else f32(P["b1"])
    b2 = bf16(P["b2"]) if "b2_rounded" in m else f32(P["b2"])
    b3 = [bf16(v) if "b3_rounded" in m else f32(v) for v in P["b3"]]
    a1 = W1 * zb + b1
    a1 = bf16(a1) if "a1_rounded" in m else a1
    h1 = math.tanh(a1)
    h1b = h1 if "h1_unrounded" in m else bf16(h1)
    a2 = W2 * h1b + b2
    a2 = bf16(a2) if "a2_rounded" in m else a2
    h2 = math.tanh(a2)
    h2b = h2 if "h2_unrounded" in m else bf16(h2)
    o = [W3 * h2b + b3[0], b3[1], b3[2]]
    o = [bf16(v) for v in o] if "o_rounded" in m else o
    s = [o[k] * f32(P["sd_out"][k]) + f32(P["mu_out"][k]) for k in range(3)]
    if "y_f64" in m:
        y = [(t[k] - P["mu_out"][k]) / P["sd_out"][k] for k in range(3)]
    else:
        y = [std_f32(t[k], P["mu_out"][k], P["sd_out"][k]) for k in range(3)]
    return {"z32": z32, "zb": zb, "W1": W1, "W2": W2, "W3": W3, "b1": b1, "b2": b2, "b3": b3,
            "a1": a1, "h1": h1, "h1b": h1b, "a2": a2, "h2": h2, "h2b": h2b, "o": o, "s": s, "y": y}


def batch(X, T, m=()):
    """Forward of every sample, the loss (Eq. 17) and the gradient."""
    rows = [sample(x, t, m) for x, t in zip(X, T)]
    n = len(rows)
    loss = sum((r["o"][k] - r["y"][k]) ** 2 for r in rows for k in range(3)) / (3 * n)
    g = {"w1": 0.0, "w2": 0.0, "w3": [0.0, 0.0, 0.0], "b1": 0.0, "b2": 0.0, "b3": [0.0, 0.0, 0.0]}
    for r in rows:
        do = [2 * (r["o"][k] - r["y"][k]) / (3 * n) for k in range(3)]
        for k in range(3):
            g["w3"][k] += (do[k] if "do_unrounded_in_gw3" in m else bf16(do[k])) * r["h2b"]
            g["b3"][k] += do[k]
        w3 = bf16(P["w3"]) if "w3_rounded_in_dz2" in m else f32(P["w3"])
        h2 = r["h2b"] if "h2b_in_tanh_prime2" in m else r["h2"]
        dz2 = do[0] * w3 * (1 - h2 * h2)
        g["w2"] += (dz2 if "dz2_unrounded_in_gw2" in m else bf16(dz2)) * r["h1b"]
        g["b2"] += dz2
        W2 = P["w2"] if "w2_unrounded_in_dz1" in m else r["W2"]
        h1 = r["h1b"] if "h1b_in_tanh_prime1" in m else r["h1"]
        dz1 = (dz2 if "dz2_unrounded_in_dz1" in m else bf16(dz2)) * W2 * (1 - h1 * h1)
        g["w1"] += (dz1 if "dz1_unrounded_in_gw1" in m else bf16(dz1)) * r["zb"]
        g["b1"] += dz1
        r.update(do=do, dz2=dz2, dz1=dz1)
    return rows, loss, g


def flat(loss, g):
    return [loss, g["w1"], g["w2"], g["b1"], g["b2"]] + g["w3"] + g["b3"]


def targets():
    rs = np.random.default_rng(T_SEED)
    return [[f32(rs.uniform(-6e-4, 6e-4)), f32(rs.uniform(-5e-5, 5e-5)), f32(rs.uniform(-5e-5, 5e-5))]
            for _ in X]


def main():
    T = targets()
    rows, loss, g = batch(X, T)
    fwd, grad = {}, {}
    for m in FORWARD_MISTAKES:
        r2, _, _ = batch(X, T, {m})
        fwd[m] = {"s0": [r["s"][0] for r in r2],
                  "max_rel_change": max(abs(a["s"][0] - b["s"][0]) / abs(b["s"][0])
                                        for a, b in zip(r2, rows))}
    for m in GRADIENT_MISTAKES:
        _, l2, g2 = batch(X, T, {m})
        grad[m] = {"loss": l2, "grad": g2,
                   "max_rel_change": max(abs(a - b) / abs(b)
                                         for a, b in zip(flat(l2, g2), flat(loss, g)))}
    out = {"about": __doc__.split("\n\n")[0] + " Written by make_bf16_single_path.py.",
           "P": P, "x": X, "t": T, "rows": rows, "s": [r["s"] for r in rows], "loss": loss,
           "grad": g, "forward_mistakes": fwd, "gradient_mistakes": grad}
    with open(os.path.join(HERE, "bf16_single_path.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("smallest change a mistake makes:",
          min(v["max_rel_change"] for v in list(fwd.values()) + list(grad.values())))


if __name__ == "__main__":
    main()
