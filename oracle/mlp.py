"""The outflow MLP of the direct-reconstruction boundary (test
infrastructure; see ``oracle/__init__``).

Sec. 3.1: a shallow fully connected network with two hidden layers maps
interior populations to corrections s_i^NN of the three unknown populations
at the outlet, f_i^B(L) = f_i(L-1) + s_i^NN for i = 3, 6, 7 (Eq. 16), and is
trained by the mean squared error against reference populations (Eq. 17).

Readings (the paper fixes neither): 27 inputs (the 9 populations at each of
x = L-1, L-2, L-3, feature k = 9 j + q for column L-1-j), two tanh hidden
layers of 64, 3 linear outputs; inputs are the offsets f - w, standardised
per feature; outputs are standardised corrections, s = o sd_out + mu_out;
Adam (Kingma & Ba 2015) with the usual defaults.

Two forward passes are given:
  * ``forward_f64``: plain FP64 algebra, used for the gradient pins;
  * ``forward_bf16``: the same algebra with the BF16 roundings the MFMA
    path makes (standardised inputs, weights, hidden activations rounded to
    BF16 by round-to-nearest-even of the FP32 value; the standardisation
    itself done in FP32), sums in FP64.
"""
import numpy as np


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even) via the FP32 value."""
    x32 = np.asarray(x, dtype=np.float32)
    b = x32.view(np.uint32).astype(np.uint64)
    b = (b + np.uint64(0x7FFF) + ((b >> np.uint64(16)) & np.uint64(1))) \
        & np.uint64(0xFFFF0000)
    r = b.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(x32), np.nan, r)


def standardise_f32(x, mu, sd):
    """z = (x - mu) * (1/sd), every operation in IEEE FP32."""
    x32 = np.asarray(x, dtype=np.float32)
    inv = np.float32(1.0) / np.asarray(sd, dtype=np.float32)
    return ((x32 - np.asarray(mu, dtype=np.float32)) * inv).astype(np.float64)


def forward_bf16(x, P):
    """Inference as the fused outflow kernel evaluates it.  ``x`` is (n, 27)
    population offsets; returns the corrections s (n, 3) in FP64."""
    z = bf16_round(standardise_f32(x, P["mu_in"], P["sd_in"]))
    a1 = z @ bf16_round(P["w1"]).T + np.asarray(P["b1"], np.float64)
    h1 = bf16_round(np.tanh(a1))
    a2 = h1 @ bf16_round(P["w2"]).T + np.asarray(P["b2"], np.float64)
    h2 = bf16_round(np.tanh(a2))
    o = h2 @ bf16_round(P["w3"]).T + np.asarray(P["b3"], np.float64)
    return o * np.asarray(P["sd_out"], np.float64) + np.asarray(P["mu_out"], np.float64)


def forward_f64(z, P):
    """FP64 forward on standardised inputs z (n, 27); returns the cache the
    backward pass needs and the standardised outputs o (n, 3)."""
    a1 = z @ P["w1"].T + P["b1"]
    h1 = np.tanh(a1)
    a2 = h1 @ P["w2"].T + P["b2"]
    h2 = np.tanh(a2)
    o = h2 @ P["w3"].T + P["b3"]
    return (z, h1, h2), o


def mse_loss(o, y):
    """Eq. 17: mean over samples and the three outputs of (o - y)^2."""
    return float(np.mean((o - y) ** 2))


def backward_f64(cache, o, y, P):
    """Gradients of mse_loss w.r.t. every parameter, by the chain rule."""
    z, h1, h2 = cache
    n = o.shape[0]
    d_o = 2.0 * (o - y) / (n * o.shape[1])
    g = {"w3": d_o.T @ h2, "b3": d_o.sum(0)}
    d_a2 = (d_o @ P["w3"]) * (1.0 - h2 * h2)
    g["w2"] = d_a2.T @ h1
    g["b2"] = d_a2.sum(0)
    d_a1 = (d_a2 @ P["w2"]) * (1.0 - h1 * h1)
    g["w1"] = d_a1.T @ z
    g["b1"] = d_a1.sum(0)
    return g


PARAM_NAMES = ("w1", "b1", "w2", "b2", "w3", "b3")


def grad_bf16(x, t, P):
    """Loss (Eq. 17 on standardised outputs) and gradients of the training
    pass as the MFMA kernels evaluate it: the forward of ``forward_bf16``
    with standardised targets y = (t - mu_out) (1/sd_out) (FP32), and the
    chain rule in FP64 where every matrix product takes its operands rounded
    to BF16 as the MFMA path does (dL/do, dL/dz2, dL/dz1, activations,
    weights; dL/dh2 uses the FP32 weights of layer 3, an elementwise product
    on the GPU).  tanh' is 1 - h^2 of the unrounded activation; bias
    gradients sum unrounded values."""
    b = bf16_round
    z = b(standardise_f32(x, P["mu_in"], P["sd_in"]))
    y = standardise_f32(t, P["mu_out"], P["sd_out"])
    W1, W2, W3 = b(P["w1"]), b(P["w2"]), b(P["w3"])
    h1 = np.tanh(z @ W1.T + P["b1"])
    h1b = b(h1)
    h2 = np.tanh(h1b @ W2.T + P["b2"])
    h2b = b(h2)
    o = h2b @ W3.T + P["b3"]
    n = x.shape[0]
    loss = float(np.mean((o - y) ** 2))
    d_o = 2.0 * (o - y) / (3 * n)
    g = {"w3": b(d_o).T @ h2b, "b3": d_o.sum(0)}
    dz2 = (d_o @ np.asarray(P["w3"], np.float64)) * (1.0 - h2 * h2)
    g["w2"] = b(dz2).T @ h1b
    g["b2"] = dz2.sum(0)
    dz1 = (b(dz2) @ W2) * (1.0 - h1 * h1)
    g["w1"] = b(dz1).T @ z
    g["b1"] = dz1.sum(0)
    return loss, g


class Adam:
    """Adam (Kingma & Ba 2015): first and second moment estimates with bias
    correction; theta <- theta - lr mhat / (sqrt(vhat) + eps)."""

    def __init__(self, P, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = {k: np.zeros_like(P[k], dtype=np.float64) for k in PARAM_NAMES}
        self.v = {k: np.zeros_like(P[k], dtype=np.float64) for k in PARAM_NAMES}
        self.t = 0

    def step(self, P, g):
        self.t += 1
        for k in PARAM_NAMES:
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * g[k]
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * g[k] * g[k]
            mhat = self.m[k] / (1 - self.b1 ** self.t)
            vhat = self.v[k] / (1 - self.b2 ** self.t)
            P[k] = P[k] - self.lr * mhat / (np.sqrt(vhat) + self.eps)
        return P
