"""Error bounds for comparing the fused outflow network with the oracle's
BF16-emulating forward pass (test helper)."""
import numpy as np

from oracle import mlp as omlp


def output_bound(x, P):
    """Per-output bound on |GPU - oracle| of the outflow network's corrections
    s (n, 3) for features x (n, 27): both sides round the same standardised
    inputs and weights to BF16, the GPU accumulates in FP32 and the oracle in
    FP64, so a hidden activation can land on the other side of a BF16
    rounding boundary.  The bound lets every hidden unit move by one BF16
    unit in the last place (2^-8 relative) plus FP32 accumulation error
    (1e-5 of the absolute sum), propagated through |W|.  Returns (bound,
    tight): tight is the FP32 part alone, which most outputs meet."""
    b = omlp.bf16_round
    z = b(omlp.standardise_f32(x, P["mu_in"], P["sd_in"]))
    W1, W2, W3 = b(P["w1"]), b(P["w2"]), b(P["w3"])
    a1 = z @ W1.T + P["b1"]
    h1 = np.tanh(a1)
    e1 = 2.0**-8 * np.abs(h1) + 1e-5 * (np.abs(z) @ np.abs(W1).T + np.abs(P["b1"]))
    a2 = b(h1) @ W2.T + P["b2"]
    h2 = np.tanh(a2)
    e2 = e1 @ np.abs(W2).T + 2.0**-8 * np.abs(h2) + 1e-5 * (np.abs(h1) @ np.abs(W2).T)
    e3 = e2 @ np.abs(W3).T + 1e-5 * (np.abs(h2) @ np.abs(W3).T + np.abs(P["b3"]))
    return e3 * P["sd_out"], 1e-5 * (np.abs(b(h2)) @ np.abs(W3).T + np.abs(P["b3"])) * P["sd_out"]
