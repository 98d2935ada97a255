"""Characteristic outflow boundary (CBC) at the right column, FP64 (test
infrastructure; see ``oracle/__init__``).

Sec. 4: at the outlet x = L the density and the velocity of the next step
follow from the characteristic (LODI) form of the isothermal equations,
Eqs. 18-20, with the wave amplitudes of Eqs. 21-23 and the transverse terms
of Eqs. 24-26; the incoming amplitude L_1 is replaced by Eq. 27 (relaxation
towards the far-field pressure with kappa_1 = sigma (1 - M^2) c_s / L of
Eq. 28, partial transverse compensation kappa_2); a forward Euler step gives
(rho, u, v) at the next step, which are mapped to the unknown populations by
the Zou & He reconstruction (Eqs. 8-10) after the correction of f_0 of
Eq. 29.  The network variant sets sigma and kappa_2 per node from nine local
features (two hidden layers of 20, LeakyReLU, sigmoid then scale and shift).

Readings (the section is terse or garbled in places):
  * p = c_s^2 rho (isothermal), c = c_s; Eqs. 21 and 23 print d rho/dx where
    the dimensions and Eq. 18 need dp/dx:
        L_1 = (u - c_s)(p_x - rho c_s u_x),  L_5 = (u + c_s)(p_x + rho c_s u_x),
        L_3 = u v_x;
  * Eqs. 24 and 26 print rho c_s v dv/dy as last term; only rho c_s v du/dy
    makes Eq. 19 carry the transverse advection -v du/dy of u:
        T_1 = -(v p_y + p v_y - rho c_s v u_y),
        T_5 = -(v p_y + p v_y + rho c_s v u_y),
        T_3 = -(v v_y + p_y / rho);
  * T_{1,exact} = 0 in Eq. 27 (no exact transverse solution is given), so
    kappa_2 = Ma is the usual partial compensation;
  * M in Eq. 28 is the reference Mach number, L the domain length; p_inf =
    c_s^2 rho_inf;
  * derivatives at the outlet node: second-order one-sided in x,
    (3 phi_L - 4 phi_{L-1} + phi_{L-2}) / 2; central in y with periodic
    laterals, the only lateral condition the section uses (the solver
    rejects walls: the inviscid update has no consistent treatment of the
    corner where the outlet meets a no-slip wall, and the wall-row velocity
    drifts there); every field is the state of the current time level (the
    moments of the stored populations, which collision conserves);
  * Eq. 29 is meant to make the reconstructed node carry the prescribed
    density; the printed form does so only up to a factor (1 + u) on the
    density defect, so the exactly consistent correction is used:
        g_0 = f_0 + rho' (1 + u') - (rho_0 + 2 rho_+);
  * network: features (p_x, u_x, v_x, p_y, u_y, v_y, p_t, u_t, v_t), the
    time derivatives being those of the previous step (zero before the
    first), standardised z = (x - mu) / sd; LeakyReLU negative slope 0.01;
    sigma = sigma_scale * sigmoid(s_0) + sigma_shift, likewise kappa_2.
"""
import numpy as np

from .d2q9 import CS2
from .zouhe import outlet_reconstruct

CS = np.sqrt(CS2)


def x_derivative(phi_l2, phi_l1, phi_l):
    """Second-order backward difference at the outlet column."""
    return 0.5 * (3.0 * phi_l - 4.0 * phi_l1 + phi_l2)


def y_derivative(phi, periodic):
    """d/dy along the outlet column (phi indexed by row)."""
    phi = np.asarray(phi, dtype=np.float64)
    if periodic:
        return 0.5 * (np.roll(phi, -1) - np.roll(phi, 1))
    d = np.empty_like(phi)
    d[1:-1] = 0.5 * (phi[2:] - phi[:-2])
    d[0] = 0.5 * (-3.0 * phi[0] + 4.0 * phi[1] - phi[2])
    d[-1] = 0.5 * (3.0 * phi[-1] - 4.0 * phi[-2] + phi[-3])
    return d


def amplitudes(rho, u, v, g):
    """Eqs. 21-26: L_1, L_3, L_5, T_1, T_3, T_5 from the outlet values and the
    gradients g = (p_x, u_x, v_x, p_y, u_y, v_y)."""
    p_x, u_x, v_x, p_y, u_y, v_y = g
    p = CS2 * rho
    L1 = (u - CS) * (p_x - rho * CS * u_x)
    L3 = u * v_x
    L5 = (u + CS) * (p_x + rho * CS * u_x)
    T1 = -(v * p_y + p * v_y - rho * CS * v * u_y)
    T3 = -(v * v_y + p_y / rho)
    T5 = -(v * p_y + p * v_y + rho * CS * v * u_y)
    return L1, L3, L5, T1, T3, T5


def time_derivatives(rho, u, v, g, sigma, kappa2, mach, length, rho_inf):
    """Eqs. 18-20 with L_1 from Eqs. 27-28: (rho_t, u_t, v_t)."""
    L1, L3, L5, T1, T3, T5 = amplitudes(rho, u, v, g)
    kappa1 = sigma * (1.0 - mach * mach) * CS / length
    L1 = kappa1 * CS2 * (rho - rho_inf) - kappa2 * T1 + T1       # T_1,exact = 0
    rho_t = (-(L5 + L1) + (T5 + T1)) / (2.0 * CS2)
    u_t = (-(L5 - L1) + (T5 - T1)) / (2.0 * rho * CS)
    v_t = -L3 + T3
    return rho_t, u_t, v_t


def gradients(rho3, u3, v3, periodic):
    """Gradients at the outlet from the three last columns of rho, u, v
    (each (3, ny): columns L-2, L-1, L)."""
    return (CS2 * x_derivative(*rho3), x_derivative(*u3), x_derivative(*v3),
            CS2 * y_derivative(rho3[2], periodic), y_derivative(u3[2], periodic),
            y_derivative(v3[2], periodic))


def network(features, P):
    """The tuning network: features (n, 9) -> sigma (n,), kappa_2 (n,)."""
    z = (np.asarray(features, np.float64) - P["mu_in"]) / P["sd_in"]
    a = P.get("leaky_slope", 0.01)

    def leaky(x):
        return np.where(x > 0.0, x, a * x)
    h1 = leaky(z @ np.asarray(P["w1"], np.float64).T + P["b1"])
    h2 = leaky(h1 @ np.asarray(P["w2"], np.float64).T + P["b2"])
    s = h2 @ np.asarray(P["w3"], np.float64).T + P["b3"]
    sig = 1.0 / (1.0 + np.exp(-s))
    return (P["sigma_scale"] * sig[:, 0] + P["sigma_shift"],
            P["kappa_scale"] * sig[:, 1] + P["kappa_shift"])


def outlet(fcol, rho3, u3, v3, prev_t, params, periodic):
    """CBC at the outlet column.

    fcol      (9, ny): populations of the outlet nodes after streaming
              (unknowns 3, 6, 7 ignored);
    rho3, u3, v3 (3, ny): the current state at columns L-2, L-1, L;
    prev_t    (ny, 3): (p_t, u_t, v_t) of the previous step (network input);
    params    dict: sigma, kappa2, mach, length, rho_inf, optional 'net'.
    Returns the completed populations and the new (p_t, u_t, v_t)."""
    g = gradients(rho3, u3, v3, periodic)
    rho, u, v = rho3[2], u3[2], v3[2]
    if params.get("net") is not None:
        feats = np.stack([*g, prev_t[:, 0], prev_t[:, 1], prev_t[:, 2]], axis=1)
        sigma, kappa2 = network(feats, params["net"])
    else:
        sigma, kappa2 = params["sigma"], params["kappa2"]
    rho_t, u_t, v_t = time_derivatives(rho, u, v, g, sigma, kappa2, params["mach"],
                                       params["length"], params["rho_inf"])
    rho1, u1, v1 = rho + rho_t, u + u_t, v + v_t                 # forward Euler
    f = np.array(fcol, dtype=np.float64, copy=True)
    known = (f[0] + f[2] + f[4]) + 2.0 * (f[1] + f[5] + f[8])    # rho_0 + 2 rho_+
    f[0] = f[0] + rho1 * (1.0 + u1) - known                      # Eq. 29 (reading)
    f = outlet_reconstruct(f, rho1, u1, v1)
    return f, np.stack([CS2 * rho_t, u_t, v_t], axis=1)
