"""Aerodynamic observables (test infrastructure; see ``oracle/__init__``).

Sec. 2.3: C_D = 2 F_x / (rho U^2 A), C_L = 2 F_y / (rho U^2 A) (Eq. 13),
and the Strouhal number St = f D / U from a fast Fourier transform of the
lift coefficient.  The paper gives no window or resolution for the FFT;
reading: Hann window over the series minus its mean, zero padding, and a
parabolic fit through the peak bin and its neighbours.
"""
import numpy as np


def force_coefficients(fx, fy, rho_ref, U, A):
    s = 2.0 / (rho_ref * U * U * A)
    return np.asarray(fx) * s, np.asarray(fy) * s


def dominant_frequency(x, dt=1.0, pad=16):
    x = np.asarray(x, dtype=np.float64)
    x = x - x.mean()
    n = len(x)
    spec = np.abs(np.fft.rfft(x * np.hanning(n), n=pad * n))
    k = int(np.argmax(spec[1:-1])) + 1
    a, b, c = spec[k - 1], spec[k], spec[k + 1]
    den = a - 2 * b + c
    delta = 0.5 * (a - c) / den if den != 0 else 0.0
    return (k + delta) / (pad * n * dt)


def strouhal(cl, D, U, dt=1.0, pad=16):
    return dominant_frequency(cl, dt, pad) * D / U


def zero_crossing_frequency(x, dt=1.0):
    """Mean frequency from the upward zero crossings of x - mean(x); a
    crossing counts only after the signal has been below -std/4 since the
    previous one (hysteresis against noise)."""
    x = np.asarray(x, dtype=np.float64) - np.mean(x)
    arm = -0.25 * np.std(x)
    armed, tc = False, []
    for k in range(len(x) - 1):
        if x[k] < arm:
            armed = True
        if armed and x[k] < 0 <= x[k + 1]:
            tc.append(k + (-x[k]) / (x[k + 1] - x[k]))
            armed = False
    if len(tc) < 2:
        return float("nan")
    return (len(tc) - 1) / ((tc[-1] - tc[0]) * dt)
