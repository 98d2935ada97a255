"""Aerodynamic observables from the per-step force history (host side).

Sec. 2.3: drag and lift coefficients C = 2 F / (rho U^2 A) (Eq. 13) and the
Strouhal number St = f D / U from the dominant frequency of the lift
coefficient.  The frequency is the peak of the spectrum of the Hann-windowed,
mean-free lift signal, zero-padded 16-fold, refined by a Gaussian fit
through the logarithms of the peak bin and its two neighbours.
"""
import numpy as np


def coefficients(fx, fy, u_ref, length, rho_ref=1.0):
    """C_D and C_L time series from force histories (lattice units)."""
    k = 2.0 / (rho_ref * u_ref * u_ref * length)
    return k * np.asarray(fx, np.float64), k * np.asarray(fy, np.float64)


def peak_frequency(signal, dt=1.0, pad=16):
    s = np.asarray(signal, np.float64)
    s = (s - s.mean()) * np.hanning(s.size)
    mag = np.abs(np.fft.rfft(s, n=pad * s.size))
    freqs = np.fft.rfftfreq(pad * s.size, d=dt)
    k = 1 + int(np.argmax(mag[1:-1]))
    la, lb, lc = np.log(mag[k - 1:k + 2] + 1e-300)
    den = la - 2.0 * lb + lc
    shift = 0.5 * (la - lc) / den if den < 0 else 0.0
    return freqs[k] + shift * (freqs[1] - freqs[0])


def summarize(fx, fy, u_ref, length, window=0.4):
    """Mean C_D, mean C_L, rms of C_L - mean, St and lift amplitude over the
    last `window` fraction of the history."""
    cd, cl = coefficients(fx, fy, u_ref, length)
    n0 = int(len(cd) * (1.0 - window))
    cd, cl = cd[n0:], cl[n0:]
    f = peak_frequency(cl)
    h = len(cl) // 2
    halves = [float(np.sqrt(np.mean((c - c.mean()) ** 2))) for c in (cl[:h], cl[h:])]
    return {"cd_mean": float(cd.mean()), "cl_mean": float(cl.mean()),
            "cl_rms": float(np.sqrt(np.mean((cl - cl.mean()) ** 2))),
            "cl_amp": float(0.5 * (cl.max() - cl.min())), "st": float(f * length / u_ref),
            "samples": int(len(cd)),
            # rms of C_L - mean in the first and second half of the window:
            # equal within a few per cent once the shedding has saturated
            "cl_rms_halves": halves}


def relative_errors(test, ref):
    """Relative deviation of mean C_D, rms C_L and St of `test` from `ref`."""
    return {k: abs(test[k] - ref[k]) / abs(ref[k]) for k in ("cd_mean", "cl_rms", "st")}
