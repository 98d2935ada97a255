"""Geometry masks for the lattice (host side, NumPy only).

Mask values, row-major (ny, nx), y up, node centres at integers:
  0 fluid, 1 body (links into it are summed into the momentum-exchange
  force), 2 inert solid (bounce-back only, no force).

These builders are input generators: they hold no lattice Boltzmann
arithmetic and are used alike by the library's callers and by its tests.
"""
import math

import numpy as np

# NACA four-digit thickness polynomial with the closed trailing edge,
# Appendix A Eq. A.1: y = +-a0 (a1 sqrt(s) + a2 s + a3 s^2 + a4 s^3 + a5 s^4).
NACA0012_COEF = (0.594689181, 0.298222773, -0.127125232, -0.357907906,
                 0.291984971, -0.105174606)


def naca0012_half_thickness(s):
    """Half thickness y_t(s)/c at chord fraction s in [0, 1] (Eq. A.1)."""
    a0, a1, a2, a3, a4, a5 = NACA0012_COEF
    s = np.asarray(s, dtype=np.float64)
    return a0 * (a1 * np.sqrt(s) + a2 * s + a3 * s**2 + a4 * s**3 + a5 * s**4)


def cylinder(nx, ny, xc, yc, diameter, value=1):
    """Solid iff (x - xc)^2 + (y - yc)^2 <= (D/2)^2 (Fig. 2 geometry)."""
    Y, X = np.mgrid[0:ny, 0:nx]
    r2 = (X - xc) ** 2 + (Y - yc) ** 2
    m = np.zeros((ny, nx), dtype=np.uint8)
    m[r2 <= (diameter / 2.0) ** 2] = value
    return m


def naca0012(nx, ny, chord, aoa_deg, pivot, value=1):
    """NACA0012 at angle of attack ``aoa_deg`` (positive = nose up for flow
    in +x) rotated about ``pivot`` = (px, py), the quarter-chord point.  A
    node is solid iff its chord coordinate s lies in [0, 1] and its normal
    distance is within the half thickness (binary mask, no sub-node
    interpolation)."""
    a = math.radians(aoa_deg)
    Y, X = np.mgrid[0:ny, 0:nx].astype(np.float64)
    dx, dy = X - pivot[0], Y - pivot[1]
    xi = math.cos(a) * dx - math.sin(a) * dy
    eta = math.sin(a) * dx + math.cos(a) * dy
    s = xi / chord + 0.25
    inside = (s >= 0.0) & (s <= 1.0)
    yt = np.zeros_like(s)
    yt[inside] = chord * naca0012_half_thickness(s[inside])
    m = np.zeros((ny, nx), dtype=np.uint8)
    m[inside & (np.abs(eta) <= yt)] = value
    return m


def channel_walls(nx, ny):
    """An empty lattice (all fluid)."""
    return np.zeros((ny, nx), dtype=np.uint8)
