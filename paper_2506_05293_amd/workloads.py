"""Seeded synthetic workloads (input generators: geometry, sizes, physical
parameters; no lattice Boltzmann arithmetic).

All cases are cylinder or NACA0012 flows in lattice units with inlet speed
u_in = 0.05 and relaxation time tau = 3 nu + 1/2, nu = u_in L_ref / Re.
The paper's own data (a converged TCLB snapshot at Re = 200, literature
force coefficients) is not available; these cases stand in for it.
"""
import math

import numpy as np

from . import geometry

U_IN = 0.05


def tau_for(re, length, u=U_IN):
    return 3.0 * u * length / re + 0.5


def channel_cylinder(nx=4096, ny=1024, D=80, re=200.0):
    """Walled channel, cylinder of diameter D at x = 10 D, y = ny/2."""
    mask = geometry.cylinder(nx, ny, 10 * D, ny // 2, D)
    return dict(mask=mask, tau=tau_for(re, D), D=D, re=re)


def truncated_cylinder(downstream_d, D=64, re=200.0, ny=512, x_c=3583, tau=None):
    """Periodic-lateral cylinder lattice, ny = 8 D, cylinder centre at x_c,
    outlet `downstream_d` diameters behind the centre (4096 x 512 at 8 D,
    6144 x 512 at 40 D).  Acoustic scaling by default (u_in = U_IN, tau from
    Re); with `tau` given, diffusive scaling (tau fixed, u_in = Re nu / D)."""
    nx = x_c + int(downstream_d * D) + 1
    mask = geometry.cylinder(nx, ny, x_c, ny // 2, D)
    if tau is None:
        return dict(mask=mask, tau=tau_for(re, D), D=D, re=re, nx=nx, u_in=U_IN)
    u = re * (tau - 0.5) / 3.0 / D
    return dict(mask=mask, tau=float(tau), D=D, re=re, nx=nx, u_in=u)


def training_pairs(n_pairs=64, seed=3, d_range=(20, 40), ld_range=(8.0, 40.0),
                   re_range=(40.0, 400.0), long_d=40.0):
    """Pairs (long twin, truncated lattice) for the training data: D uniform
    in d_range (integers), height 8 D, centre 4 D behind the inlet, a
    truncated lattice whose outlet is L_d ~ U(ld_range) D behind the centre
    and a twin reaching long_d D; Re uniform in re_range.  Returns the
    lattice list for the batch (long twins log inputs and targets at the cut
    column, truncated lattices their own stencils there) and the pairs."""
    rng = np.random.default_rng(seed)
    lattices, pairs, row = [], [], 0
    for k in range(n_pairs):
        D = int(rng.integers(d_range[0], d_range[1] + 1))
        ny, x_c = 8 * D, 4 * D
        ld = int(round(rng.uniform(*ld_range) * D))
        re = float(rng.uniform(*re_range))
        tau = tau_for(re, D)
        x_cut = x_c + ld
        nx_long = x_c + int(long_d * D) + 1
        lseed = int(rng.integers(1, 2**62))
        long_mask = geometry.cylinder(nx_long, ny, x_c, ny // 2, D)
        short_mask = geometry.cylinder(x_cut + 1, ny, x_c, ny // 2, D)
        lattices.append(dict(mask=long_mask, tau=tau, u_in=U_IN, seed=lseed, log_role=1,
                             log_x=x_cut, log_row0=row))
        lattices.append(dict(mask=short_mask, tau=tau, u_in=U_IN, seed=lseed, log_role=2,
                             log_x=x_cut, log_row0=row))
        pairs.append(dict(D=D, ny=ny, re=re, tau=tau, ld=ld, x_cut=x_cut, row0=row,
                          long=2 * k, short=2 * k + 1))
        row += ny
    return lattices, pairs, row


def naca_case(aoa_deg, chord=256, nx=3072, ny=1024, after_te_chords=3.0, re=1000.0):
    """NACA0012 of chord c at angle of attack aoa_deg, quarter-chord pivot at
    mid-height, trailing edge `after_te_chords` chords before the outlet
    (3 C: 3072 x 1024; 12 C: the same placement on a 5376-wide lattice)."""
    px = 3072 - 1 - 3.0 * chord - 0.75 * chord        # fixed from the inlet
    nx = int(math.ceil(px + 0.75 * chord + after_te_chords * chord)) + 1
    mask = geometry.naca0012(nx, ny, chord, aoa_deg, (px, ny / 2.0))
    return dict(mask=mask, tau=tau_for(re, chord), chord=chord, re=re, nx=nx, aoa=aoa_deg)


def convected_vortex(nx=200, ny=400, ma=0.3, rc=20.0, beta=0.5, x0=150.0, re=750.0,
                     length=200.0):
    """Lamb-Oseen vortex in a uniform stream u0 = Ma c_s (Sec. 4.1): centre
    (x0, ny/2), core radius rc, strength beta; density from the isothermal
    radial pressure balance, rho = exp(-(beta u0)^2 / (2 c_s^2) e^{-r^2/rc^2});
    Re = u0 * length / nu.  Returns the mask, tau, the initial fields and u0.
    The reference lattice is the same with a larger nx."""
    cs2 = 1.0 / 3.0
    u0 = ma * math.sqrt(cs2)
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    y0 = ny / 2.0
    r2 = (x - x0) ** 2 + (y - y0) ** 2
    e = np.exp(-r2 / (2.0 * rc * rc))
    ux = u0 - beta * u0 * (y - y0) / rc * e
    uy = beta * u0 * (x - x0) / rc * e
    rho = np.exp(-(beta * u0) ** 2 / (2.0 * cs2) * np.exp(-r2 / (rc * rc)))
    nu = u0 * length / re
    return dict(mask=np.zeros((ny, nx), np.uint8), tau=3.0 * nu + 0.5, rho=rho, ux=ux, uy=uy,
                u0=u0, ma=ma, nx=nx, ny=ny)


def smooth_fields(shape, u_in, amp=0.02, modes=4, seed=0):
    """Seeded smooth initial fields on a lattice of `shape` ((ny, nx) or
    (nz, ny, nx)): rho = 1 + a sum of `modes` sine modes of amplitude
    amp / modes, and u = (u_in, 0[, 0]) plus such sums in every component;
    wavenumbers 1..4 along each axis and phases are drawn from
    default_rng(seed).  Returns rho and u (components first)."""
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")

    def field():
        f = np.zeros(shape)
        for _ in range(modes):
            arg = sum(2.0 * math.pi * rng.integers(1, 5) * g / n + rng.uniform(0, 2 * math.pi)
                      for g, n in zip(grids, shape))
            f += amp / modes * np.sin(arg)
        return f
    rho = 1.0 + field()
    u = np.stack([field() for _ in shape][::-1])       # x component first
    u[0] += u_in
    return rho, u
