"""Zou & He boundary columns in FP64 (test infrastructure; see
``oracle/__init__``).

Sec. 2.2: the density at a boundary node follows from the known populations
and the normal velocity (Eqs. 5-7); the unknown populations are the
equilibrium plus the non-equilibrium part of the opposite population, with a
transverse correction (Eqs. 8-10); all other populations stay as streamed
(Eq. 11); the other sides follow by symmetry.

Readings where the paper is silent or garbled:
  * Eq. 6 prints f_1 + f_2 + f_3; only rho u = rho+ - (f_3 + f_6 + f_7)
    yields Eq. 7, so that is what is used.
  * The pressure outlet prescribes rho = rho_out and v = 0 (the original
    Zou & He pressure condition); the velocity inlet prescribes (u_in, 0) or
    a per-row profile u_in(y).
  * The inlet is the left-side mirror (x -> -x maps 1<->3, 5<->6, 8<->7).
"""
import numpy as np

from .d2q9 import equilibrium


def outlet_reconstruct(fcol, rho, u, v):
    """Right boundary (x = L): the unknowns 3, 6, 7 from Eqs. 8-10 for a
    prescribed density and velocity (rho, u, v), each a scalar or per node;
    the known populations are kept (Eq. 11)."""
    f = np.array(fcol, dtype=np.float64, copy=True)
    n = f.shape[1]
    rho, u, v = (np.broadcast_to(np.asarray(a, dtype=np.float64), (n,)) for a in (rho, u, v))
    feq = equilibrium(rho, u, v)
    fneq = f - feq
    f[6] = feq[6] + fneq[8] + 0.5 * (fneq[4] - fneq[2])   # Eq. 8
    f[3] = feq[3] + fneq[1]                                # Eq. 9
    f[7] = feq[7] + fneq[5] - 0.5 * (fneq[4] - fneq[2])   # Eq. 10
    return f


def outlet_pressure(fcol, rho_out):
    """Right boundary (x = L), unknowns 3, 6, 7.

    ``fcol`` is (9, n): the populations of the boundary nodes after streaming,
    with the unknown entries ignored.  Returns the completed (9, n) array and
    the normal velocity u from Eq. 7 solved for u at the prescribed rho."""
    f = np.asarray(fcol, dtype=np.float64)
    rho0 = f[0] + f[2] + f[4]
    rhop = f[1] + f[5] + f[8]
    rho = np.full(f.shape[1], float(rho_out))
    u = (rho0 + 2.0 * rhop) / rho - 1.0          # Eq. 7
    return outlet_reconstruct(f, rho, u, 0.0), u


def inlet_velocity(fcol, ux, uy=0.0):
    """Left boundary (x = 0), unknowns 1, 5, 8; mirror of Eqs. 7-10.

    ``ux`` may be a scalar or a per-node array.  Returns the completed
    populations and the density from the mirrored Eq. 7."""
    f = np.array(fcol, dtype=np.float64, copy=True)
    n = f.shape[1]
    ux = np.broadcast_to(np.asarray(ux, dtype=np.float64), (n,))
    uy = np.broadcast_to(np.asarray(uy, dtype=np.float64), (n,))
    rho0 = f[0] + f[2] + f[4]
    rhom = f[3] + f[6] + f[7]
    rho = (rho0 + 2.0 * rhom) / (1.0 - ux)        # Eq. 7 mirrored
    feq = equilibrium(rho, ux, uy)
    fneq = f - feq
    f[5] = feq[5] + fneq[7] + 0.5 * (fneq[4] - fneq[2])   # mirror of Eq. 8
    f[1] = feq[1] + fneq[3]                                # mirror of Eq. 9
    f[8] = feq[8] + fneq[6] - 0.5 * (fneq[4] - fneq[2])   # mirror of Eq. 10
    return f, rho
