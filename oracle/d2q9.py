"""D2Q9 lattice core in FP64 (test infrastructure; see ``oracle/__init__``).

Populations are arrays ``f[q, y, x]``.  Velocity numbering follows the
standard D2Q9 convention that makes {3, 6, 7} the unknown populations at a
right boundary and {1, 5, 8} at a left one (Sec. 2.2, Zou and He boundary
condition):

    q :   0      1      2      3       4      5      6       7        8
    c : (0,0)  (1,0)  (0,1)  (-1,0)  (0,-1)  (1,1)  (-1,1)  (-1,-1)  (1,-1)
    w :  4/9    1/9    1/9    1/9     1/9    1/36   1/36    1/36     1/36
"""
import numpy as np

C = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1],
              [1, 1], [-1, 1], [-1, -1], [1, -1]], dtype=np.int64)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=np.float64)
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6], dtype=np.int64)
CS2 = 1.0 / 3.0          # squared lattice speed of sound


def equilibrium(rho, ux, uy):
    """Second-order equilibrium, Sec. 2.1 Eq. 3:
    f_i^eq = w_i rho (1 + u.c_i/cs^2 + (u.c_i)^2/(2 cs^4) - u.u/(2 cs^2))."""
    rho = np.asarray(rho, dtype=np.float64)
    ux = np.asarray(ux, dtype=np.float64)
    uy = np.asarray(uy, dtype=np.float64)
    shape = np.broadcast(rho, ux, uy).shape
    feq = np.empty((9,) + shape)
    usq = ux * ux + uy * uy
    for i in range(9):
        cu = C[i, 0] * ux + C[i, 1] * uy
        feq[i] = W[i] * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2)
                               - usq / (2.0 * CS2))
    return feq


def moments(f):
    """Density and velocity from the populations, Sec. 2.1 Eq. 4:
    rho = sum_i f_i, rho u = sum_i c_i f_i."""
    rho = f.sum(axis=0)
    jx = np.tensordot(C[:, 0].astype(np.float64), f, axes=(0, 0))
    jy = np.tensordot(C[:, 1].astype(np.float64), f, axes=(0, 0))
    return rho, jx / rho, jy / rho


def tau_from_viscosity(nu):
    """BGK relaxation time tied to the kinematic viscosity (Sec. 2.1, after
    Eq. 2), in lattice units: nu = cs^2 (tau - 1/2)."""
    return nu / CS2 + 0.5


def bgk_collide(f, tau):
    """BGK collision, Sec. 2.1 Eqs. 1-2: f* = f - (f - f^eq)/tau."""
    rho, ux, uy = moments(f)
    return f - (f - equilibrium(rho, ux, uy)) / tau


# --- MRT -------------------------------------------------------------------
# The paper names the multi-relaxation-time operator (Sec. 3.2) without
# defining it.  Reading: the orthogonal Lallemand-Luo moment basis
# (rho, e, eps, jx, qx, jy, qy, pxx, pxy), equilibrium moments taken as the
# moments of the same quadratic equilibrium (m^eq = M f^eq), shear rate
# s_nu = 1/tau and free rates s_e, s_eps, s_q.
MRT_M = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],            # rho
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],       # e
    [4, -2, -2, -2, -2, 1, 1, 1, 1],        # eps
    [0, 1, 0, -1, 0, 1, -1, -1, 1],         # jx
    [0, -2, 0, 2, 0, 1, -1, -1, 1],         # qx
    [0, 0, 1, 0, -1, 1, 1, -1, -1],         # jy
    [0, 0, -2, 0, 2, 1, 1, -1, -1],         # qy
    [0, 1, -1, 1, -1, 0, 0, 0, 0],          # pxx
    [0, 0, 0, 0, 0, 1, -1, 1, -1],          # pxy
], dtype=np.float64)


def mrt_magic_sq(tau):
    """s_q that fixes the two-relaxation-time 'magic' combination
    (1/s_nu - 1/2)(1/s_q - 1/2) = 3/16 with s_nu = 1/tau."""
    return 1.0 / (0.5 + (3.0 / 16.0) / (tau - 0.5))


def mrt_rates(tau, s_e=1.0, s_eps=1.0, s_q=None):
    """Relaxation matrix diagonal in the MRT_M row order."""
    if s_q is None or s_q <= 0:
        s_q = mrt_magic_sq(tau)
    s_nu = 1.0 / tau
    return np.array([0.0, s_e, s_eps, 0.0, s_q, 0.0, s_q, s_nu, s_nu])


def mrt_collide(f, tau, s_e=1.0, s_eps=1.0, s_q=None):
    """MRT collision f* = f - M^-1 S (M f - M f^eq), with M^-1 from a
    library inverse and the equilibrium of Eq. 3."""
    S = mrt_rates(tau, s_e, s_eps, s_q)
    Minv = np.linalg.inv(MRT_M)
    rho, ux, uy = moments(f)
    m = np.tensordot(MRT_M, f, axes=(1, 0))
    meq = np.tensordot(MRT_M, equilibrium(rho, ux, uy), axes=(1, 0))
    dm = S.reshape((9,) + (1,) * (f.ndim - 1)) * (m - meq)
    return f - np.tensordot(Minv, dm, axes=(1, 0))
