"""D3Q19 lattice Boltzmann step in FP64 (test infrastructure; see
``oracle/__init__``): the three-dimensional extension of the method's step.

The paper works in two dimensions and names three-dimensional flows as the
next step (Sec. 5).  The D3Q19 step here carries over the two-dimensional
step of Secs. 2.1-2.3 one to one:

  * BGK collision (Eq. 2) with the second-order equilibrium (Eq. 3) and
    the moments of Eq. 4 on 19 velocities;
  * pull streaming (Eq. 1); a source outside the x-range is an unknown of
    the inlet or outlet face (this wins at edges and corners); a source
    outside the y- or z-range bounces back half-way off a wall or wraps
    round (periodic); a solid source bounces back half-way (Eq. 12 read as
    the half-way variant);
  * the momentum-exchange force (Eqs. 14-15) over the links into the body;
  * Zou & He faces (Sec. 2.2) carried to 3D: the density follows from the
    known populations and the normal velocity (Eqs. 5-7), each unknown
    population is the opposite one plus the equilibrium difference
    (non-equilibrium bounce-back, Eqs. 8-10), and the unknowns with a
    transverse component are corrected by -c_t . N, N chosen so that the
    node carries exactly the prescribed transverse momentum (the
    construction of Hecht & Harting 2010; in 2D it is the
    (f_4 - f_2)/2 term of Eqs. 8 and 10).  Velocity inlet at x = 0 with
    u = (u_in, 0, 0); pressure outlet at x = nx-1 with rho = rho_out and
    zero transverse velocity.

Populations are arrays f[q, z, y, x].  Numbering: q = 0 rest; 1-6 the
axis directions +x, -x, +y, -y, +z, -z; 7-18 the edge directions in
opposite pairs (2k+1, 2k+2).  Mask values: 0 fluid, 1 body (links to it
are force-summed).
"""
import numpy as np

C = np.array([[0, 0, 0],
              [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
              [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
              [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=np.int64)
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12, dtype=np.float64)
OPP = np.array([0] + [q + 1 if q % 2 else q - 1 for q in range(1, 19)], dtype=np.int64)
CS2 = 1.0 / 3.0


def equilibrium(rho, u):
    """Eq. 3 on D3Q19: f_i^eq = w_i rho (1 + c.u/cs^2 + (c.u)^2/(2cs^4) - u.u/(2cs^2)).
    rho (...), u (3, ...) -> (19, ...)."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    usq = (u * u).sum(axis=0)
    out = np.empty((19,) + rho.shape)
    for i in range(19):
        cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
        out[i] = W[i] * rho * (1 + cu / CS2 + cu * cu / (2 * CS2 * CS2) - usq / (2 * CS2))
    return out


def moments(f):
    """Eq. 4: rho and u (3, ...)."""
    rho = f.sum(axis=0)
    j = np.tensordot(C.T.astype(np.float64), f, axes=(1, 0))
    return rho, j / rho


def bgk_collide(f, tau):
    rho, u = moments(f)
    return f - (f - equilibrium(rho, u)) / tau


def face_unknowns(f, rho, u, side):
    """Complete a boundary face (f: (19, n) streamed populations, unknowns
    ignored) for the prescribed rho (n,) and u (3, n).  side 'in' (x = 0,
    unknowns c_x = +1) or 'out' (x = nx-1, unknowns c_x = -1)."""
    f = np.array(f, dtype=np.float64, copy=True)
    sgn = 1 if side == "in" else -1
    unk = [i for i in range(19) if C[i, 0] == sgn]
    feq = equilibrium(rho, u)
    for i in unk:                                   # non-equilibrium bounce-back
        f[i] = f[OPP[i]] + feq[i] - feq[OPP[i]]
    for a in (1, 2):                                # transverse momentum
        have = sum(C[i, a] * f[i] for i in range(19) if C[i, a] != 0)
        N = (have - rho * u[a]) / sum(C[i, a] ** 2 for i in unk)
        for i in unk:
            if C[i, a] != 0:
                f[i] = f[i] - C[i, a] * N
    return f


def inlet_density(f, ux):
    """Eq. 7 mirrored: rho = (rho_0 + 2 rho_-) / (1 - u_x) from the populations
    with c_x = 0 and c_x = -1."""
    r0 = sum(f[i] for i in range(19) if C[i, 0] == 0)
    rm = sum(f[i] for i in range(19) if C[i, 0] == -1)
    return (r0 + 2 * rm) / (1 - ux)


def outlet_velocity(f, rho_out):
    """Eq. 7: u_x = (rho_0 + 2 rho_+) / rho_out - 1."""
    r0 = sum(f[i] for i in range(19) if C[i, 0] == 0)
    rp = sum(f[i] for i in range(19) if C[i, 0] == 1)
    return (r0 + 2 * rp) / rho_out - 1


class Lattice3:
    """D3Q19 lattice, mask (nz, ny, nx) with 0 fluid / 1 body; lateral
    ('walls' or 'periodic', or a pair for y and z); xbc 'inout' or
    'periodic'.  State: pre-collision populations f[q, z, y, x]."""

    def __init__(self, mask, tau, *, lateral="walls", xbc="inout", u_in=0.05, rho_out=1.0):
        self.mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self.nz, self.ny, self.nx = self.mask.shape
        self.fluid = self.mask == 0
        self.tau = float(tau)
        self.lat_y, self.lat_z = (lateral, lateral) if isinstance(lateral, str) else lateral
        self.xbc = xbc
        self.u_in, self.rho_out = float(u_in), float(rho_out)
        u = np.zeros((3,) + self.mask.shape)
        u[0] = np.where(self.fluid, self.u_in, 0.0)
        self.f = equilibrium(np.ones(self.mask.shape), u)
        self.fx_hist, self.fy_hist, self.fz_hist = [], [], []

    def set_fields(self, rho, u):
        rho = np.where(self.fluid, rho, 1.0)
        u = np.where(self.fluid[None], u, 0.0)
        self.f = equilibrium(rho, u)

    def collide(self, f=None):
        f = self.f if f is None else f
        return np.where(self.fluid[None], bgk_collide(f, self.tau), f)

    def _source(self, c):
        Z, Y, X = np.mgrid[0:self.nz, 0:self.ny, 0:self.nx]
        sx, sy, sz = X - c[0], Y - c[1], Z - c[2]
        if self.xbc == "periodic":
            sx, xout = sx % self.nx, np.zeros(sx.shape, bool)
        else:
            xout = (sx < 0) | (sx >= self.nx)
        lout = np.zeros(sy.shape, bool)
        if self.lat_y == "periodic":
            sy = sy % self.ny
        else:
            lout |= (sy < 0) | (sy >= self.ny)
        if self.lat_z == "periodic":
            sz = sz % self.nz
        else:
            lout |= (sz < 0) | (sz >= self.nz)
        return (np.clip(sx, 0, self.nx - 1), np.clip(sy, 0, self.ny - 1),
                np.clip(sz, 0, self.nz - 1), xout, lout)

    def stream(self, fs):
        """Pull streaming with half-way bounce-back; unknowns are NaN."""
        out = np.empty_like(fs)
        for i in range(19):
            sx, sy, sz, xout, lout = self._source(C[i])
            solid = (self.mask[sz, sy, sx] != 0) & ~xout & ~lout
            bounce = (lout | solid) & ~xout
            val = np.where(bounce, fs[OPP[i]], fs[i][sz, sy, sx])
            out[i] = np.where(xout, np.nan, val)
        return out

    def momentum_exchange(self, fs, fn):
        """Eqs. 14-15 over every fluid-to-body link."""
        dP = np.zeros(3)
        for i in range(1, 19):
            sx, sy, sz, xout, lout = self._source(C[OPP[i]])     # x + c_i
            link = self.fluid & ~xout & ~lout & (self.mask[sz, sy, sx] == 1)
            if link.any():
                dP += fs[i][link].sum() * C[i] - fn[OPP[i]][link].sum() * C[OPP[i]]
        return dP

    def _advance(self, fs):
        fn = self.stream(fs)
        F = self.momentum_exchange(fs, fn)
        if self.xbc == "inout":
            col = fn[:, :, :, 0].reshape(19, -1)
            rho = inlet_density(col, self.u_in)
            u = np.zeros((3, col.shape[1]))
            u[0] = self.u_in
            fn[:, :, :, 0] = face_unknowns(col, rho, u, "in").reshape(19, self.nz, self.ny)
            col = fn[:, :, :, -1].reshape(19, -1)
            u = np.zeros((3, col.shape[1]))
            u[0] = outlet_velocity(col, self.rho_out)
            fn[:, :, :, -1] = face_unknowns(col, np.full(col.shape[1], self.rho_out), u,
                                            "out").reshape(19, self.nz, self.ny)
        return np.where(self.fluid[None], fn, fs), F

    def step(self, n=1):
        for _ in range(n):
            fn, F = self._advance(self.collide())
            self.f = np.where(self.fluid[None], fn, self.f)
            self.fx_hist.append(F[0])
            self.fy_hist.append(F[1])
            self.fz_hist.append(F[2])
        return self

    def advance_post(self, fs):
        """f*(t) -> f*(t+1) and F(t) without touching the stored state."""
        fn, F = self._advance(np.asarray(fs, dtype=np.float64))
        return self.collide(fn), F

    def post_collision(self):
        return self.collide()

    def momentum(self):
        fl = self.f[:, self.fluid]
        return np.array([(C[:, a, None] * fl).sum() for a in range(3)])
