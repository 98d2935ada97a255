"""The D2Q9 time step in FP64 (test infrastructure; see ``oracle/__init__``).

State: the pre-collision populations f(t) of Eq. 1, array f[q, y, x].
One step t -> t+1, in the order the paper's method implies:

  1. moments (Eq. 4) and collision (BGK Eq. 2, or MRT) on fluid nodes -> f*;
  2. pull streaming f_i(x, t+1) = f*_i(x - c_i, t) (Eq. 1), where
       * a source left of column 0 or right of column nx-1 is an unknown
         population, filled in step 4 (this wins at corners);
       * a source outside rows [0, ny) bounces back off a wall (half-way) or
         wraps round (periodic laterals, Fig. 2);
       * a solid source bounces back half-way: f_i(x, t+1) = f*_ibar(x, t)
         (Eq. 12 read as the half-way variant);
  3. the momentum-exchange force of Eq. 14 over every fluid-to-body link,
     F(t) = Delta P / Delta t (Eq. 15), lattice units (Delta x = Delta t = 1);
  4. boundary columns: Zou & He velocity inlet at x = 0; at x = nx-1 the
     Zou & He pressure outlet, the neural reconstruction of Eq. 16 with a
     per-node Zou & He fallback, or the characteristic outflow of Sec. 4
     (oracle/cbc.py) from the state of the three last columns at time t.

Geometry mask values: 0 fluid, 1 body (links to it are force-summed),
2 inert solid (bounce-back only).  Solid nodes are never updated.
"""
import numpy as np

from . import cbc, d2q9
from .d2q9 import C, OPP, W
from .mlp import forward_bf16
from .splitmix64 import velocity_noise
from .zouhe import inlet_velocity, outlet_pressure


class Lattice:
    def __init__(self, mask, tau, *, collision="bgk", s_e=1.0, s_eps=1.0,
                 s_q=None, lateral="walls", xbc="inout", u_in=0.05,
                 inlet_profile=None, rho_out=1.0, noise_amp=0.0, seed=0):
        self.mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self.ny, self.nx = self.mask.shape
        self.fluid = self.mask == 0
        self.tau = float(tau)
        self.collision = collision
        self.mrt = (s_e, s_eps, s_q)
        assert lateral in ("walls", "periodic") and xbc in ("inout", "periodic")
        self.lateral, self.xbc = lateral, xbc
        self.u_in = float(u_in)
        self.inlet_profile = None if inlet_profile is None else \
            np.asarray(inlet_profile, dtype=np.float64)
        self.rho_out = float(rho_out)
        self.outflow = "zouhe"
        self.mlp = None
        self.mass_bound = 1e-2
        self.cbc = None
        self.cbc_prev = np.zeros((self.ny, 3))
        self.t = 0
        self.fx_hist, self.fy_hist, self.mass_hist = [], [], []
        self.n_fallback = 0
        # Initial state: f^eq(1, (u_in, 0) + noise) on fluid, f^eq(1, 0) on
        # solid nodes.
        nux, nuy = velocity_noise(seed, self.nx, self.ny, noise_amp)
        ux = np.where(self.fluid, self.u_in + nux, 0.0)
        uy = np.where(self.fluid, nuy, 0.0)
        self.f = d2q9.equilibrium(np.ones((self.ny, self.nx)), ux, uy)

    # -- configuration ------------------------------------------------------
    def set_equilibrium(self, rho, ux, uy):
        """Replace the state by f^eq(rho, u) (solid nodes: f^eq(1, 0))."""
        rho = np.where(self.fluid, rho, 1.0)
        self.f = d2q9.equilibrium(rho, np.where(self.fluid, ux, 0.0),
                                  np.where(self.fluid, uy, 0.0))

    def set_outflow_nn(self, P, mass_bound=1e-2):
        """Use the neural reconstruction (Eq. 16) at the outlet column."""
        self.outflow, self.mlp, self.mass_bound = "nn", P, float(mass_bound)

    def set_outflow_cbc(self, sigma=0.0, kappa2=0.0, mach=0.0, length=None, rho_inf=1.0,
                        net=None):
        """Use the characteristic outflow of Sec. 4 (Eqs. 18-29), with fixed
        sigma and kappa_2 or, given ``net``, the tuning network.  Periodic
        laterals only: the section gives no treatment of the corners where
        the outlet meets a no-slip wall."""
        if self.lateral != "periodic":
            raise ValueError("the characteristic outflow needs periodic laterals")
        self.outflow = "cbc"
        self.cbc = dict(sigma=float(sigma), kappa2=float(kappa2), mach=float(mach),
                        length=float(self.nx if length is None else length),
                        rho_inf=float(rho_inf), net=net)
        self.cbc_prev = np.zeros((self.ny, 3))

    def set_outflow_zouhe(self):
        self.outflow, self.mlp = "zouhe", None

    # -- the step -----------------------------------------------------------
    def collide(self, f=None):
        """Post-collision populations f* on fluid nodes (solid nodes copied)."""
        f = self.f if f is None else f
        if self.collision == "bgk":
            fs = d2q9.bgk_collide(f, self.tau)
        else:
            fs = d2q9.mrt_collide(f, self.tau, *self.mrt)
        return np.where(self.fluid[None], fs, f)

    def _source(self, cx, cy):
        """Source indices of the pull x - c for every node, with the flags
        'x outside' and 'y outside' after the lateral/periodic rules."""
        Y, X = np.mgrid[0:self.ny, 0:self.nx]
        sx, sy = X - cx, Y - cy
        if self.xbc == "periodic":
            sx, xout = sx % self.nx, np.zeros_like(sx, dtype=bool)
        else:
            xout = (sx < 0) | (sx >= self.nx)
        if self.lateral == "periodic":
            sy, yout = sy % self.ny, np.zeros_like(sy, dtype=bool)
        else:
            yout = (sy < 0) | (sy >= self.ny)
        return np.clip(sx, 0, self.nx - 1), np.clip(sy, 0, self.ny - 1), xout, yout

    def stream(self, fstar):
        """Pull streaming with half-way bounce-back.  Unknown entries (source
        outside the x-range) are returned as NaN."""
        fnew = np.empty_like(fstar)
        for i in range(9):
            sx, sy, xout, yout = self._source(C[i, 0], C[i, 1])
            solid_src = (self.mask[sy, sx] != 0) & ~xout & ~yout
            bounce = (yout | solid_src) & ~xout
            val = np.where(bounce, fstar[OPP[i]], fstar[i][sy, sx])
            fnew[i] = np.where(xout, np.nan, val)
        return fnew

    def _links(self, i):
        """Fluid nodes whose neighbour x + c_i is a body node."""
        # x + c_i is the pull source of direction OPP[i].
        cx, cy = C[OPP[i]]
        sx, sy, xout, yout = self._source(cx, cy)
        return self.fluid & ~xout & ~yout & (self.mask[sy, sx] == 1)

    def momentum_exchange(self, fstar, fnew):
        """Eq. 14-15: Delta P = sum over links (f_i^in c_i - f_ibar^out c_ibar),
        f^in the post-collision population moving into the body, f^out the
        population that comes back to the same fluid node."""
        dP = np.zeros(2)
        for i in range(1, 9):
            link = self._links(i)
            if not link.any():
                continue
            f_in = fstar[i][link].sum()
            f_out = fnew[OPP[i]][link].sum()
            dP += f_in * C[i] - f_out * C[OPP[i]]
        return dP          # / Delta t = 1

    def nn_outlet(self, fnew):
        """Eq. 16 at the outlet column with the Zou & He fallback, from the
        pre-collision populations ``fnew`` of the next step (the outlet
        unknowns may be NaN).  Returns a dict: ``nn`` and ``zh`` the outlet
        column (9, ny) reconstructed both ways, ``ok`` the per-row decision
        (True: the reconstruction is kept), ``jump`` the FP32 density jump
        |rho_g - rho(L-1)| the decision compared with the bound, ``positive``
        the FP32 positivity test.

        The decision is a floating-point test that selects between two
        results, so it is taken in the kernel's precision: positivity of the
        reconstructed absolute populations rounded to FP32, and the density
        jump as the difference of the two densities' offsets rho - 1 (summed
        in FP64 from f - w, each rounded to FP32), subtracted and compared in
        FP32."""
        L = self.nx - 1
        feats = np.concatenate([(fnew[:, :, L - 1 - j] - W[:, None]).T
                                for j in range(3)], axis=1)      # (ny, 27)
        n_in = np.shape(self.mlp["w1"])[1]      # 9: the paper's column L-1 only
        s = forward_bf16(feats[:, :n_in], self.mlp)              # (ny, 3)
        g = fnew[:, :, L].copy()
        for k, q in enumerate((3, 6, 7)):
            g[q] = fnew[q, :, L - 1] + s[:, k]
        zh, _ = outlet_pressure(fnew[:, :, L], self.rho_out)
        g32 = g.astype(np.float32)
        positive = np.all(g32[[3, 6, 7]] > 0, axis=0)
        drho_g = (g - W[:, None]).sum(0).astype(np.float32)
        drho_prev = (fnew[:, :, L - 1] - W[:, None]).sum(0).astype(np.float32)
        jump = np.abs(drho_g - drho_prev)                         # FP32
        ok = positive & (jump < np.float32(self.mass_bound))
        return {"nn": g, "zh": zh, "ok": ok, "jump": jump, "positive": positive}

    def _outlet_nn(self, fnew):
        r = self.nn_outlet(fnew)
        self.n_fallback += int((~r["ok"]).sum())
        return np.where(r["ok"][None], r["nn"], r["zh"])

    def nn_outlet_candidates(self, fstar):
        """For a post-collision state fstar(t): the post-collision outlet
        column of step t+1 with the reconstruction kept at every row
        (``post_nn``) and with the Zou & He fallback at every row
        (``post_zh``), and the per-row decision the step takes (``ok``,
        ``jump``, ``positive`` as in nn_outlet).  Does not touch the state."""
        fnew = self.stream(np.asarray(fstar, dtype=np.float64))
        if self.xbc == "inout":
            ux = self.u_in if self.inlet_profile is None else self.inlet_profile
            fnew[:, :, 0], _ = inlet_velocity(fnew[:, :, 0], ux, 0.0)
        r = self.nn_outlet(fnew)
        out = {k: r[k] for k in ("ok", "jump", "positive")}
        for name in ("nn", "zh"):
            f = fnew.copy()
            f[:, :, -1] = r[name]
            f = np.where(self.fluid[None], f, fstar)
            out["post_" + name] = self.collide(f)[:, :, -1]
        return out

    def _advance(self, fstar):
        """Streaming, force and boundary columns from the post-collision
        state fstar: returns the pre-collision populations of the next step
        and the force F of this step."""
        fnew = self.stream(fstar)
        F = self.momentum_exchange(fstar, fnew)
        if self.xbc == "inout":
            ux = self.u_in if self.inlet_profile is None else self.inlet_profile
            fnew[:, :, 0], _ = inlet_velocity(fnew[:, :, 0], ux, 0.0)
            if self.outflow == "nn":
                fnew[:, :, -1] = self._outlet_nn(fnew)
            elif self.outflow == "cbc":
                rho, ux, uy = d2q9.moments(fstar[:, :, -3:])      # state at time t
                fnew[:, :, -1], self.cbc_prev = cbc.outlet(
                    fnew[:, :, -1], rho.T, ux.T, uy.T, self.cbc_prev, self.cbc,
                    self.lateral == "periodic")
            else:
                fnew[:, :, -1], _ = outlet_pressure(fnew[:, :, -1], self.rho_out)
        return np.where(self.fluid[None], fnew, fstar), F

    def step(self, n=1):
        for _ in range(n):
            fnew, F = self._advance(self.collide())
            self.f = np.where(self.fluid[None], fnew, self.f)
            self.fx_hist.append(F[0])
            self.fy_hist.append(F[1])
            self.mass_hist.append(self.f[:, self.fluid].sum())
            self.t += 1
        return self

    def advance_post(self, fstar):
        """One step expressed on post-collision states: f*(t) -> f*(t+1)
        (and F(t)).  Does not touch the stored state."""
        fnew, F = self._advance(np.asarray(fstar, dtype=np.float64))
        return self.collide(fnew), F

    # -- read-out -------------------------------------------------------------
    def post_collision(self):
        """f*(t): the collided state (fluid nodes), solid nodes as stored."""
        return self.collide()

    def macroscopic(self):
        return d2q9.moments(self.f)

    def momentum(self):
        """Total momentum sum_x sum_i c_i f_i over fluid nodes."""
        fl = self.f[:, self.fluid]
        return np.array([(C[:, 0, None] * fl).sum(), (C[:, 1, None] * fl).sum()])
