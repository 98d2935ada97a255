"""Seeded synthetic cases shared by the tests (inputs only: sizes, masks,
physical parameters).  Sizes follow the paper's cylinder workloads scaled to
what the oracle finishes in seconds, plus the full-size lattices."""
import numpy as np

from paper_2506_05293_amd import geometry


def c1(re=100.0, collision="bgk"):
    """Channel 200 x 80, walls, cylinder D = 20 at (40, 40), BGK, Re = 100
    (nu = u D / Re = 0.01, tau = 0.53), u_in = 0.05, noise 1e-4, seed 1.
    With BGK this literal case diverges after ~500 steps (from the Zou & He
    inlet); Re = 75 (tau = 0.54) is the lowest-tau BGK variant that stays
    finite, and MRT is stable at Re = 100."""
    nx, ny = 200, 80
    return dict(mask=geometry.cylinder(nx, ny, 40, 40, 20.0), tau=3 * 0.05 * 20 / re + 0.5,
                collision=collision, lateral="walls", u_in=0.05, noise_amp=1e-4, seed=1)


def ragged(collision="mrt", lateral="periodic"):
    """A lattice whose sizes are no multiple of any tile (203 x 77), with a
    body and an inert solid touching the lateral edges."""
    nx, ny = 203, 77
    m = geometry.cylinder(nx, ny, 51.3, 37.6, 17.0)
    m[0:3, 120:124] = 2
    m[74:77, 150:152] = 1
    return dict(mask=m, tau=0.56, collision=collision, lateral=lateral, u_in=0.06,
                noise_amp=1e-3, seed=7)


def c2(nx=4096, ny=1024):
    """Channel 4096 x 1024, walls, cylinder D = 80 at x = 10 D, MRT, Re = 200
    (nu = 0.02, tau = 0.56), u_in = 0.05, noise 1e-4, seed 2."""
    D = 80.0 * nx / 4096
    return dict(mask=geometry.cylinder(nx, ny, 10 * D, ny // 2, D), tau=3 * 0.05 * D / 200 + 0.5,
                collision="mrt", lateral="walls", u_in=0.05, noise_amp=1e-4, seed=2)


def oracle_kwargs(case):
    keys = ("tau", "collision", "lateral", "u_in", "noise_amp", "seed")
    return {k: case[k] for k in keys}


def random_params(seed, w_scale=1.0, out_sd=1e-3):
    """A seeded 27-64-64-3 outflow network (Glorot-uniform weights scaled by
    w_scale, output standardisation of scale out_sd)."""
    rng = np.random.default_rng(seed)

    def glorot(o, i):
        a = np.sqrt(6.0 / (o + i)) * w_scale
        return rng.uniform(-a, a, (o, i))
    return {"w1": glorot(64, 27), "b1": 0.1 * rng.standard_normal(64),
            "w2": glorot(64, 64), "b2": 0.1 * rng.standard_normal(64),
            "w3": glorot(3, 64), "b3": 0.1 * rng.standard_normal(3),
            "mu_in": 0.002 * rng.standard_normal(27), "sd_in": 0.01 + 0.01 * rng.random(27),
            "mu_out": 1e-4 * rng.standard_normal(3), "sd_out": out_sd * (1 + rng.random(3))}


def f32_values(P):
    """The network's values rounded to FP32 (the form the step holds)."""
    return {k: np.asarray(v, np.float32).astype(np.float64) for k, v in P.items()}

