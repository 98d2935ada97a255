"""SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), generated sequentially
(test infrastructure; see ``oracle/__init__``).

The state advances by the golden-ratio increment 0x9e3779b97f4a7c15 and each
output is the state passed through the variant-13 finaliser.  The initial
velocity noise of a lattice draws output k (k >= 1) for node (x, y) and
component comp (0 = u_x, 1 = u_y) at k = 2 (y nx + x) + comp + 1, and maps it
to a uniform number U = (out >> 11) 2^-53 and a noise value a (2U - 1).
"""
import numpy as np

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


class SplitMix64:
    def __init__(self, seed):
        self.state = int(seed) & _MASK

    def next(self):
        self.state = (self.state + _GAMMA) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)


def sequence(seed, n):
    """The first n outputs, as a uint64 array (vectorised by stepping the
    whole sequence of states at once; identical to calling next() n times)."""
    k = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(int(seed) & _MASK) + k * np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def velocity_noise(seed, nx, ny, amp):
    """Noise fields (nu_x, nu_y), each (ny, nx), drawn as described above."""
    out = sequence(seed, 2 * nx * ny).reshape(ny, nx, 2)
    u01 = (out >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    noise = amp * (2.0 * u01 - 1.0)
    return noise[..., 0], noise[..., 1]
