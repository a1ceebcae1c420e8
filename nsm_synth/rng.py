"""SplitMix64 counter-based generator (Steele, Lea, Flood, OOPSLA 2014)."""
import math

import numpy as np

_GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK = (1 << 64) - 1


def _mix(z):
    z = ((z ^ (z >> 30)) * _M1) & _MASK
    z = ((z ^ (z >> 27)) * _M2) & _MASK
    return z ^ (z >> 31)


def _mix_np(z):
    z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
    return z ^ (z >> np.uint64(31))


class SplitMix64:
    """Sequential SplitMix64 stream with float64 helpers.

    ``next_u64`` follows the published definition: add the golden-ratio
    increment to the state, then apply the two xor-shift-multiply rounds.
    """

    def __init__(self, seed):
        self.state = int(seed) & _MASK

    def next_u64(self):
        self.state = (self.state + _GOLDEN) & _MASK
        return _mix(self.state)

    def uniform(self, lo=0.0, hi=1.0):
        u = (self.next_u64() >> 11) * (1.0 / (1 << 53))
        return lo + (hi - lo) * u

    def uniforms(self, n, lo=0.0, hi=1.0):
        """``n`` consecutive draws, vectorised (same values as ``uniform``)."""
        n = int(n)
        if n == 0:
            return np.zeros(0, np.float64)
        with np.errstate(over="ignore"):
            k = np.arange(1, n + 1, dtype=np.uint64)
            st = np.uint64(self.state) + k * np.uint64(_GOLDEN)
            z = _mix_np(st)
        self.state = (self.state + n * _GOLDEN) & _MASK
        u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
        return lo + (hi - lo) * u

    def normals(self, n):
        """Standard normal draws by the Box-Muller transform."""
        m = (int(n) + 1) // 2
        u = self.uniforms(2 * m)
        u1 = 1.0 - u[0::2]  # (0, 1]
        u2 = u[1::2]
        r = np.sqrt(-2.0 * np.log(u1))
        z = np.concatenate([r * np.cos(2 * math.pi * u2), r * np.sin(2 * math.pi * u2)])
        return z[: int(n)]

    def fork(self, tag):
        """An independent child stream keyed by an integer tag."""
        return SplitMix64(_mix((self.state ^ (int(tag) * _M2)) & _MASK))
