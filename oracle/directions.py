"""Random directions xi_1..xi_P uniform on S^{d-1} (Algorithm "alg:fast_Fourier_sliced", first step).

The paper only says "draw P random directions"; the generator is fixed here so
that the GPU library and the oracle can draw the same directions independently:

  * SplitMix64 (Steele, Lea, Flood 2014): the c-th output (c = 0, 1, ...) for a
    seed s is mix(s + (c+1) * 0x9E3779B97F4A7C15 mod 2^64), where
    mix(z): z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
            z *= 0x94D049BB133111EB; z ^= z >> 31.
  * coordinate i of direction p uses the two outputs c = 2(p*d + i) and c+1:
    u1 = ((o1 >> 11) + 1) * 2^-53 in (0,1],  u2 = (o2 >> 11) * 2^-53 in [0,1),
    g = sqrt(-2 ln u1) * cos(2 pi u2)      (Box-Muller, cosine branch),
  * xi_p = g_p / ||g_p||, the squared norm summed in coordinate order.

Normalising a standard Gaussian vector gives the uniform distribution on the
sphere.  Because the counter only depends on (p, i, d), the first Q directions
of a P-direction set equal the Q-direction set for the same seed and d.
"""
from __future__ import annotations

import math

import numpy as np

_MASK = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


def splitmix64(seed: int, c: int) -> int:
    """The c-th SplitMix64 output (0-based) of a generator seeded with `seed`."""
    z = (seed + (c + 1) * _GOLDEN) & _MASK
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & _MASK
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & _MASK
    z ^= z >> 31
    return z


def gaussian(seed: int, p: int, i: int, d: int) -> float:
    c = 2 * (p * d + i)
    o1 = splitmix64(seed, c)
    o2 = splitmix64(seed, c + 1)
    u1 = ((o1 >> 11) + 1) * (2.0 ** -53)
    u2 = (o2 >> 11) * (2.0 ** -53)
    return math.sqrt(-2.0 * math.log(u1)) * math.cos(6.283185307179586 * u2)


def directions(d: int, P: int, seed: int) -> np.ndarray:
    """(P, d) FP64 array of unit vectors; row p is xi_p."""
    out = np.empty((P, d), dtype=np.float64)
    for p in range(P):
        g = [gaussian(seed, p, i, d) for i in range(d)]
        nrm2 = 0.0
        for v in g:
            nrm2 += v * v
        nrm = math.sqrt(nrm2)
        for i in range(d):
            out[p, i] = g[i] / nrm
    return out
