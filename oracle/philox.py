"""Philox4x32-10 counter-based generator and Gaussian test matrices (NumPy).

Test infrastructure (see the package docstring); imports nothing from the GPU path.

Philox4x32 with 10 rounds is the generator of Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
as easy as 1, 2, 3" (SC'11): a 4 x 32-bit counter and a 2 x 32-bit key; each round multiplies
counter words 0 and 2 by the constants M0, M1, recombines the high / low halves with words 1, 3 and
the key, and the key is advanced by the Weyl constants W0, W1 between rounds.

Gaussian entry Omega[i, j] of the p x ell test matrix (rows i = 2m, 2m + 1 share one call):
counter = (m, j, counter_lo, counter_hi), key = (seed_lo, seed_hi); two 53-bit uniforms in (0, 1)
u1 = ((x0 >> 5) 2^26 + (x1 >> 6) + 1/2) 2^-53, u2 likewise from (x2, x3); Box-Muller
Omega[2m, j] = sqrt(-2 ln u1) cos(2 pi u2), Omega[2m+1, j] = sqrt(-2 ln u1) sin(2 pi u2).
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 on uint32 arrays; returns four uint32 arrays."""
    c = [np.asarray(v, dtype=np.uint64) & _MASK for v in (c0, c1, c2, c3)]
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + np.uint64(W0)) & _MASK
            k1 = (k1 + np.uint64(W1)) & _MASK
        p0 = np.uint64(M0) * c[0]
        p1 = np.uint64(M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return [v.astype(np.uint32) for v in c]


def _u53(a, b):
    a = a.astype(np.uint64) >> np.uint64(5)
    b = b.astype(np.uint64) >> np.uint64(6)
    return ((a * np.uint64(67108864) + b).astype(np.float64) + 0.5) * 2.0 ** -53


def gaussian_omega(n_params: int, ell: int, seed: int, counter: int = 0) -> np.ndarray:
    """p x ell standard normal test matrix generated from (seed, counter)."""
    m = np.arange((n_params + 1) // 2, dtype=np.uint64)
    out = np.empty((2 * len(m), ell))
    for j in range(ell):
        x0, x1, x2, x3 = philox4x32_10(m, np.full_like(m, j), np.full_like(m, counter & 0xFFFFFFFF),
                                       np.full_like(m, (counter >> 32) & 0xFFFFFFFF),
                                       seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
        u1, u2 = _u53(x0, x1), _u53(x2, x3)
        rad = np.sqrt(-2.0 * np.log(u1))
        out[0::2, j] = rad * np.cos(2.0 * np.pi * u2)
        out[1::2, j] = rad * np.sin(2.0 * np.pi * u2)
    return out[:n_params]
