"""Gaussian test matrices (the ``randn`` of Fig. 2 and Fig. 4).

The paper only asks for i.i.d. standard normal entries (Sec. 2.5).  To let
two independent implementations draw *identical* test matrices, the stream is
defined by global coordinates rather than by call order:

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC'11): 10 rounds of the 4x32 Philox S-box with multipliers
  0xD2511F53 / 0xCD9E8D57 and Weyl key increments 0x9E3779B9 / 0xBB67AE85.
* counter ``(row i, column pair j>>1, level, phase)``, key ``(seed mod 2^32,
  seed >> 32)``.  Phase 0: the level's Gaussian block G_l (N x r); phase 1:
  probe vectors of the error estimate E.
* two 53-bit uniforms from the four output words, ``u1 = (m1+1) 2^-53`` in
  (0,1], ``u2 = m2 2^-53`` in [0,1), and Box-Muller: even columns take
  ``sqrt(-2 ln u1) cos(2 pi u2)``, odd columns the ``sin`` branch.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 on arrays of 32-bit words held in uint64; returns the
    four output words."""
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK
    c2 = np.asarray(c2, dtype=np.uint64) & _MASK
    c3 = np.asarray(c3, dtype=np.uint64) & _MASK
    k0 = np.uint64(k0 & _MASK)
    k1 = np.uint64(k1 & _MASK)
    m0, m1 = np.uint64(M0), np.uint64(M1)
    for _ in range(10):
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(_MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(_MASK)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = np.uint64((int(k0) + W0) & _MASK)
        k1 = np.uint64((int(k1) + W1) & _MASK)
    return c0, c1, c2, c3


def gaussian_block(seed: int, level: int, rows: np.ndarray, ncols: int,
                   phase: int = 0) -> np.ndarray:
    """Entries ``G(i, j)`` of the stream for the given global rows i and
    columns j = 0..ncols-1, float64 array (len(rows), ncols)."""
    rows = np.asarray(rows, dtype=np.uint64)
    i = np.repeat(rows[:, None], ncols, axis=1)
    j = np.repeat(np.arange(ncols, dtype=np.uint64)[None, :], len(rows), axis=0)
    w0, w1, w2, w3 = philox4x32_10(i, j >> np.uint64(1), np.uint64(level),
                                   np.uint64(phase), seed & _MASK,
                                   (seed >> 32) & _MASK)
    m1 = (w0 >> np.uint64(5)) * np.uint64(67108864) + (w1 >> np.uint64(6))
    m2 = (w2 >> np.uint64(5)) * np.uint64(67108864) + (w3 >> np.uint64(6))
    u1 = (m1.astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = m2.astype(np.float64) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    odd = (j & np.uint64(1)).astype(bool)
    return np.where(odd, rad * np.sin(ang), rad * np.cos(ang))


def level_gaussian(seed: int, level: int, n: int, r: int) -> np.ndarray:
    """The level's Gaussian block G_l, N x r.  Fig. 2/4 draw ``randn(n_a, r)``
    for each left child a and ``randn(n_b, r)`` for each right child b; here
    both are the rows I_a / I_b of this one block, which is equally i.i.d."""
    return gaussian_block(seed, level, np.arange(n), r, phase=0)


def probe_vectors(seed: int, n: int, count: int = 10) -> np.ndarray:
    """Unit vectors uniform on the sphere (normalised Gaussians), N x count,
    for the error estimate E of Sec. 5."""
    g = gaussian_block(seed, 0, np.arange(n), count, phase=1)
    return g / np.linalg.norm(g, axis=0, keepdims=True)
