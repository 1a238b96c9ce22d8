"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module only *creates inputs*: point sets, generator factors of synthetic
rank-structured operators, right-hand sides.  It contains none of the
compression method's arithmetic (no sampling, no peeling, no factorisation of
samples, no apply of a compressed form), so both the CPU oracle and the HIP
path can take its outputs without sharing any code of the method itself.

All randomness here comes from ``numpy.random.default_rng(seed)`` (PCG64);
the Gaussian test matrices that the method itself draws are *not* made here:
each side implements the counter-based generator on its own.

Workload recipes (sizes and laws are those of the configurations the build is
measured on; the paper's own geometries exist only as figures, so these
synthetic stand-ins replace them):

* ellipse points (log kernel, HODLR test case): ``x_i = (cos t_i, 0.5 sin t_i)``,
  ``t_i = 2 pi i / N``.
* random-Fourier closed curve (near-singular kernel, mixed-precision case):
  ``rho(t) = 1 + 0.2 s(t) / max_i |s(t_i)|``, ``s = sum_{m=1..8} a_m cos mt +
  b_m sin mt``, ``a, b ~ N(0,1)``; ``x_i = rho(t_i) (cos t_i, sin t_i)``.
* synthetic HODLR of exact off-diagonal rank k: every sibling block is
  ``P Q^T`` with Gaussian ``P, Q`` of k columns; diagonal leaf blocks Gaussian.
* synthetic HBS of exact rank k with nested bases: Haar-random orthonormal
  leaf bases (n_leaf x k) and transfer matrices (2k x k), sibling blocks
  ``N(0,1) * 2**-level``, leaf diagonal blocks ``N(0,1) + 8 I``.
* batched instances: ``N_i = 64 * round(exp(U[ln 512, ln 8192]) / 64)``,
  ``k_i ~ U{8..40}``.
* conduction grid of nested dissection (Sec. 5.4, geometry of Fig. 13): a grid of
  ``height`` rows and ``width`` (= 41) columns of nodes; every bar between two
  neighbouring nodes has a conductivity drawn from U[1, 2].  Horizontal bars
  ``ch[i, j]`` join nodes (i, j) and (i, j+1); vertical bars ``cv[i, j]`` join
  (i, j) and (i+1, j).  Only the conductivities are made here; the matrix
  they define is each consumer's own.

The synthetic operators are *defined* on the uniform binary partition of
``[0, N)``: depth ``L = ceil(log2(N / leaf))`` (0 if ``N <= leaf``), every
interval split so that its left half holds ``ceil(n/2)`` indices.  That
partition is part of the operator's definition here (which blocks are low
rank), so it is spelled out below; both consumers build their own trees.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "operator_partition",
    "ellipse_points",
    "fourier_curve_points",
    "synthetic_hodlr_dense",
    "synthetic_hbs",
    "batched_instances",
    "gaussian",
]


def operator_partition(n: int, leaf: int):
    """Intervals of the uniform binary partition that defines the synthetic
    operators: returns ``(L, lo, hi)`` with heap numbering (root 1, children
    2t and 2t+1) and ``lo, hi`` int64 arrays of length ``2**(L+1)``."""
    if n < 1 or leaf < 1:
        raise ValueError("n and leaf must be positive")
    L = 0 if n <= leaf else int(math.ceil(math.log2(n / leaf)))
    size = 2 ** (L + 1)
    lo = np.zeros(size, dtype=np.int64)
    hi = np.zeros(size, dtype=np.int64)
    lo[1], hi[1] = 0, n
    for t in range(1, 2 ** L):
        a, b = int(lo[t]), int(hi[t])
        mid = a + (b - a + 1) // 2
        lo[2 * t], hi[2 * t] = a, mid
        lo[2 * t + 1], hi[2 * t + 1] = mid, b
    return L, lo, hi


def ellipse_points(n: int, a: float = 1.0, b: float = 0.5) -> np.ndarray:
    """``n`` points equispaced in angle on the ellipse with semi-axes a, b; (n, 2)."""
    t = 2.0 * np.pi * np.arange(n, dtype=np.float64) / n
    return np.stack([a * np.cos(t), b * np.sin(t)], axis=1)


def fourier_curve_points(n: int, modes: int = 8, amplitude: float = 0.2,
                         seed: int = 3) -> np.ndarray:
    """``n`` points on a smooth star-shaped closed curve with a random Fourier
    radius (see module docstring); (n, 2) float64, ordered along the curve."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(modes)
    b = rng.standard_normal(modes)
    t = 2.0 * np.pi * np.arange(n, dtype=np.float64) / n
    m = np.arange(1, modes + 1, dtype=np.float64)
    s = np.cos(np.outer(t, m)) @ a + np.sin(np.outer(t, m)) @ b
    rho = 1.0 + amplitude * s / np.max(np.abs(s))
    return np.stack([rho * np.cos(t), rho * np.sin(t)], axis=1)


def _haar(rng, n: int, k: int) -> np.ndarray:
    """Haar-distributed n x k matrix with orthonormal columns (QR of a Gaussian
    with the signs of diag(R) folded in)."""
    g = rng.standard_normal((n, k))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def synthetic_hodlr_dense(n: int, leaf: int, k: int, seed: int = 0) -> np.ndarray:
    """Dense n x n matrix whose every sibling block ``A(I_a, I_b)`` equals
    ``P Q^T`` with Gaussian P (n_a x k), Q (n_b x k); leaf diagonal blocks
    Gaussian.  Off-diagonal rank is exactly ``min(k, n_a, n_b)``."""
    L, lo, hi = operator_partition(n, leaf)
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n))
    for t in range(1, 2 ** L):
        a, b = 2 * t, 2 * t + 1
        for (x, y) in ((a, b), (b, a)):
            P = rng.standard_normal((hi[x] - lo[x], k))
            Q = rng.standard_normal((hi[y] - lo[y], k))
            A[lo[x]:hi[x], lo[y]:hi[y]] = P @ Q.T
    for t in range(2 ** L, 2 ** (L + 1)):
        m = hi[t] - lo[t]
        A[lo[t]:hi[t], lo[t]:hi[t]] = rng.standard_normal((m, m))
    return A


def synthetic_hbs(n: int, leaf: int, k: int, seed: int = 1,
                  dtype=np.float64) -> dict:
    """Generators of a synthetic HBS matrix of uniform rank k with nested
    orthonormal bases, in the flat layout both consumers read:

    * ``U``, ``V``: (n, k).  Rows ``I_t`` of a leaf t hold its basis.
    * ``Ut``, ``Vt``: (2**(L+1), 2k, k) transfer matrices of non-root,
      non-leaf nodes (zero elsewhere); rows 0..k-1 couple to the left child.
    * ``B``: (2**(L+1), k, k); ``B[v]`` is the sibling matrix of the ordered
      pair (sibling(v), v): ``A(I_sib(v), I_v) = Ulong_sib B[v] Vlong_v^T``.
      Entries ``N(0,1) * 2**-level(v)``.
    * ``D``: (n, nmax); rows ``I_t`` of a leaf t hold ``D_t`` in columns
      ``0..n_t-1`` (``N(0,1) + 8 I``), zero-padded to ``nmax`` columns.
    """
    L, lo, hi = operator_partition(n, leaf)
    rng = np.random.default_rng(seed)
    nn = 2 ** (L + 1)
    leaves = range(2 ** L, nn)
    nmax = int(max(hi[t] - lo[t] for t in leaves))
    if min(hi[t] - lo[t] for t in leaves) < k and L > 0:
        raise ValueError("every leaf must hold at least k indices")
    U = np.zeros((n, k))
    V = np.zeros((n, k))
    for t in leaves:
        m = hi[t] - lo[t]
        if L > 0:
            U[lo[t]:hi[t]] = _haar(rng, m, k)
            V[lo[t]:hi[t]] = _haar(rng, m, k)
    Ut = np.zeros((nn, 2 * k, k))
    Vt = np.zeros((nn, 2 * k, k))
    for t in range(2, 2 ** L):
        Ut[t] = _haar(rng, 2 * k, k)
        Vt[t] = _haar(rng, 2 * k, k)
    B = np.zeros((nn, k, k))
    for t in range(2, nn):
        lev = int(math.floor(math.log2(t)))
        B[t] = rng.standard_normal((k, k)) * 2.0 ** (-lev)
    D = np.zeros((n, nmax))
    for t in leaves:
        m = hi[t] - lo[t]
        D[lo[t]:hi[t], :m] = rng.standard_normal((m, m)) + 8.0 * np.eye(m)
    cast = lambda a: np.ascontiguousarray(a, dtype=dtype)
    return dict(n=n, leaf=leaf, k=k, L=L, U=cast(U), V=cast(V), Ut=cast(Ut),
                Vt=cast(Vt), B=cast(B), D=cast(D))


def batched_instances(count: int = 256, seed: int = 2, nmin: int = 512,
                      nmax: int = 8192, kmin: int = 8, kmax: int = 40):
    """Sizes of the uneven batch: list of ``(N_i, k_i)``."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        x = math.exp(rng.uniform(math.log(nmin), math.log(nmax)))
        n = max(64, 64 * int(round(x / 64.0)))
        kk = int(rng.integers(kmin, kmax + 1))
        out.append((n, kk))
    return out


def gaussian(shape, seed: int, dtype=np.float64) -> np.ndarray:
    """Gaussian array from PCG64(seed) (right-hand sides, upstream gradients)."""
    rng = np.random.default_rng(seed)
    return np.asarray(rng.standard_normal(shape), dtype=dtype)


def grid_conductivities(height: int, width: int = 41, seed: int = 7):
    """Bar conductivities of the ``height`` x ``width`` conduction grid, drawn
    from U[1, 2] with PCG64(seed): ``ch`` is ``height x (width - 1)``
    (horizontal bars), ``cv`` is ``(height - 1) x width`` (vertical bars),
    both C-ordered FP64 (``ch[i, j]`` joins nodes (i, j) and (i, j + 1),
    ``cv[i, j]`` joins (i, j) and (i + 1, j))."""
    if height < 1 or width < 3 or width % 2 == 0:
        raise ValueError("height >= 1 and an odd width >= 3")
    rng = np.random.default_rng(seed)
    ch = rng.uniform(1.0, 2.0, size=(height, width - 1))
    cv = rng.uniform(1.0, 2.0, size=(max(height - 1, 0), width))
    return np.ascontiguousarray(ch), np.ascontiguousarray(cv)
