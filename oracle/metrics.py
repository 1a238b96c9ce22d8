"""Error measures.

* ``estimate_E`` -- the randomized error estimate of Sec. 5: the largest of
  ``||A w_i - A_c w_i|| / ||A w_i||`` over ten unit vectors ``w_i`` drawn
  uniformly on the sphere (normalised Gaussians from phase 1 of the counter
  stream; the paper says "uniform on the unit sphere").
* ``rel_fro`` -- ``||X - Y||_F / ||Y||_F`` of dense matrices.
"""
from __future__ import annotations

import numpy as np

from . import rng


def estimate_E(apply_exact, apply_comp, n: int, seed: int = 12345,
               count: int = 10) -> float:
    W = rng.probe_vectors(seed, n, count)
    Ya = apply_exact(W)
    Yc = apply_comp(W)
    num = np.linalg.norm(Ya - Yc, axis=0)
    den = np.linalg.norm(Ya, axis=0)
    return float(np.max(num / den))


def rel_fro(X: np.ndarray, Y: np.ndarray) -> float:
    return float(np.linalg.norm(X - Y) / np.linalg.norm(Y))

