"""Black-box operators ``x -> A x`` and ``x -> A^* x`` on N x c blocks
(Sec. 1: the method touches A only through such products).

* ``DenseOp``  -- an explicit matrix.
* ``KernelOp`` -- a kernel matrix ``A(i,j) = K(x_i, x_j)`` on 2-D points,
  evaluated tile by tile (never stored whole):
  ``"log"``: ``log|x_i - x_j|`` off the diagonal, 1 on it;
  ``"near"``: ``1 / (|x_i - x_j| + delta)`` everywhere (delta = 1e-3 default).
* ``HBSOp``    -- a matrix given in HBS form, applied in O(N k) (Fig. 7 + D).
* ``ProductOp`` -- the product ``A1 A2`` of two black boxes (Sec. 5.2,
  operator multiplication: a product of compressed operators, recompressed
  from products with vectors alone).
* ``PerturbedOp`` -- another operator whose every output entry is multiplied
  by ``1 + d`` with ``d`` uniform in ``[-rel, rel]``: the products a sampler
  with rounding error of that size could return.  Running the compression
  with it measures how far rounding of the samples alone moves the result
  (the method's own sensitivity), which is the yardstick for comparing two
  correct implementations whose products round differently.

This module is test infrastructure: only the tests, the smoke check and the
benchmark's CPU baseline use it.
"""
from __future__ import annotations

import concurrent.futures as cf

import numpy as np


class DenseOp:
    def __init__(self, A: np.ndarray):
        self.A = np.asarray(A, dtype=np.float64)
        self.n = self.A.shape[0]

    def apply(self, X):
        return self.A @ X

    def apply_adjoint(self, X):
        return self.A.T @ X

    def entries(self, rows, cols):
        return self.A[np.ix_(rows, cols)]


class KernelOp:
    def __init__(self, points: np.ndarray, kind: str = "near", delta: float = 1e-3,
                 tile: int = 512, workers: int = 1):
        self.p = np.asarray(points, dtype=np.float64)
        self.n = self.p.shape[0]
        if kind not in ("log", "near"):
            raise ValueError(kind)
        self.kind = kind
        self.delta = delta
        self.tile = tile
        # row tiles are independent, so several threads may evaluate them
        # (NumPy releases the interpreter lock inside its array operations);
        # each tile's arithmetic is the same whatever the thread count
        self.workers = max(1, int(workers))

    def entries(self, rows, cols):
        rows = np.asarray(rows)
        cols = np.asarray(cols)
        dx = self.p[rows, 0][:, None] - self.p[cols, 0][None, :]
        dy = self.p[rows, 1][:, None] - self.p[cols, 1][None, :]
        d = np.sqrt(dx * dx + dy * dy)
        if self.kind == "near":
            return 1.0 / (d + self.delta)
        same = rows[:, None] == cols[None, :]
        with np.errstate(divide="ignore"):
            v = np.log(np.where(same, 1.0, d))
        return np.where(same, 1.0, v)

    def apply(self, X):
        X = np.asarray(X, dtype=np.float64)
        vec = X.ndim == 1
        if vec:
            X = X[:, None]
        Y = np.zeros((self.n, X.shape[1]))
        cols = np.arange(self.n)

        def tile(i0):
            rows = np.arange(i0, min(i0 + self.tile, self.n))
            Y[rows] = self.entries(rows, cols) @ X

        starts = range(0, self.n, self.tile)
        if self.workers == 1:
            for i0 in starts:
                tile(i0)
        else:
            with cf.ThreadPoolExecutor(self.workers) as ex:
                list(ex.map(tile, starts))
        return Y[:, 0] if vec else Y

    apply_adjoint = apply          # both kernels are symmetric

    def dense(self):
        idx = np.arange(self.n)
        return self.entries(idx, idx)


class HBSOp:
    def __init__(self, h):
        self.h = h
        self.n = h.tree.n

    def apply(self, X):
        return self.h.apply(X)

    def apply_adjoint(self, X):
        return self.h.apply_adjoint(X)


class ProductOp:
    """``x -> A1 (A2 x)`` and ``x -> A2^* (A1^* x)``."""

    def __init__(self, op1, op2):
        if op1.n != op2.n:
            raise ValueError("factor sizes differ")
        self.op1, self.op2 = op1, op2
        self.n = op1.n

    def apply(self, X):
        return self.op1.apply(self.op2.apply(X))

    def apply_adjoint(self, X):
        return self.op2.apply_adjoint(self.op1.apply_adjoint(X))


class PerturbedOp:
    """``op`` with relative noise on its products: every entry of ``A X``
    (and of ``A^* X``) is multiplied by ``1 + d``, ``d ~ U[-rel, rel]``
    independently, from ``numpy.random.default_rng(seed)``.  ``rel`` =
    2**-52 is one unit in the last place of FP64."""

    def __init__(self, op, rel: float, seed: int):
        self.op = op
        self.n = op.n
        self.rel = float(rel)
        self.gen = np.random.default_rng(seed)

    def _noisy(self, Y):
        return Y * (1.0 + self.gen.uniform(-self.rel, self.rel, size=Y.shape))

    def apply(self, X):
        return self._noisy(self.op.apply(X))

    def apply_adjoint(self, X):
        return self._noisy(self.op.apply_adjoint(X))

    def entries(self, rows, cols):
        return self.op.entries(rows, cols)
