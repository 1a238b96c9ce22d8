"""Frontal matrix of nested dissection (Sec. 5.4, Fig. 13 and the equation
defining A there).

The conduction grid has ``H`` rows and ``W`` (odd, 41 in the paper) columns of
nodes; node (i, j) has index ``i * W + j``.  Every bar between neighbouring
nodes carries a conductivity (``ch`` horizontal, ``cv`` vertical, see
``workloads.grid_conductivities``).  ``B`` is the matrix of the network: the
weighted graph Laplacian, with the sum of the conductivities of the bars at a
node on the diagonal and minus the bar's conductivity between neighbours.
The index sets (Fig. 13): ``I3`` is the middle column ``j = (W - 1) / 2``
ordered by row, ``I1`` the columns left of it and ``I2`` those right of it.
Then

    A = B33 - B31 B11^{-1} B13 - B32 B22^{-1} B23          (H x H)

with ``Bij = B(Ii, Ij)``.  ``B12`` is zero (no bar crosses the middle column),
and ``B11``, ``B22`` are nonsingular: each is a principal block of the
Laplacian of a connected network that keeps a bar to a node outside it.

The products with A use a sparse LU factorisation of B11 and B22 (SciPy's
SuperLU) as the library primitive that applies their inverses; the paper's
experiments apply them the same way, with a sparse direct solver.  A is
symmetric, so the adjoint product is the same product.

This module is test infrastructure: only the tests, the smoke check and the
benchmark's CPU baseline use it.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def laplacian(ch: np.ndarray, cv: np.ndarray) -> sp.csr_matrix:
    """The network matrix B of the grid (graph Laplacian, bars as edges)."""
    H, Wm1 = ch.shape
    W = Wm1 + 1
    rows, cols, vals = [], [], []

    def bar(p, q, c):
        # a bar of conductivity c between nodes p and q adds c to both
        # diagonal entries and -c to the two coupling entries
        rows.extend([p, q, p, q])
        cols.extend([p, q, q, p])
        vals.extend([c, c, -c, -c])

    for i in range(H):
        for j in range(W - 1):
            bar(i * W + j, i * W + j + 1, ch[i, j])
    for i in range(H - 1):
        for j in range(W):
            bar(i * W + j, (i + 1) * W + j, cv[i, j])
    n = H * W
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def index_sets(H: int, W: int):
    """I1 (left of the middle column), I2 (right of it), I3 (the middle
    column, by row), as node indices."""
    mid = (W - 1) // 2
    grid = np.arange(H * W).reshape(H, W)
    return grid[:, :mid].ravel(), grid[:, mid + 1:].ravel(), grid[:, mid].copy()


class FrontalOp:
    """The black box x -> A x of Sec. 5.4 on N x c blocks (N = H)."""

    def __init__(self, ch: np.ndarray, cv: np.ndarray):
        self.ch = np.asarray(ch, dtype=np.float64)
        self.cv = np.asarray(cv, dtype=np.float64)
        H, Wm1 = self.ch.shape
        self.H, self.W = H, Wm1 + 1
        self.n = H
        B = laplacian(self.ch, self.cv).tocsc()
        I1, I2, I3 = index_sets(self.H, self.W)
        blk = lambda r, c: B[r][:, c].tocsc()
        self.B11, self.B13 = blk(I1, I1), blk(I1, I3)
        self.B22, self.B23 = blk(I2, I2), blk(I2, I3)
        self.B31, self.B32, self.B33 = blk(I3, I1), blk(I3, I2), blk(I3, I3)
        self.lu1 = spla.splu(self.B11)
        self.lu2 = spla.splu(self.B22)

    def apply(self, X):
        X = np.asarray(X, dtype=np.float64)
        vec = X.ndim == 1
        X2 = X.reshape(self.n, -1)
        Y = (self.B33 @ X2
             - self.B31 @ self.lu1.solve(np.asarray(self.B13 @ X2))
             - self.B32 @ self.lu2.solve(np.asarray(self.B23 @ X2)))
        Y = np.asarray(Y)
        return Y.ravel() if vec else Y

    def apply_adjoint(self, X):
        return self.apply(X)

    def dense(self) -> np.ndarray:
        return self.apply(np.eye(self.n))

    def entries(self, rows, cols):
        E = np.zeros((self.n, len(cols)))
        E[np.asarray(cols), np.arange(len(cols))] = 1.0
        return self.apply(E)[np.asarray(rows)]
