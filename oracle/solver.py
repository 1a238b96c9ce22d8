"""Test infrastructure (not the product): the fast direct solver of an HBS
matrix, the consumer the paper names for the compressed form (Sec. 1, the
compressed operator is inverted by fast direct solvers it cites).

The paper cites these solvers and does not state one.  Written here from the
published method of Gillman, Young and Martinsson (2012) for HBS matrices of
uniform rank k, which telescopes the Sherman-Morrison-Woodbury formula over
the tree.  At one level A = D + U A~ V^* (D block diagonal, U and V the node
bases, A~ the couplings of the coarser levels).  Per node,

    Dh = (V^* D^-1 U)^-1,  E = D^-1 U Dh,  F = D^-* V Dh^*,
    G  = D^-1 - D^-1 U Dh V^* D^-1,

and then A^-1 = E (Dh + A~)^-1 F^* + G.  Dh + A~ is again HBS one level up:
the block of a parent t with children a, b is [Dh_a  B_ab; B_ba  Dh_b], and
its bases are t's transfer matrices.  At the root that block is inverted
outright.  The solve takes b^_t = F_t^* b_t up the tree and
x_t = E_t x^_t + G_t b_t back down it (for a parent, "x_t" and "b_t" are the
stacked children's expansions).

Each block inverse is LAPACK's (``numpy.linalg.inv``).  The plain definition
``x = A_H^-1 b`` is :func:`oracle.hbs.solve`; the tests pin this solver to
it, and the residual of this solver is what the GPU solver's error bounds are
calibrated on.  The formulas need no pivoting across levels, so the error
grows with the conditioning of the D blocks and of V^* D^-1 U, not only with
cond(A).
"""
from __future__ import annotations

import numpy as np

from .hbs import HBS


class Factor:
    """The per-node E, F, G of every non-root node and the inverse of the
    root's block, for an HBS of uniform rank k."""

    def __init__(self, h: HBS):
        t_ = h.tree
        if t_.L < 1:
            raise ValueError("a tree without levels: invert D directly")
        ks = {h.rank_u(t) for t in range(2, 2 ** (t_.L + 1))} | \
            {h.rank_v(t) for t in range(2, 2 ** (t_.L + 1))}
        if len(ks) != 1:
            raise ValueError("node ranks must all be equal")
        self.h, self.k = h, ks.pop()
        self.E, self.F, self.G, Dh = {}, {}, {}, {}
        inv = np.linalg.inv

        def node(t, D, U, V):
            Di = inv(D)
            Dh[t] = inv(V.T @ Di @ U)
            self.E[t] = Di @ U @ Dh[t]
            self.F[t] = Di.T @ V @ Dh[t].T
            self.G[t] = Di - Di @ U @ Dh[t] @ V.T @ Di

        def block(t):
            a, b = 2 * t, 2 * t + 1
            return np.block([[Dh[a], h.B[(a, b)]], [h.B[(b, a)], Dh[b]]])

        for t in t_.leaves():
            node(t, h.D[t], h.U[t], h.V[t])
        for lev in range(t_.L - 1, 0, -1):
            for t in t_.level_nodes(lev):
                node(t, block(t), h.Ut[t], h.Vt[t])
        self.Groot = inv(block(1))

    def solve(self, b: np.ndarray) -> np.ndarray:
        t_, k = self.h.tree, self.k
        b = np.asarray(b, dtype=np.float64)
        bh, xh = {}, {}
        # upward: b^_t = F_t^* b_t (a parent's b_t stacks its children's b^)
        for t in t_.leaves():
            bh[t] = self.F[t].T @ b[t_.I(t)]
        stack = lambda d, t: np.vstack([d[2 * t], d[2 * t + 1]])
        for lev in range(t_.L - 1, 0, -1):
            for t in t_.level_nodes(lev):
                bh[t] = self.F[t].T @ stack(bh, t)
        # root, then downward: children's x^ = E_t x^_t + G_t b_t
        z = self.Groot @ stack(bh, 1)
        xh[2], xh[3] = z[:k], z[k:]
        for lev in range(1, t_.L):
            for t in t_.level_nodes(lev):
                z = self.E[t] @ xh[t] + self.G[t] @ stack(bh, t)
                xh[2 * t], xh[2 * t + 1] = z[:k], z[k:]
        x = np.zeros_like(b)
        for t in t_.leaves():
            x[t_.I(t)] = self.E[t] @ xh[t] + self.G[t] @ b[t_.I(t)]
        return x
