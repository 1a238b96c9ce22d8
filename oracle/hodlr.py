"""HODLR matrices and their randomized compression (Sec. 2.8, Sec. 3, Fig. 2).

Representation: every ordered sibling pair (a, b) on levels 1..L stores
``A(I_a, I_b) = U[a] B[(a,b)] V[b]^*`` with orthonormal long bases U[a]
(n_a x k) and V[b]; leaves store ``D[t]``.  (Sec. 2.8 prints the
factorisation as ``U_a A~_ab U_b`` and calls ``U_a`` and ``B_b``
orthonormal; read as ``U_a B_ab V_b^*`` with U and V orthonormal.)

``A^(l)`` keeps the sibling blocks of levels 1..l and zeroes everything
finer (Sec. 2.8); its apply costs O(l k N) (eq. dev2).

Fig. 2 uses the SVD variant (eq. SVDtogetV / SVDtogetB), so every B is
diagonal; Fig. 2 names the third SVD output of the second call
``V^_a`` and then uses ``U^_a`` -- read as ``U^_a``.
"""
from __future__ import annotations

import numpy as np

from . import lowrank, rng
from .hbs import CompressStats, _sample
from .tree import Tree


class HODLR:
    def __init__(self, tree: Tree):
        self.tree = tree
        self.U, self.V = {}, {}      # node -> long basis, nodes on levels 1..L
        self.B = {}                  # (a, b) -> B_ab (diagonal for Fig. 2)
        self.D = {}

    def apply_truncated(self, m: int, x: np.ndarray, adjoint: bool = False):
        """``A^(m) x`` (or its adjoint)."""
        tree = self.tree
        x = np.asarray(x, dtype=np.float64)
        vec = x.ndim == 1
        if vec:
            x = x[:, None]
        y = np.zeros_like(x)
        for lev in range(1, m + 1):
            for t in tree.level_nodes(lev - 1):
                a, b = tree.children(t)
                for (p, q) in ((a, b), (b, a)):
                    if adjoint:   # (A^*)_qp = V_q B_pq^* U_p^*
                        y[tree.I(q)] += self.V[q] @ (self.B[(p, q)].T @ (self.U[p].T @ x[tree.I(p)]))
                    else:
                        y[tree.I(p)] += self.U[p] @ (self.B[(p, q)] @ (self.V[q].T @ x[tree.I(q)]))
        return y[:, 0] if vec else y

    def apply(self, x, adjoint: bool = False):
        tree = self.tree
        x = np.asarray(x, dtype=np.float64)
        vec = x.ndim == 1
        if vec:
            x = x[:, None]
        y = self.apply_truncated(tree.L, x, adjoint)
        for t in tree.leaves():
            D = self.D[t].T if adjoint else self.D[t]
            y[tree.I(t)] += D @ x[tree.I(t)]
        return y[:, 0] if vec else y

    def apply_adjoint(self, x):
        return self.apply(x, adjoint=True)

    def dense(self):
        return self.apply(np.eye(self.tree.n))

    def storage_reals(self) -> int:
        tot = 0
        for d in (self.U, self.V, self.D):
            tot += sum(x.size for x in d.values())
        tot += sum(np.count_nonzero(np.diag(b)) if b.ndim == 2 else b.size
                   for b in self.B.values())
        return tot

    def ranks(self):
        return {key: b.shape[0] for key, b in self.B.items()}


def compress(op, n: int, leaf: int, r: int, seed: int, rank: int | None = None,
             tol: float | None = None):
    """Fig. 2.  ``r`` samples per level; the SVD of each Z block is truncated
    at ``tol`` (relative, per block) or to ``rank``."""
    tree = Tree(n, leaf)
    L = tree.L
    h = HODLR(tree)
    stats = CompressStats()
    for lev in range(L):
        # Build the random matrices Omega_1 and Omega_2.
        G = rng.level_gaussian(seed, lev, n, r)
        Om1 = np.zeros((n, r))
        Om2 = np.zeros((n, r))
        for t in tree.level_nodes(lev):
            a, b = tree.children(t)
            Om1[tree.I(a)] = G[tree.I(a)]
            Om2[tree.I(b)] = G[tree.I(b)]
        # Samples for the incoming bases.
        Y1 = _sample(op, Om2, False, stats) - h.apply_truncated(lev, Om2)
        Y2 = _sample(op, Om1, False, stats) - h.apply_truncated(lev, Om1)
        # Orthonormalise.
        U = {}
        for t in tree.level_nodes(lev):
            a, b = tree.children(t)
            U[a] = lowrank.qr(Y1[tree.I(a)])
            U[b] = lowrank.qr(Y2[tree.I(b)])
            Om1[tree.I(a)] = 0.0
            Om2[tree.I(b)] = 0.0
            Om1[tree.I(a), :U[a].shape[1]] = U[a]
            Om2[tree.I(b), :U[b].shape[1]] = U[b]
        # Samples for the outgoing bases.
        Z1 = _sample(op, Om2, True, stats) - h.apply_truncated(lev, Om2, adjoint=True)
        Z2 = _sample(op, Om1, True, stats) - h.apply_truncated(lev, Om1, adjoint=True)
        # Local SVDs: outgoing bases, diagonal sibling matrices, rank update.
        for t in tree.level_nodes(lev):
            a, b = tree.children(t)
            Va, s21, Uhb = lowrank.svd(Z1[tree.I(a), :U[b].shape[1]], k=rank, eps=tol)
            Vb, s12, Uha = lowrank.svd(Z2[tree.I(b), :U[a].shape[1]], k=rank, eps=tol)
            h.V[a], h.V[b] = Va, Vb
            h.B[(b, a)] = np.diag(s21)
            h.B[(a, b)] = np.diag(s12)
            h.U[b] = U[b] @ Uhb
            h.U[a] = U[a] @ Uha
    # Extract the diagonal matrices.
    nmax = tree.nmax()
    Om = np.zeros((n, nmax))
    for t in tree.leaves():
        Om[tree.I(t), :tree.size(t)] = np.eye(tree.size(t))
    Yd = _sample(op, Om, False, stats) - h.apply_truncated(L, Om)
    for t in tree.leaves():
        h.D[t] = Yd[tree.I(t), :tree.size(t)].copy()
    return h, stats
