"""HBS (= HSS) matrices: representation, the apply of Fig. 7, the
storage-efficient compression of Fig. 4 and the HBS-ID conversion of Fig. 5.

Representation (Sec. 2.9, eq. babytelescope, Def. 2.2): a leaf t stores long
bases ``U[t]`` (n_t x k_t) and ``V[t]``; a non-root, non-leaf node t stores
short transfers ``Ut[t]``, ``Vt[t]`` of size (k_a + k_b) x k_t with
``Ulong_t = diag(Ulong_a, Ulong_b) Ut[t]``; every ordered sibling pair stores
``B[(a, b)]`` (k_a x k_b) with ``A(I_a, I_b) = Ulong_a B[(a,b)] Vlong_b^*``;
leaves store ``D[t] = A(I_t, I_t)``.  Ranks may differ per node.

Readings of the paper taken here (each is pinned by a test):

* Fig. 3/4 write ``B_ab = X_1(1:r,:) diag(b_12)``.  From the SVD
  ``Z_1^loc = V_a diag(b_21) X_1^*`` and ``Z_1(I_a,:) = A_ba^* U_b`` one gets
  ``A_ba = U_b X_1(1:r,:) diag(b_21) V_a^*``: the block built from ``X_1`` is
  ``B_ba`` and carries ``b_21``; symmetrically ``B_ab = X_2(1:r,:) diag(b_12)``.
  (Exact recovery of exact-rank operators fails with the printed pairing.)
* Fig. 7 runs its downward pass over ``l = (m-1):(-1):1``; incoming
  expansions must flow from coarse to fine, so the pass here runs over
  levels ``1 .. m-1``.  ``U_t(J_a, :)`` there is the block of rows of the
  *short* transfer ``Ut[t]`` that couples to child a.
"""
from __future__ import annotations

import numpy as np

from . import lowrank, metrics, rng
from .tree import Tree


class HBS:
    def __init__(self, tree: Tree):
        self.tree = tree
        self.U, self.V = {}, {}          # leaf long bases
        self.Ut, self.Vt = {}, {}        # short transfers (non-root, non-leaf)
        self.B = {}                      # (a, b) -> B_ab
        self.D = {}                      # leaf diagonal blocks
        self.skel_in, self.skel_out = {}, {}   # HBS-ID skeletons (global rows)
        # pivot margins of each node's ID (lowrank.cpqr), for comparing
        # skeletons with another implementation
        self.gaps_in, self.gaps_out = {}, {}
        self.is_id = False

    # ranks ------------------------------------------------------------------
    def rank_u(self, t):
        return (self.U[t] if t in self.U else self.Ut[t]).shape[1]

    def rank_v(self, t):
        return (self.V[t] if t in self.V else self.Vt[t]).shape[1]

    def storage_reals(self) -> int:
        tot = 0
        for d in (self.U, self.V, self.Ut, self.Vt, self.B, self.D):
            tot += sum(x.size for x in d.values())
        return tot

    # apply -------------------------------------------------------------------
    def apply(self, x: np.ndarray) -> np.ndarray:
        """``A x`` for the represented matrix (Fig. 7 with m = L, plus D)."""
        return apply_hbs(self, x, adjoint=False)

    def apply_adjoint(self, x: np.ndarray) -> np.ndarray:
        return apply_hbs(self, x, adjoint=True)

    def dense(self) -> np.ndarray:
        return self.apply(np.eye(self.tree.n))


def apply_partial(tree: Tree, m: int, Ulong: dict, Vlong: dict, Ut: dict,
                  Vt: dict, B: dict, q: np.ndarray,
                  downward: str = "coarse-to-fine") -> np.ndarray:
    """``u = A^(m) q`` by Fig. 7: outgoing expansions from the long bases
    ``Vlong`` on level m, upward pass with short ``Vt``, sibling matrices at
    the root's children, downward pass (levels 1..m-1) with short ``Ut``,
    incoming expansions through the long bases ``Ulong`` on level m.
    ``downward="as-printed"`` runs the downward pass in Fig. 7's printed
    order (fine to coarse); it exists only so a test can show it is wrong."""
    q = np.asarray(q, dtype=np.float64)
    vec = q.ndim == 1
    if vec:
        q = q[:, None]
    u = np.zeros_like(q)
    if m == 0:
        return u[:, 0] if vec else u
    qh, uh = {}, {}
    # Build outgoing expansions on level m.
    for t in tree.level_nodes(m):
        qh[t] = Vlong[t].T @ q[tree.I(t)]
    # Upward pass: levels m-1 .. 1.
    for lev in range(m - 1, 0, -1):
        for t in tree.level_nodes(lev):
            a, b = tree.children(t)
            qh[t] = Vt[t].T @ np.vstack([qh[a], qh[b]])
    # Incoming expansions for the children of the root.
    a, b = tree.children(1)
    uh[a] = B[(a, b)] @ qh[b]
    uh[b] = B[(b, a)] @ qh[a]
    # Downward pass: levels 1 .. m-1 (coarse to fine).
    order = range(1, m) if downward == "coarse-to-fine" else range(m - 1, 0, -1)
    for lev in order:
        for t in tree.level_nodes(lev):
            if t not in uh:
                uh[t] = np.zeros((Ut[t].shape[1], q.shape[1]))
            a, b = tree.children(t)
            ka = _rank(tree, m, Ulong, Ut, a)
            uh[a] = B[(a, b)] @ qh[b] + Ut[t][:ka] @ uh[t]
            uh[b] = B[(b, a)] @ qh[a] + Ut[t][ka:] @ uh[t]
    # Incoming expansions on level m.
    for t in tree.level_nodes(m):
        u[tree.I(t)] = Ulong[t] @ uh[t]
    return u[:, 0] if vec else u


def _rank(tree, m, Ulong, Ut, a):
    """Rank of node a's incoming basis: the long basis on level m, else the
    column count of its short transfer.  It is also the number of rows of the
    parent's short transfer that couple to a."""
    if tree.level(a) == m:
        return Ulong[a].shape[1]
    return Ut[a].shape[1]


def apply_partial_adjoint(tree, m, Ulong, Vlong, Ut, Vt, B, q):
    """``(A^(m))^* q``: the same sweep with U and V exchanged and
    ``B_ab -> B_ba^*``."""
    Bt = {(a, b): B[(b, a)].T for (a, b) in B}
    return apply_partial(tree, m, Vlong, Ulong, Vt, Ut, Bt, q)


def apply_hbs(h: HBS, x: np.ndarray, adjoint: bool = False) -> np.ndarray:
    tree = h.tree
    x = np.asarray(x, dtype=np.float64)
    vec = x.ndim == 1
    if vec:
        x = x[:, None]
    if adjoint:
        y = apply_partial_adjoint(tree, tree.L, h.U, h.V, h.Ut, h.Vt, h.B, x)
    else:
        y = apply_partial(tree, tree.L, h.U, h.V, h.Ut, h.Vt, h.B, x)
    for t in tree.leaves():
        D = h.D[t].T if adjoint else h.D[t]
        y[tree.I(t)] += D @ x[tree.I(t)]
    return y[:, 0] if vec else y


# ---------------------------------------------------------------------------
# Compression: Fig. 4 (storage-efficient scheme)
# ---------------------------------------------------------------------------
class CompressStats:
    def __init__(self):
        self.calls = 0          # black-box invocations (A or A^*)
        self.columns = 0        # columns sampled in total


def _sample(op, X, adjoint, stats):
    stats.calls += 1
    stats.columns += X.shape[1]
    return op.apply_adjoint(X) if adjoint else op.apply(X)


def compress(op, n: int, leaf: int, r: int, seed: int, rank: int | None = None,
             tol: float | None = None, to_id: bool = True,
             b_pairing: str = "derived", trace: dict | None = None):
    """Randomized HBS compression of the black box ``op`` (with ``apply`` and
    ``apply_adjoint`` on N x c blocks).  ``r`` = samples per level (= k + p).
    Fig. 4 builds the orthonormal HBS keeping r columns per node; if
    ``to_id`` the Fig. 5 sweep converts it to HBS-ID, truncating to ``rank``
    (fixed-rank mode, when ``tol`` is None) or to tolerance ``tol``.
    Returns ``(HBS, stats, extras)``; ``extras`` holds the orthonormal form
    and the spanning-matrix weights y, z.
    ``b_pairing="as-printed"`` builds B with Fig. 4's printed pairing of X
    and b; ``trace`` (a dict) receives per-level samples and long bases.
    Both exist only for tests."""
    tree = Tree(n, leaf)
    L = tree.L
    h = HBS(tree)
    stats = CompressStats()
    Ulong, Vlong = {}, {}       # long bases of the level being processed
    y, z = {}, {}               # spanning matrices Y_t = Ulong_t diag(y_t)
    for lev in range(L):
        # Build the random matrices Omega_1 and Omega_2.
        G = rng.level_gaussian(seed, lev, n, r)
        Om1 = np.zeros((n, r))
        Om2 = np.zeros((n, r))
        for t in tree.level_nodes(lev):
            a, b = tree.children(t)
            Om1[tree.I(a)] = G[tree.I(a)]
            Om2[tree.I(b)] = G[tree.I(b)]
        # Samples for the incoming bases, minus the coarser levels A^(lev).
        sub = lambda X: apply_partial(tree, lev, Ulong, Vlong, h.Ut, h.Vt, h.B, X)
        Y1 = _sample(op, Om2, False, stats) - sub(Om2)
        Y2 = _sample(op, Om1, False, stats) - sub(Om1)
        if trace is not None:
            trace.setdefault("G", []).append(G)
            trace.setdefault("Y1", []).append(Y1)
            trace.setdefault("Y2", []).append(Y2)
        # Orthonormalise to build the incoming bases.
        newU = {}
        for t in tree.level_nodes(lev):
            a, b = tree.children(t)
            if t == 1:
                Y1loc = Y1[tree.I(a)]
                Y2loc = Y2[tree.I(b)]
            else:
                Y1loc = np.hstack([Y1[tree.I(a)], Ulong[t][tree.J(a)] * y[t][None, :]])
                Y2loc = np.hstack([Y2[tree.I(b)], Ulong[t][tree.J(b)] * y[t][None, :]])
            Ua, ya, _ = lowrank.svd(Y1loc, k=r)
            Ub, yb, _ = lowrank.svd(Y2loc, k=r)
            newU[a], newU[b], y[a], y[b] = Ua, Ub, ya, yb
            Om1[tree.I(a)] = 0.0
            Om2[tree.I(b)] = 0.0
            Om1[tree.I(a), :Ua.shape[1]] = Ua
            Om2[tree.I(b), :Ub.shape[1]] = Ub
            if t != 1:
                h.Ut[t] = np.vstack([Ua.T @ Ulong[t][tree.J(a)],
                                     Ub.T @ Ulong[t][tree.J(b)]])
        # Samples for the outgoing bases, minus (A^(lev))^*.
        subT = lambda X: apply_partial_adjoint(tree, lev, Ulong, Vlong, h.Ut, h.Vt, h.B, X)
        Z1 = _sample(op, Om2, True, stats) - subT(Om2)
        Z2 = _sample(op, Om1, True, stats) - subT(Om1)
        newV = {}
        for t in tree.level_nodes(lev):
            a, b = tree.children(t)
            ka, kb = newU[a].shape[1], newU[b].shape[1]
            if t == 1:
                Z1loc = Z1[tree.I(a), :kb]
                Z2loc = Z2[tree.I(b), :ka]
            else:
                Z1loc = np.hstack([Z1[tree.I(a), :kb], Vlong[t][tree.J(a)] * z[t][None, :]])
                Z2loc = np.hstack([Z2[tree.I(b), :ka], Vlong[t][tree.J(b)] * z[t][None, :]])
            Va, b21, X1 = lowrank.svd(Z1loc, k=r)
            Vb, b12, X2 = lowrank.svd(Z2loc, k=r)
            newV[a], newV[b], z[a], z[b] = Va, Vb, b21, b12
            # Sibling matrices (pairing of X and b as derived, see module doc).
            if b_pairing == "derived":
                h.B[(b, a)] = X1[:kb, :] * b21[None, :]
                h.B[(a, b)] = X2[:ka, :] * b12[None, :]
            else:
                h.B[(a, b)] = X1[:kb, :] * b12[None, :]
                h.B[(b, a)] = X2[:ka, :] * b21[None, :]
            if t != 1:
                h.Vt[t] = np.vstack([Va.T @ Vlong[t][tree.J(a)],
                                     Vb.T @ Vlong[t][tree.J(b)]])
        if trace is not None:
            trace.setdefault("Ulong", []).append(dict(newU))
            trace.setdefault("Vlong", []).append(dict(newV))
        # The long bases of level lev are no longer needed.
        Ulong, Vlong = newU, newV
    # Extract the diagonal matrices.
    nmax = tree.nmax()
    Om = np.zeros((n, nmax))
    for t in tree.leaves():
        Om[tree.I(t), :tree.size(t)] = np.eye(tree.size(t))
    Yd = _sample(op, Om, False, stats) - apply_partial(tree, L, Ulong, Vlong, h.Ut, h.Vt, h.B, Om)
    for t in tree.leaves():
        h.D[t] = Yd[tree.I(t), :tree.size(t)].copy()
    if L == 0:
        return h, stats, dict(y=y, z=z)
    h.U, h.V = Ulong, Vlong
    extras = dict(y=dict(y), z=dict(z), ortho=_copy_hbs(h))
    if to_id:
        hbs_id(h, y, z, rank=rank, tol=tol, r=r)
    return h, stats, extras


def compress_adaptive(op, n: int, leaf: int, k0: int, p: int, seed: int, tol: float,
                      e_target: float, r_max: int = 48):
    """Adaptive sampling around Fig. 4/5 (the paper fixes the samples per
    level in advance, to be picked above any numerical rank met, and notes
    that adaptive rank determination could be built in; Sec. 4.3, Remark 1.1
    on the failure risk, Sec. 2.5): compress in tolerance mode with rank cap
    k and r = k + p samples per level; if some node's revealed eps-rank
    reaches the cap (the samples may not have captured its block), or the
    posterior estimate E of Sec. 5 (ten probes, phase 1 of the stream keyed
    by ``seed``) exceeds ``e_target``, double the cap (at most r_max - p) and
    compress again.  The Gaussian blocks are defined by (row, column, level),
    so a larger r keeps the first columns of every level's block.  Returns
    ``(h, rounds)`` with ``rounds`` a list of ``(k, saturated, E)``."""
    k = k0
    rounds = []
    while True:
        h, st, _ = compress(op, n, leaf, k + p, seed, rank=k, tol=tol)
        nodes = range(2, 2 ** (h.tree.L + 1))
        sat = any(h.rank_u(t) >= k or h.rank_v(t) >= k for t in nodes)
        E = metrics.estimate_E(op.apply, h.apply, n, seed=seed)
        rounds.append((k, sat, E))
        if (not sat and E <= e_target) or k + p >= r_max:
            return h, rounds
        k = min(2 * k, r_max - p)


def _copy_hbs(h: HBS) -> HBS:
    c = HBS(h.tree)
    for name in ("U", "V", "Ut", "Vt", "B", "D"):
        setattr(c, name, {k: v.copy() for k, v in getattr(h, name).items()})
    return c


# ---------------------------------------------------------------------------
# Fig. 5: conversion to HBS-ID with adaptive (or fixed) ranks
# ---------------------------------------------------------------------------
def hbs_id(h: HBS, y: dict, z: dict, rank: int | None, tol: float | None, r: int):
    """In-place conversion of the orthonormal HBS ``h`` (with spanning weights
    y, z) to HBS-ID: interpolative bases with an identity on the skeleton
    rows, and sibling matrices ``B^skel = U_a^samp B_ab (V_b^samp)^*``, which
    equal ``A(skel_in_a, skel_out_b)`` (eq. ben0-ben2)."""
    tree = h.tree
    L = tree.L
    kmax = r if rank is None else rank
    eps = tol
    Usamp, Vsamp = {}, {}
    newU, newV, newUt, newVt, newB = {}, {}, {}, {}, {}
    # Leaves.
    for t in tree.leaves():
        Ytmp = h.U[t] * y[t][None, :]
        Ztmp = h.V[t] * z[t][None, :]
        gi, go = [], []
        Jin, Pin = lowrank.id_rows(Ytmp, kmax, eps, gi)
        Jout, Pout = lowrank.id_rows(Ztmp, kmax, eps, go)
        h.gaps_in[t], h.gaps_out[t] = np.array(gi), np.array(go)
        Usamp[t] = h.U[t][Jin]
        Vsamp[t] = h.V[t][Jout]
        newU[t], newV[t] = Pin, Pout
        h.skel_in[t] = tree.lo[t] + Jin
        h.skel_out[t] = tree.lo[t] + Jout
    # Parents, levels L-1 .. 1.
    for lev in range(L - 1, 0, -1):
        for t in tree.level_nodes(lev):
            a, b = tree.children(t)
            ka_old = h.rank_u(a)
            kva_old = h.rank_v(a)
            Utmp = np.vstack([Usamp[a] @ h.Ut[t][:ka_old], Usamp[b] @ h.Ut[t][ka_old:]])
            Vtmp = np.vstack([Vsamp[a] @ h.Vt[t][:kva_old], Vsamp[b] @ h.Vt[t][kva_old:]])
            gi, go = [], []
            Jin, Pin = lowrank.id_rows(Utmp * y[t][None, :], kmax, eps, gi)
            Jout, Pout = lowrank.id_rows(Vtmp * z[t][None, :], kmax, eps, go)
            h.gaps_in[t], h.gaps_out[t] = np.array(gi), np.array(go)
            newB[(a, b)] = Usamp[a] @ h.B[(a, b)] @ Vsamp[b].T
            newB[(b, a)] = Usamp[b] @ h.B[(b, a)] @ Vsamp[a].T
            Usamp[t] = Utmp[Jin]
            Vsamp[t] = Vtmp[Jout]
            newUt[t], newVt[t] = Pin, Pout
            cand_in = np.concatenate([h.skel_in[a], h.skel_in[b]])
            cand_out = np.concatenate([h.skel_out[a], h.skel_out[b]])
            h.skel_in[t] = cand_in[Jin]
            h.skel_out[t] = cand_out[Jout]
    # The children of the root.
    a, b = tree.children(1)
    newB[(a, b)] = Usamp[a] @ h.B[(a, b)] @ Vsamp[b].T
    newB[(b, a)] = Usamp[b] @ h.B[(b, a)] @ Vsamp[a].T
    h.U, h.V, h.Ut, h.Vt, h.B = newU, newV, newUt, newVt, newB
    h.is_id = True
    return h


def solve(h: HBS, b: np.ndarray) -> np.ndarray:
    """``x = A_H^-1 b`` by its plain definition: LU (LAPACK) of the densified
    represented matrix (small N only); the reference for the fast direct
    solver built on the compressed form."""
    return np.linalg.solve(h.dense(), np.asarray(b, dtype=np.float64))


# ---------------------------------------------------------------------------
# Building an HBS from flat generator arrays (the synthetic operators)
# ---------------------------------------------------------------------------
def from_generators(g: dict) -> HBS:
    """HBS object from the flat layout of ``workloads.synthetic_hbs``."""
    tree = Tree(g["n"], g["leaf"])
    h = HBS(tree)
    k = g["k"]
    f = lambda a: np.asarray(a, dtype=np.float64)
    for t in tree.leaves():
        I = tree.I(t)
        if tree.L > 0:
            h.U[t] = f(g["U"][I]).copy()
            h.V[t] = f(g["V"][I]).copy()
        h.D[t] = f(g["D"][I, :tree.size(t)]).copy()
    for t in range(2, 2 ** tree.L):
        h.Ut[t] = f(g["Ut"][t]).copy()
        h.Vt[t] = f(g["Vt"][t]).copy()
    for t in range(2, 2 ** (tree.L + 1)):
        h.B[(t ^ 1, t)] = f(g["B"][t]).copy()
    return h
