"""Reference gradients of the compressed apply ``y = A_H(U, V, Ut, Vt, B, D) x``.

``A_H`` is assembled *densely* from its generators by the definition of the
HBS format (Sec. 2.9, eq. babytelescope): long bases by explicit telescoping
``Ulong_t = diag(Ulong_a, Ulong_b) Ut[t]``, every sibling block
``A(I_sib(v), I_v) = Ulong_sib B[v] Vlong_v^T``, diagonal leaf blocks ``D``.
Torch CPU autograd in float64 then differentiates ``<gy, A_H x>``; no sweep,
no expansion and nothing of the fast apply is used, so this is independent of
any fast backward.

Generators use the flat layout of ``workloads.synthetic_hbs``: U, V (n, k);
Ut, Vt (2**(L+1), 2k, k); B (2**(L+1), k, k); D (n, nmax).
"""
from __future__ import annotations

import numpy as np
import torch

from .tree import Tree


def dense_from_generators(tree: Tree, U, V, Ut, Vt, B, D):
    n, L = tree.n, tree.L
    A = torch.zeros((n, n), dtype=U.dtype)
    # Diagonal blocks.
    parts = []
    for t in tree.leaves():
        I = tree.I(t)
        m = tree.size(t)
        pad_l = tree.lo[t]
        pad_r = n - tree.hi[t]
        parts.append(torch.nn.functional.pad(D[I, :m], (pad_l, pad_r)))
    A = A + torch.cat(parts, dim=0)
    if L == 0:
        return A
    # Long bases by explicit telescoping, finest level first.
    Ul = {t: U[tree.I(t)] for t in tree.leaves()}
    Vl = {t: V[tree.I(t)] for t in tree.leaves()}
    for lev in range(L - 1, 0, -1):
        for t in tree.level_nodes(lev):
            a, b = tree.children(t)
            k = Ul[a].shape[1]
            Ul[t] = torch.cat([Ul[a] @ Ut[t][:k], Ul[b] @ Ut[t][k:]], dim=0)
            Vl[t] = torch.cat([Vl[a] @ Vt[t][:k], Vl[b] @ Vt[t][k:]], dim=0)
    # Sibling blocks.
    for v in range(2, 2 ** (L + 1)):
        s = v ^ 1
        blk = Ul[s] @ B[v] @ Vl[v].T
        pad = (tree.lo[v], n - tree.hi[v], tree.lo[s], n - tree.hi[s])
        A = A + torch.nn.functional.pad(blk, pad)
    return A


def reference_gradients(g: dict, x: np.ndarray, gy: np.ndarray):
    """Gradients of ``<gy, A_H x>`` w.r.t. x and the generators; returns a
    dict of float64 numpy arrays in the generators' layout."""
    tree = Tree(g["n"], g["leaf"])
    T = lambda a: torch.tensor(np.asarray(a, dtype=np.float64), requires_grad=True)
    U, V, Ut, Vt, B, D = (T(g[k]) for k in ("U", "V", "Ut", "Vt", "B", "D"))
    xt = T(x)
    A = dense_from_generators(tree, U, V, Ut, Vt, B, D)
    y = A @ xt
    loss = (torch.tensor(np.asarray(gy, dtype=np.float64)) * y).sum()
    loss.backward()
    out = dict(x=xt.grad, U=U.grad, V=V.grad, Ut=Ut.grad, Vt=Vt.grad, B=B.grad, D=D.grad)
    return {k: v.detach().numpy() for k, v in out.items()}, y.detach().numpy()
