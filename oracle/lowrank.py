"""The functions ``qr``, ``svd`` and ``id`` of Sec. 2.6 in their modes
(full / rank k / tolerance eps), Sec. 2.2-2.4.

As the paper does for small inputs (Sec. 2.6), mode 2 and mode 3 compute a
full factorisation with LAPACK and truncate it.

Reading of the tolerance (the paper states ``||A - ...|| <= eps`` with eps in
(0,1) and leaves absolute vs. relative open): it is *relative per block* --
keep singular values ``s_j > eps * s_1`` (SVD) and pivots
``|R_jj| > eps * |R_11|`` (ID).

The ID is column-pivoted QR in the Businger-Golub order (pivot = remaining
column of largest residual norm, lowest index on ties), residual norms
recomputed exactly at every step, stopped after k steps or at the tolerance;
``X = [I, R11^-1 R12]`` in pivoted order (Sec. 2.4).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular


def qr(A: np.ndarray, k: int | None = None) -> np.ndarray:
    """Orthonormal basis of the columns of A (Householder QR, economy).
    Mode 2 keeps the first ``k`` columns of Q."""
    Q, _ = np.linalg.qr(A, mode="reduced")
    if k is not None:
        Q = Q[:, :k]
    return Q


def svd(A: np.ndarray, k: int | None = None, eps: float | None = None):
    """``[U, s, V] = svd(A, .)``: economy SVD, truncated to rank k (mode 2) or
    to ``s_j > eps s_1`` (mode 3); returns ``U`` (m x k), ``s`` (k,),
    ``V`` (n x k) with ``A ~ U diag(s) V^T``."""
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    if eps is not None:
        keep = int(np.sum(s > eps * s[0])) if s.size and s[0] > 0 else 0
        if k is not None:
            keep = min(keep, k)
    elif k is not None:
        keep = min(k, s.size)
    else:
        keep = s.size
    return U[:, :keep], s[:keep], Vt[:keep].T


def cpqr(M: np.ndarray, kmax: int, eps: float | None = None, gaps: list | None = None):
    """Column-pivoted Householder QR of M (m x n), at most ``kmax`` steps,
    stopping early when the largest remaining residual column norm is
    ``<= eps * |R_11|``.  Returns ``(perm, k, R)`` with ``M[:, perm] ~ Q R``,
    R of shape (k, n) upper trapezoidal in pivoted order.
    If ``gaps`` is a list, step j appends ``(n1 - n2) / |R_11|``, the margin
    by which the chosen pivot's residual norm n1 beat the runner-up's n2
    (0 with a single candidate left): a pivot decided by a margin far above
    the rounding of the input is the same in any correct implementation."""
    A = np.array(M, dtype=np.float64, copy=True)
    m, n = A.shape
    perm = np.arange(n)
    steps = min(m, n, kmax)
    ref = None
    k = 0
    for j in range(steps):
        norms = np.sqrt(np.sum(A[j:, j:] ** 2, axis=0))
        p = j + int(np.argmax(norms))          # first maximum: lowest index
        nrm = norms[p - j]
        if ref is None:
            ref = nrm
        if nrm == 0.0 or (eps is not None and nrm <= eps * ref):
            break
        if gaps is not None:
            rest = np.delete(norms, p - j)
            gaps.append((nrm - (rest.max() if rest.size else nrm)) / ref)
        if p != j:
            A[:, [j, p]] = A[:, [p, j]]
            perm[[j, p]] = perm[[p, j]]
        # Householder reflector zeroing A[j+1:, j].
        x = A[j:, j].copy()
        alpha = -np.copysign(np.linalg.norm(x), x[0])
        v = x
        v[0] -= alpha
        vn = np.dot(v, v)
        if vn > 0.0:
            A[j:, j:] -= np.outer(v, (2.0 / vn) * (v @ A[j:, j:]))
        A[j, j] = alpha
        A[j + 1:, j] = 0.0
        k = j + 1
    R = np.triu(A[:k, :])
    return perm, k, R


def id_rows(Y: np.ndarray, kmax: int, eps: float | None = None, gaps: list | None = None):
    """``[T, J] = id(Y^*, .)`` of Sec. 4.3 (eq. buildTJ), in the form used to
    make interpolative bases: returns ``(J, P)`` where ``J`` lists the k
    skeleton rows of Y and ``P`` (n x k) satisfies ``Y ~ P Y[J, :]`` with
    ``P[J, :] = I_k`` (P is the transpose of the ID's X).  ``gaps``: see
    ``cpqr``."""
    Mt = Y.T                                   # r x n; columns = rows of Y
    n = Mt.shape[1]
    perm, k, R = cpqr(Mt, kmax, eps, gaps)
    J = perm[:k].copy()
    X = np.zeros((k, n))
    if k > 0:
        X[:, perm[:k]] = np.eye(k)
        if n > k:
            X[:, perm[k:]] = solve_triangular(R[:, :k], R[:, k:], lower=False)
    return J, X.T
