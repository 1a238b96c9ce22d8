"""Pins of the oracle's building blocks against what the paper and the
mathematics fix: the Fig. 1 tree, Philox known answers and Gaussian
statistics, Eckart-Young for the truncated SVD (Sec. 2.3), the ID's identity
and boundedness (Sec. 2.4) and its agreement with LAPACK's pivoted QR."""
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

from oracle import lowrank, rng
from oracle.tree import Tree

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                out.append(line.split())
    return out


def test_tree_matches_fig1():
    t = Tree(400, 50)
    assert t.L == 3
    for node, first, last in _rows("fig1_tree.txt"):
        node, first, last = int(node), int(first), int(last)
        assert t.lo[node] == first - 1 and t.hi[node] == last


@pytest.mark.parametrize("n,leaf", [(1, 1), (5, 8), (1000, 64), (576, 128), (8191, 64)])
def test_tree_partition_invariants(n, leaf):
    t = Tree(n, leaf)
    # Leaves partition [0, n) in order and hold at most `leaf` indices.
    leaves = list(t.leaves())
    assert t.lo[leaves[0]] == 0 and t.hi[leaves[-1]] == n
    for a, b in zip(leaves, leaves[1:]):
        assert t.hi[a] == t.lo[b]
    assert max(t.size(x) for x in leaves) <= leaf
    for p in range(1, 2 ** t.L):
        a, b = t.children(p)
        assert t.lo[a] == t.lo[p] and t.hi[b] == t.hi[p] and t.hi[a] == t.lo[b]
        assert abs(t.size(a) - t.size(b)) <= 1


def test_philox_known_answers():
    for row in _rows("philox4x32_10_kat.txt"):
        v = [int(x, 16) for x in row]
        out = rng.philox4x32_10(*[np.array([c]) for c in v[:4]], v[4], v[5])
        assert [int(o[0]) for o in out] == v[6:]


def test_box_muller_formula_and_statistics():
    g = rng.gaussian_block(2024, 3, np.arange(20000), 8, phase=0)
    # One entry by hand from the definition.
    w = rng.philox4x32_10(np.array([5]), np.array([3]), np.array([3]), np.array([0]), 2024, 0)
    m1 = (int(w[0][0]) >> 5) * 2 ** 26 + (int(w[1][0]) >> 6)
    m2 = (int(w[2][0]) >> 5) * 2 ** 26 + (int(w[3][0]) >> 6)
    u1, u2 = (m1 + 1) / 2.0 ** 53, m2 / 2.0 ** 53
    rad = np.sqrt(-2 * np.log(u1))
    assert g[5, 6] == pytest.approx(rad * np.cos(2 * np.pi * u2), rel=1e-15)
    assert g[5, 7] == pytest.approx(rad * np.sin(2 * np.pi * u2), rel=1e-15)
    flat = g.ravel()
    assert abs(flat.mean()) < 0.01 and abs(flat.var() - 1.0) < 0.02
    assert scipy.stats.kstest(flat, "norm").pvalue > 1e-3
    # Different levels / phases / seeds give different streams.
    assert not np.allclose(g, rng.gaussian_block(2024, 4, np.arange(20000), 8))
    assert not np.allclose(g, rng.gaussian_block(2025, 3, np.arange(20000), 8))


def test_stream_depends_only_on_coordinates():
    full = rng.gaussian_block(7, 2, np.arange(300), 12)
    part = rng.gaussian_block(7, 2, np.arange(100, 200), 12)
    assert np.array_equal(full[100:200], part)


def test_svd_modes_eckart_young():
    r = np.random.default_rng(0)
    A = r.standard_normal((60, 40)) @ np.diag(0.5 ** np.arange(40)) @ r.standard_normal((40, 40))
    s = np.linalg.svd(A, compute_uv=False)
    U, sk, V = lowrank.svd(A, k=7)
    err = np.linalg.norm(A - U @ np.diag(sk) @ V.T, 2)
    assert err == pytest.approx(s[7], rel=1e-10)                  # spectral: s_{k+1}
    ferr = np.linalg.norm(A - U @ np.diag(sk) @ V.T)
    assert ferr == pytest.approx(np.sqrt(np.sum(s[7:] ** 2)), rel=1e-10)
    U, se, V = lowrank.svd(A, eps=1e-6)
    assert se.size == int(np.sum(s > 1e-6 * s[0]))
    assert np.linalg.norm(U.T @ U - np.eye(se.size)) < 1e-13


def test_qr_orthonormal_basis():
    r = np.random.default_rng(1)
    Y = r.standard_normal((200, 30)) @ r.standard_normal((30, 30))
    Q = lowrank.qr(Y)
    assert np.linalg.norm(Q.T @ Q - np.eye(30)) < 1e-13
    assert np.linalg.norm(Y - Q @ (Q.T @ Y)) < 1e-12 * np.linalg.norm(Y)


def test_cpqr_pivots_match_lapack_on_generic_matrices():
    r = np.random.default_rng(2)
    for trial in range(5):
        M = r.standard_normal((30, 80)) * np.exp(r.uniform(-3, 3, 80))[None, :]
        perm, k, R = lowrank.cpqr(M, kmax=30)
        _, R2, P2 = scipy.linalg.qr(M, pivoting=True, mode="economic")
        assert k == 30
        assert np.array_equal(perm[:20], P2[:20])
        assert np.allclose(np.abs(np.diag(R)[:20]), np.abs(np.diag(R2)[:20]), rtol=1e-10)


def test_id_identity_and_exact_rank():
    r = np.random.default_rng(3)
    Y = r.standard_normal((120, 12)) @ r.standard_normal((12, 40))   # rank 12
    J, P = lowrank.id_rows(Y, kmax=40, eps=1e-12)
    assert len(J) == 12
    assert np.allclose(P[J], np.eye(12), atol=0)
    assert np.linalg.norm(Y - P @ Y[J]) < 1e-11 * np.linalg.norm(Y)
    assert np.max(np.abs(P)) <= 4.0           # CPQR ID: entries about <= 1
    J2, P2 = lowrank.id_rows(Y, kmax=5)       # fixed-rank mode
    assert len(J2) == 5 and np.allclose(P2[J2], np.eye(5))


def test_id_bound_random_samples():
    r = np.random.default_rng(4)
    for _ in range(10):
        Y = r.standard_normal((128, 48)) @ np.diag(0.7 ** np.arange(48))
        J, P = lowrank.id_rows(Y, kmax=32)
        assert np.max(np.abs(P)) <= 4.0
