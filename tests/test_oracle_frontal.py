"""Pins of the frontal-matrix oracle (Sec. 5.4): the network matrix of a tiny
grid written out by hand, closed forms from series / parallel conductances,
the invariants of a Schur complement of a graph Laplacian (a Laplacian again,
with the same effective resistances between the kept nodes, computed here
through the pseudo-inverse of the whole network), and the rank structure the
section's tables show (an HBS row block ranks twice a HODLR sibling block)."""
import numpy as np
import pytest

import workloads as wl
from oracle import frontal, hodlr


def test_network_matrix_of_a_two_by_three_grid():
    ch = np.array([[1.1, 1.2], [1.3, 1.4]])
    cv = np.array([[1.5, 1.6, 1.7]])
    B = frontal.laplacian(ch, cv).toarray()
    # nodes 0 1 2 / 3 4 5; bars 0-1 1.1, 1-2 1.2, 3-4 1.3, 4-5 1.4, 0-3 1.5, 1-4 1.6, 2-5 1.7
    E = np.zeros((6, 6))
    for p, q, c in ((0, 1, 1.1), (1, 2, 1.2), (3, 4, 1.3), (4, 5, 1.4), (0, 3, 1.5), (1, 4, 1.6),
                    (2, 5, 1.7)):
        E[p, p] += c
        E[q, q] += c
        E[p, q] = E[q, p] = -c
    np.testing.assert_array_equal(B, E)


def test_index_sets_split_at_the_middle_column():
    I1, I2, I3 = frontal.index_sets(3, 5)
    np.testing.assert_array_equal(I3, [2, 7, 12])
    np.testing.assert_array_equal(I1, [0, 1, 5, 6, 10, 11])
    np.testing.assert_array_equal(I2, [3, 4, 8, 9, 13, 14])


def test_one_row_is_zero():
    # a single grid row: each half is a dead-end chain hanging off the middle
    # node, so no current flows through it and A = 0
    ch, cv = wl.grid_conductivities(1, 41, seed=3)
    A = frontal.FrontalOp(ch, cv).dense()
    assert A.shape == (1, 1)
    assert abs(A[0, 0]) < 1e-13


def test_two_rows_three_columns_is_series_and_parallel():
    # middle nodes (0,1) and (1,1): joined directly by cv[0,1] and through each
    # side by three bars in series, the three paths in parallel
    ch, cv = wl.grid_conductivities(2, 3, seed=5)
    series = lambda *c: 1.0 / sum(1.0 / x for x in c)
    g = cv[0, 1] + series(ch[0, 0], cv[0, 0], ch[1, 0]) + series(ch[0, 1], cv[0, 2], ch[1, 1])
    A = frontal.FrontalOp(ch, cv).dense()
    np.testing.assert_allclose(A, g * np.array([[1.0, -1.0], [-1.0, 1.0]]), rtol=1e-14)


def test_unit_ladder_is_the_sum_of_its_parts():
    # width 3, unit bars: A is the middle column's own chain plus, for each
    # side, the reduction onto the middle nodes of that side's chain and its
    # rungs (built here by hand as a 2H-node network, reduced by a dense solve)
    H = 5
    A = frontal.FrontalOp(np.ones((H, 2)), np.ones((H - 1, 3))).dense()
    Lc = np.zeros((2 * H, 2 * H))

    def bar(p, q):
        Lc[p, p] += 1.0
        Lc[q, q] += 1.0
        Lc[p, q] -= 1.0
        Lc[q, p] -= 1.0

    for i in range(H):
        bar(i, H + i)          # rung: side node i -- middle node i
    for i in range(H - 1):
        bar(i, i + 1)          # side chain
    K = Lc[H:, H:] - Lc[H:, :H] @ np.linalg.solve(Lc[:H, :H], Lc[:H, H:])
    Lmid = np.diag([1.0] + [2.0] * (H - 2) + [1.0]) - np.eye(H, k=1) - np.eye(H, k=-1)
    np.testing.assert_allclose(A, Lmid + 2.0 * K, atol=1e-13)


@pytest.mark.parametrize("H,W", [(6, 7), (9, 41), (30, 11)])
def test_effective_resistances_are_kept(H, W):
    # Kron reduction keeps the effective resistance between kept nodes:
    # R(a, b) = (e_a - e_b)^T L^+ (e_a - e_b) in the whole network and in A
    ch, cv = wl.grid_conductivities(H, W, seed=H + W)
    B = frontal.laplacian(ch, cv).toarray()
    A = frontal.FrontalOp(ch, cv).dense()
    mid = (W - 1) // 2
    Bp, Ap = np.linalg.pinv(B), np.linalg.pinv(A)
    rng = np.random.default_rng(1)
    for _ in range(10):
        a, b = rng.choice(H, 2, replace=False)
        e = np.zeros(H * W)
        e[a * W + mid], e[b * W + mid] = 1.0, -1.0
        f = np.zeros(H)
        f[a], f[b] = 1.0, -1.0
        np.testing.assert_allclose(f @ Ap @ f, e @ Bp @ e, rtol=1e-10)


def test_schur_complement_is_a_connected_laplacian():
    ch, cv = wl.grid_conductivities(60, 41, seed=2)
    A = frontal.FrontalOp(ch, cv).dense()
    assert np.abs(A - A.T).max() < 1e-13 * np.abs(A).max()
    np.testing.assert_allclose(A @ np.ones(60), 0.0, atol=1e-12)
    off = A - np.diag(np.diag(A))
    assert off.max() <= 1e-14
    ev = np.linalg.eigvalsh(A)
    assert abs(ev[0]) < 1e-12 and ev[1] > 1e-6      # one null vector: connected


def test_sparse_products_match_the_dense_schur_complement():
    # the black box (sparse LU solves on N x c blocks) against A assembled
    # column by column from dense solves of the whole network: the solution
    # of B u = [0; 0; f] with u3 = x fixed gives A x as the net current
    H, W = 12, 9
    ch, cv = wl.grid_conductivities(H, W, seed=4)
    op = frontal.FrontalOp(ch, cv)
    B = frontal.laplacian(ch, cv).toarray()
    I1, I2, I3 = frontal.index_sets(H, W)
    inner = np.concatenate([I1, I2])
    X = wl.gaussian((H, 3), seed=9)
    # harmonic extension: potentials x on I3, no net current at inner nodes
    u = np.zeros((H * W, 3))
    u[I3] = X
    u[inner] = -np.linalg.solve(B[np.ix_(inner, inner)], B[np.ix_(inner, I3)] @ X)
    np.testing.assert_allclose(op.apply(X), (B @ u)[I3], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(op.apply_adjoint(X), op.apply(X), rtol=0, atol=0)


def test_hbs_rank_is_twice_the_hodlr_rank():
    # Tables 8 and 9: the HBS-ID rank (18) is twice the HODLR rank (9) -- a
    # segment of the separator talks to the rest through its two ends.  The
    # same 2:1 holds for this workload's blocks at eps = 1e-9
    H = 400
    ch, cv = wl.grid_conductivities(H, 41, seed=7)
    A = frontal.FrontalOp(ch, cv).dense()
    rank = lambda M: int((np.linalg.svd(M, compute_uv=False) > 1e-9 * np.linalg.norm(M, 2)).sum())
    sib = rank(A[:100, 100:200])
    row = rank(np.hstack([A[100:200, :100], A[100:200, 200:]]))
    assert 6 <= sib <= 16
    assert row == 2 * sib
    h, _ = hodlr.compress(frontal.FrontalOp(ch, cv), H, 100, 25, seed=11, rank=20, tol=1e-9)[:2]
    assert max(h.ranks().values()) == sib
