"""Pins of the oracle's HBS path (Fig. 4, Fig. 5, Fig. 7) against what the
paper and the mathematics fix:

* exact recovery of operators with off-diagonal rank exactly k (range
  finder with s_{k+1} = 0, Sec. 2.5; peeling identity eq. gretchen), with
  revealed ranks exactly k;
* Fig. 7 + D equals a dense assembly written from the format's definition
  (eq. babytelescope), and the adjoint passes the dot-product test;
* the peeled sample equals the sibling block times the Gaussian (eq. gretchen);
* telescoping of the spanning matrices, orthonormality, the HBS-ID identity,
  nested skeletons, and ``B^skel = A(skel_in, skel_out)`` (eq. ben1);
* the literal sample count of Fig. 4 (4 r L + n_max columns);
* brute-force neutered-block optimality on tiny N (Eckart-Young + eq. err_prob);
* the paper's printed B pairing (Fig. 3/4) and downward order (Fig. 7) fail.
"""
import numpy as np
import pytest

import workloads as W
from oracle import grad, hbs, metrics, operators
from oracle.tree import Tree


def _dense_from_gen(g):
    import torch
    tree = Tree(g["n"], g["leaf"])
    T = {k: torch.tensor(g[k]) for k in ("U", "V", "Ut", "Vt", "B", "D")}
    return grad.dense_from_generators(tree, **T).numpy()


@pytest.fixture(scope="module")
def syn():
    g = W.synthetic_hbs(1024, 64, 10, seed=1)
    return g, _dense_from_gen(g)


def test_apply_equals_dense_definition(syn):
    g, A = syn
    h = hbs.from_generators(g)
    x = W.gaussian((1024, 3), seed=5)
    assert np.linalg.norm(h.apply(x) - A @ x) < 1e-13 * np.linalg.norm(A @ x)
    assert np.linalg.norm(h.apply_adjoint(x) - A.T @ x) < 1e-13 * np.linalg.norm(A.T @ x)
    yv = W.gaussian(1024, seed=6)
    lhs = yv @ h.apply(x[:, 0])
    rhs = h.apply_adjoint(yv) @ x[:, 0]
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_printed_downward_order_fails(syn):
    g, A = syn
    h = hbs.from_generators(g)
    x = W.gaussian((1024, 2), seed=5)
    y = hbs.apply_partial(h.tree, h.tree.L, h.U, h.V, h.Ut, h.Vt, h.B, x,
                          downward="as-printed")
    for t in h.tree.leaves():
        y[h.tree.I(t)] += h.D[t] @ x[h.tree.I(t)]
    assert np.linalg.norm(y - A @ x) > 1e-3 * np.linalg.norm(A @ x)


@pytest.mark.parametrize("to_id", [False, True])
def test_exact_recovery_synthetic_hbs(syn, to_id):
    g, A = syn
    h, st, ex = hbs.compress(operators.DenseOp(A), 1024, 64, r=20, seed=11, rank=10,
                             to_id=to_id)
    assert metrics.rel_fro(h.dense(), A) < 1e-12
    if to_id:
        assert all(h.rank_u(t) == 10 and h.rank_v(t) == 10 for t in range(2, 2 ** (h.tree.L + 1)))


def test_exact_recovery_tolerance_mode_reveals_rank(syn):
    g, A = syn
    h, st, ex = hbs.compress(operators.DenseOp(A), 1024, 64, r=20, seed=12, tol=1e-11)
    assert metrics.rel_fro(h.dense(), A) < 1e-12
    ranks = {h.rank_u(t) for t in range(2, 2 ** (h.tree.L + 1))}
    assert ranks == {10}


def test_printed_b_pairing_fails(syn):
    g, A = syn
    h, _, ex = hbs.compress(operators.DenseOp(A), 1024, 64, r=20, seed=11, rank=10,
                            to_id=False, b_pairing="as-printed")
    assert metrics.rel_fro(h.dense(), A) > 1e-3


def test_sample_count_fig4(syn):
    g, A = syn
    n, leaf, r = 1024, 64, 20
    h, st, _ = hbs.compress(operators.DenseOp(A), n, leaf, r=r, seed=1, rank=10)
    L = h.tree.L
    assert st.columns == 4 * r * L + h.tree.nmax()
    assert st.calls == 4 * L + 1


def test_peeling_identity_eq_gretchen(syn):
    g, A = syn
    tr = {}
    hbs.compress(operators.DenseOp(A), 1024, 64, r=20, seed=3, rank=10, trace=tr)
    tree = Tree(1024, 64)
    for lev in range(tree.L):
        G, Y1, Y2 = tr["G"][lev], tr["Y1"][lev], tr["Y2"][lev]
        for t in tree.level_nodes(lev):
            a, b = tree.children(t)
            ref1 = A[tree.I(a), tree.I(b)] @ G[tree.I(b)]
            ref2 = A[tree.I(b), tree.I(a)] @ G[tree.I(a)]
            assert np.linalg.norm(Y1[tree.I(a)] - ref1) < 1e-12 * np.linalg.norm(ref1)
            assert np.linalg.norm(Y2[tree.I(b)] - ref2) < 1e-12 * np.linalg.norm(ref2)


def test_orthonormality_and_telescoping(syn):
    g, A = syn
    tr = {}
    h, _, ex = hbs.compress(operators.DenseOp(A), 1024, 64, r=20, seed=4, rank=10, trace=tr)
    tree = h.tree
    y = ex["y"]
    o = ex["ortho"]
    for lev in range(1, tree.L):
        Ul_parent, Ul_child = tr["Ulong"][lev - 1], tr["Ulong"][lev]
        for t in tree.level_nodes(lev):
            a, b = tree.children(t)
            Q = Ul_parent[t]
            assert np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1])) < 1e-13
            tele = np.vstack([Ul_child[a] @ o.Ut[t][:Ul_child[a].shape[1]],
                              Ul_child[b] @ o.Ut[t][Ul_child[a].shape[1]:]])
            # The spanning matrix Y_t = Ulong_t diag(y_t) telescopes.
            err = np.linalg.norm((Q - tele) * y[t][None, :])
            assert err < 1e-12 * np.linalg.norm(y[t])


def test_hbs_id_structure_and_submatrix_property(syn):
    g, A = syn
    h, _, _ = hbs.compress(operators.DenseOp(A), 1024, 64, r=20, seed=5, rank=10)
    tree = h.tree
    for t in tree.leaves():
        J = h.skel_in[t] - tree.lo[t]
        assert np.allclose(h.U[t][J], np.eye(len(J)))
    for lev in range(1, tree.L):
        for t in tree.level_nodes(lev):
            a, b = tree.children(t)
            assert set(h.skel_in[t]) <= set(h.skel_in[a]) | set(h.skel_in[b])
            assert set(h.skel_out[t]) <= set(h.skel_out[a]) | set(h.skel_out[b])
    for v in range(2, 2 ** (tree.L + 1)):
        s = v ^ 1
        ref = A[np.ix_(h.skel_in[s], h.skel_out[v])]
        assert np.linalg.norm(h.B[(s, v)] - ref) < 1e-12 * np.linalg.norm(ref)


@pytest.fixture(scope="module")
def logker():
    P = W.ellipse_points(512)
    K = operators.KernelOp(P, "log")
    return K, K.dense()


def test_kernel_tolerance_mode_error_and_E(logker):
    K, A = logker
    h, _, ex = hbs.compress(K, 512, 32, r=50, seed=7, tol=1e-10)
    assert metrics.rel_fro(ex["ortho"].dense(), A) < 1e-12
    assert metrics.rel_fro(h.dense(), A) < 1e-8
    E = metrics.estimate_E(K.apply, h.apply, 512)
    assert E < 1e-8


def test_kernel_submatrix_property_to_tolerance(logker):
    K, A = logker
    h, _, _ = hbs.compress(K, 512, 32, r=50, seed=8, tol=1e-10)
    for v in range(2, 2 ** (h.tree.L + 1)):
        s = v ^ 1
        ref = A[np.ix_(h.skel_in[s], h.skel_out[v])]
        assert np.linalg.norm(h.B[(s, v)] - ref) < 1e-7 * np.linalg.norm(A)


def test_neutered_block_error_bruteforce(logker):
    """Fixed rank k: on every neutered row block A(I_t, I_t^c) the HBS error
    is within the randomized bound (eq. err_prob, with a factor L for
    aggregation over levels) of the best rank-k error (Eckart-Young).  A
    node's neutered block contains its ancestors' far field, so the bound
    takes the largest s_{k+1} over the node and its ancestors."""
    K, A = logker
    k, p = 16, 10
    h, _, ex = hbs.compress(K, 512, 32, r=k + p, seed=9, rank=k)
    Ah = h.dense()
    tree = h.tree
    sk1 = {}
    for lev in range(1, tree.L + 1):
        for t in tree.level_nodes(lev):
            I = np.arange(tree.lo[t], tree.hi[t])
            Ic = np.setdiff1d(np.arange(512), I)
            s = np.linalg.svd(A[np.ix_(I, Ic)], compute_uv=False)
            sk1[t] = max(s[k], sk1.get(t // 2, 0.0))
            err = np.linalg.norm(A[np.ix_(I, Ic)] - Ah[np.ix_(I, Ic)], 2)
            bound = (1 + 11 * np.sqrt(k + p) * np.sqrt(min(len(I), len(Ic)))) * sk1[t]
            assert err <= tree.L * bound
            assert err >= 0.99 * s[k]          # never better than optimal


def test_storage_linear_in_n():
    """HBS memory per index stays flat as N doubles (Sec. 4.4, Sec. 5)."""
    per = []
    for n in (512, 1024, 2048):
        g = W.synthetic_hbs(n, 64, 8, seed=2)
        A = _dense_from_gen(g)
        h, _, _ = hbs.compress(operators.DenseOp(A), n, 64, r=16, seed=1, rank=8)
        per.append(h.storage_reals() / n)
    assert max(per) / min(per) < 1.15


def _export_like(ho, R):
    """The oracle's HBS-ID form in the layout of the library's export (heap
    indexed, ranks padded to R), to check the parity helpers themselves."""
    import torch
    t_ = ho.tree
    L, n = t_.L, t_.n
    nn = 2 ** (L + 1)
    U, V = np.zeros((n, R)), np.zeros((n, R))
    Ut, Vt = np.zeros((nn, 2 * R, R)), np.zeros((nn, 2 * R, R))
    B = np.zeros((nn, R, R))
    ru, rv = np.zeros(nn, np.int32), np.zeros(nn, np.int32)
    si, so = np.full((nn, R), -1, np.int32), np.full((nn, R), -1, np.int32)
    for t in range(2, nn):
        ru[t], rv[t] = ho.rank_u(t), ho.rank_v(t)
        si[t, :ru[t]], so[t, :rv[t]] = ho.skel_in[t], ho.skel_out[t]
        if t in ho.U:
            U[t_.I(t), :ru[t]], V[t_.I(t), :rv[t]] = ho.U[t], ho.V[t]
        else:
            a, b = 2 * t, 2 * t + 1
            for M, src, ka, kb in ((Ut, ho.Ut[t], ho.rank_u(a), ho.rank_u(b)),
                                   (Vt, ho.Vt[t], ho.rank_v(a), ho.rank_v(b))):
                M[t, :ka, :src.shape[1]] = src[:ka]
                M[t, R:R + kb, :src.shape[1]] = src[ka:]
        Bb = ho.B[(t ^ 1, t)]
        B[t, :Bb.shape[0], :Bb.shape[1]] = Bb
    T = torch.from_numpy
    return dict(U=T(U), V=T(V), Ut=T(Ut), Vt=T(Vt), B=T(B), rank_u=ru, rank_v=rv, skel_in=si,
                skel_out=so, L=L, R=R)


def test_parity_helpers_accept_the_oracle_and_catch_planted_errors():
    """The structural checks the GPU tests apply (identity rows, nested
    skeletons, B^skel = A(skel)) and the skeleton-prefix comparison accept
    the oracle's own exact HBS-ID, and catch a swapped skeleton and a
    perturbed B^skel (mistakes planted in a copy of the oracle's output)."""
    import parity_util as PU
    n, leaf, k, p = 512, 64, 8, 6
    g = W.synthetic_hbs(n, leaf, k, seed=3)
    hf = hbs.from_generators(g)
    A = hf.dense()
    ho, _, _ = hbs.compress(operators.HBSOp(hf), n, leaf, k + p, 2, rank=k)
    ent = lambda r, c: A[np.ix_(r, c)]
    e = _export_like(ho, k + p)
    assert PU.hbs_id_structure(e, ent) < 1e-12
    assert PU.skeleton_prefix_mismatches(e, ho)[0] == []
    e2 = _export_like(ho, k + p)
    e2["B"][5, 0, 0] += 1e-6 * float(np.abs(A).max())
    assert PU.hbs_id_structure(e2, ent) > 1e-7
    e3 = _export_like(ho, k + p)
    leaf0 = 2 ** ho.tree.L
    e3["skel_in"][leaf0, [0, 1]] = e3["skel_in"][leaf0, [1, 0]]
    bad, _ = PU.skeleton_prefix_mismatches(e3, ho)
    assert bad and bad[0][1] == leaf0
    with pytest.raises(AssertionError):
        PU.hbs_id_structure(e3, ent)


def test_product_of_hbs_operators_has_rank_2k():
    """Sec. 5.2 (operator multiplication): the product of two HBS operators
    of rank k with nested bases is HBS of rank at most 2k -- the incoming
    basis of a node t must span H1(I_t, I_t) U2_t and U1_t, both nested in
    the children's.  Compressing the product black box recovers it exactly
    at rank 2k and not at 2k - 1 (a pin of the product operator and of the
    compression on a black box that is not itself given in HBS form)."""
    n, leaf, k, p = 1024, 64, 6, 8
    h1 = hbs.from_generators(W.synthetic_hbs(n, leaf, k, seed=11))
    h2 = hbs.from_generators(W.synthetic_hbs(n, leaf, k, seed=12))
    A = h1.dense() @ h2.dense()
    op = operators.ProductOp(operators.HBSOp(h1), operators.HBSOp(h2))
    x = W.gaussian((n, 3), seed=1)
    assert np.allclose(op.apply(x), A @ x, rtol=0, atol=1e-12 * np.abs(A).max() * n)
    assert np.allclose(op.apply_adjoint(x), A.T @ x, rtol=0, atol=1e-12 * np.abs(A).max() * n)
    ho, _, _ = hbs.compress(op, n, leaf, 2 * k + p, 5, rank=2 * k)
    assert np.abs(ho.dense() - A).max() < 1e-13 * np.abs(A).max()
    ho1, _, _ = hbs.compress(op, n, leaf, 2 * k - 1 + p, 5, rank=2 * k - 1)
    assert np.abs(ho1.dense() - A).max() > 1e-6 * np.abs(A).max()


def test_adaptive_sampling_grows_the_cap_until_ranks_are_revealed():
    """Adaptive sampling: a synthetic HBS operator of rank exactly 20,
    compressed in tolerance mode from a cap of 8 (r = 16): the revealed
    ranks saturate at caps 8 and 16 (no block of rank 20 fits), so the cap
    doubles twice; at 32 every node reveals rank exactly 20, E is at
    rounding level and the operator is recovered exactly."""
    n, leaf = 1024, 64
    hf = hbs.from_generators(W.synthetic_hbs(n, leaf, 20, seed=3))
    h, rounds = hbs.compress_adaptive(operators.HBSOp(hf), n, leaf, 8, 8, 7, 1e-10, 1e-10)
    assert [r[0] for r in rounds] == [8, 16, 32]
    assert [r[1] for r in rounds] == [True, True, False]
    assert rounds[0][2] > 1e-3 and rounds[-1][2] < 1e-13
    for t in range(2, 2 ** (h.tree.L + 1)):
        assert h.rank_u(t) == 20 and h.rank_v(t) == 20
    A = hf.dense()
    assert np.abs(h.dense() - A).max() < 1e-13 * np.abs(A).max()


def test_adaptive_sampling_stops_at_the_sample_limit():
    """When the cap reaches r_max - p with a node still saturated, the last
    compression is returned as it is (the caller is told)."""
    n, leaf = 1024, 64
    hf = hbs.from_generators(W.synthetic_hbs(n, leaf, 30, seed=4))
    h, rounds = hbs.compress_adaptive(operators.HBSOp(hf), n, leaf, 6, 8, 7, 1e-10, 1e-10,
                                      r_max=32)
    assert [r[0] for r in rounds] == [6, 12, 24]
    assert rounds[-1][1] is True


def test_dense_solve_of_the_represented_matrix():
    """The solver reference is the plain definition x = A_H^-1 b: its
    residual A_H x - b vanishes to rounding (relative to |A_H| |x|)."""
    n, leaf, k = 512, 64, 8
    h = hbs.from_generators(W.synthetic_hbs(n, leaf, k, seed=5))
    b = W.gaussian((n, 3), seed=1)
    x = hbs.solve(h, b)
    A = h.dense()
    res = np.linalg.norm(A @ x - b) / (np.linalg.norm(A) * np.linalg.norm(x))
    assert res < 1e-15
