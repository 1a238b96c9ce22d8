"""Pins of the oracle's HODLR path (Fig. 2) and of the reference gradient.

* exact recovery of the synthetic HODLR of rank exactly 10, revealed ranks 10;
* the SVD variant (eq. SVDtogetV) gives diagonal B equal to the leading
  singular values of each sibling block (Eckart-Young, Sec. 2.3);
* log kernel at tol 1e-10 meets the tolerance and the estimate E (Sec. 5);
* HODLR storage per index grows with log N (Sec. 3.1, eq. T_HODLR) while
  the column count of Fig. 2 is 4 r L + n_max;
* the reference gradient matches central finite differences.
"""
import numpy as np
import pytest

import workloads as W
from oracle import grad, hodlr, metrics, operators
from oracle.tree import Tree


@pytest.fixture(scope="module")
def syn():
    return W.synthetic_hodlr_dense(1024, 64, 10, seed=0)


def test_exact_recovery_and_ranks(syn):
    h, st = hodlr.compress(operators.DenseOp(syn), 1024, 64, r=20, seed=2, tol=1e-10)
    assert metrics.rel_fro(h.dense(), syn) < 1e-12
    assert set(h.ranks().values()) == {10}
    assert st.columns == 4 * 20 * h.tree.L + h.tree.nmax()


def test_svd_variant_b_is_singular_values(syn):
    h, _ = hodlr.compress(operators.DenseOp(syn), 1024, 64, r=20, seed=3, rank=10)
    tree = h.tree
    for lev in range(1, tree.L + 1):
        for t in tree.level_nodes(lev - 1):
            a, b = tree.children(t)
            s = np.linalg.svd(syn[tree.I(a), tree.I(b)], compute_uv=False)[:10]
            assert np.allclose(np.diag(h.B[(a, b)]), s, rtol=1e-11)
            assert np.allclose(h.B[(a, b)], np.diag(np.diag(h.B[(a, b)])))


def test_log_kernel_tolerance():
    P = W.ellipse_points(1024)
    K = operators.KernelOp(P, "log")
    h, _ = hodlr.compress(K, 1024, 64, r=50, seed=4, tol=1e-10)
    A = K.dense()
    assert metrics.rel_fro(h.dense(), A) < 1e-9
    assert metrics.estimate_E(K.apply, h.apply, 1024) < 1e-9
    assert max(h.ranks().values()) < 50 - 5     # not saturated: r - p headroom


def test_storage_grows_like_log_n():
    per = []
    for n in (512, 1024, 2048):
        A = W.synthetic_hodlr_dense(n, 64, 6, seed=1)
        h, _ = hodlr.compress(operators.DenseOp(A), n, 64, r=12, seed=1, rank=6)
        per.append((h.storage_reals() - n * 64) / n)     # off-diagonal part
    # U and V of k columns on each of L levels: 2 k L per index.
    Ls = [Tree(n, 64).L for n in (512, 1024, 2048)]
    assert np.allclose(per, [2 * 6 * L + 6 * (2 ** (L + 1) - 2) / n for L, n in zip(Ls, (512, 1024, 2048))], rtol=1e-12)


def test_reference_gradient_finite_differences():
    g = W.synthetic_hbs(256, 32, 4, seed=3)
    x = W.gaussian((256, 2), seed=4)
    gy = W.gaussian((256, 2), seed=5)
    grads, y = grad.reference_gradients(g, x, gy)
    tree = Tree(256, 32)
    import torch
    def f(gg, xx):
        T = {k: torch.tensor(gg[k]) for k in ("U", "V", "Ut", "Vt", "B", "D")}
        A = grad.dense_from_generators(tree, **T).numpy()
        return float(np.sum(gy * (A @ xx)))
    rng = np.random.default_rng(0)
    h = 1e-6
    for key in ("x", "U", "V", "Ut", "Vt", "B", "D"):
        base = x if key == "x" else g[key]
        d = rng.standard_normal(base.shape)
        if key in ("Ut", "Vt"):
            d[:2] = 0.0; d[2 ** tree.L:] = 0.0       # only non-root, non-leaf nodes exist
        if key == "B":
            d[:2] = 0.0
        if key == "D":
            d = d * (g["D"] != 0)
        def shifted(s):
            if key == "x":
                return f(g, x + s * d)
            gg = dict(g); gg[key] = g[key] + s * d
            return f(gg, x)
        fd = (shifted(h) - shifted(-h)) / (2 * h)
        an = float(np.sum(grads[key] * d))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), key
