"""Pins of the oracle's HBS direct solver (Gillman-Young-Martinsson
telescoping of the Woodbury formula): against the plain definition
x = A_H^-1 b (LAPACK LU of the densified matrix) on well-conditioned HBS
matrices, where any wrong term, transposition or index in E, F, G, Dh or the
sweeps shows at O(1); on the synthetic workload (diagonal blocks N(0,1) + 8 I,
some near singular) within the error growth the method is known to have."""
import numpy as np
import pytest

import workloads as W
from oracle import hbs, operators, solver


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _dominant(n, leaf, k, seed):
    """The synthetic generators with V = U, Vt = Ut and diagonal blocks
    20 I + N(0,1): every D block and every V^* D^-1 U (about I / 20) is well
    conditioned, so the solver's error stays at a few eps cond(A)."""
    g = W.synthetic_hbs(n, leaf, k, seed=seed)
    g["D"] = g["D"] + 12.0 * _eye_rows(g)
    g["V"], g["Vt"] = g["U"].copy(), g["Ut"].copy()
    return g


def _eye_rows(g):
    n, nmax = g["D"].shape
    L, lo, hi = W.operator_partition(n, g["leaf"])
    e = np.zeros_like(g["D"])
    for t in range(2 ** L, 2 ** (L + 1)):
        m = hi[t] - lo[t]
        e[lo[t]:hi[t], :m] = np.eye(m)
    return e


@pytest.mark.parametrize("n,leaf,k", [(256, 32, 4), (1000, 64, 6), (2048, 64, 12)])
def test_solver_equals_dense_solve_when_well_conditioned(n, leaf, k):
    h = hbs.from_generators(_dominant(n, leaf, k, seed=4))
    b = W.gaussian((n, 3), seed=2)
    x = solver.Factor(h).solve(b)
    xd = hbs.solve(h, b)
    assert rel(x, xd) < 1e-13


def test_single_level_is_block_woodbury():
    """L = 1: A = diag(D2, D3) + [[0, U2 B23 V3^*], [U3 B32 V2^*, 0]];
    the solver's answer is the dense solve."""
    g = _dominant(128, 64, 5, seed=1)
    h = hbs.from_generators(g)
    assert h.tree.L == 1
    b = W.gaussian((128, 2), seed=3)
    assert rel(solver.Factor(h).solve(b), hbs.solve(h, b)) < 1e-14


def test_solver_on_compressed_kernel_matrix():
    n = 1024
    op = operators.KernelOp(W.fourier_curve_points(n, seed=3), "near", 1e-3)
    h, _, _ = hbs.compress(op, n, 64, 30, 5, rank=20)
    b = W.gaussian((n, 2), seed=1)
    assert rel(solver.Factor(h).solve(b), hbs.solve(h, b)) < 1e-13


def test_solver_on_the_synthetic_workload_within_its_error_growth():
    h = hbs.from_generators(W.synthetic_hbs(1024, 64, 10, seed=5))
    b = W.gaussian((1024, 3), seed=7)
    x, xd = solver.Factor(h).solve(b), hbs.solve(h, b)
    cond = np.linalg.cond(h.dense())
    # the formulas invert D and V^* D^-1 U without pivoting across levels:
    # the error grows past cond(A) eps (here by about 50x), never to O(1)
    assert rel(x, xd) < 1e3 * cond * np.finfo(float).eps


def test_solver_rejects_mixed_ranks():
    op = operators.KernelOp(W.fourier_curve_points(512, seed=3), "log", 0.0)
    h, _, _ = hbs.compress(op, 512, 64, 40, 5, tol=1e-8)
    if len({h.rank_u(t) for t in range(2, 2 ** (h.tree.L + 1))}) > 1:
        with pytest.raises(ValueError):
            solver.Factor(h)
