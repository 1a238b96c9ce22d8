"""Pins of the oracle's black-box operators and of the pivot margins its ID
reports, against values fixed by hand:

* the near-singular kernel ``1/(|x - y| + delta)`` and the log kernel
  ``log|x - y|`` (1 on the diagonal) on points whose distances are exact
  (a 3-4-5 right triangle), and the diagonal of the near kernel, 1/delta;
* the tiled (and threaded) kernel product against a brute-force double loop;
* the noisy operator used to measure the method's own rounding spread stays
  within its stated relative amplitude;
* the pivot margins of the column-pivoted QR on a diagonal matrix, whose
  residual column norms are its diagonal entries.
"""
import math

import numpy as np

from oracle import lowrank
from oracle import operators as oops

# (0,0), (3,0), (3,4): distances 3, 4 and 5 exactly
TRI = np.array([[0.0, 0.0], [3.0, 0.0], [3.0, 4.0]])


def test_near_kernel_entries_by_hand():
    K = oops.KernelOp(TRI, "near", delta=1e-3)
    A = K.dense()
    # 1/(d + 1/1000) = 1000 / (1000 d + 1)
    want = np.array([[1000.0, 1000 / 3001, 1000 / 5001],
                     [1000 / 3001, 1000.0, 1000 / 4001],
                     [1000 / 5001, 1000 / 4001, 1000.0]])
    # FP64 evaluation of 1/(d + delta) rounds twice (the sum, then the
    # quotient): within two units in the last place of the exact rational
    np.testing.assert_allclose(A, want, rtol=4.5e-16, atol=0)
    assert abs(A[0, 2] - 0.19996000799840032) < 6e-17   # 1000/5001 to 17 digits


def test_log_kernel_entries_by_hand():
    K = oops.KernelOp(TRI, "log")
    A = K.dense()
    ln3, ln4, ln5 = 1.0986122886681098, 1.3862943611198906, 1.6094379124341003
    want = np.array([[1.0, ln3, ln5], [ln3, 1.0, ln4], [ln5, ln4, 1.0]])
    np.testing.assert_allclose(A, want, rtol=2.3e-16, atol=0)
    # unit distance: log 1 = 0 exactly
    assert oops.KernelOp(np.array([[0.0, 0.0], [0.6, 0.8]]), "log").dense()[0, 1] == 0.0


def test_kernel_entries_on_index_subsets():
    K = oops.KernelOp(TRI, "near")
    sub = K.entries(np.array([2, 0]), np.array([1]))
    assert sub.shape == (2, 1)
    np.testing.assert_allclose(sub[:, 0], [1000 / 4001, 1000 / 3001], rtol=4.5e-16, atol=0)


def test_kernel_apply_equals_brute_force():
    r = np.random.default_rng(1)
    pts = r.standard_normal((37, 2))
    X = r.standard_normal((37, 3))
    for kind in ("near", "log"):
        want = np.zeros((37, 3))
        for i in range(37):
            for j in range(37):
                d = math.hypot(pts[i, 0] - pts[j, 0], pts[i, 1] - pts[j, 1])
                if kind == "near":
                    a = 1.0 / (d + 1e-3)
                else:
                    a = 1.0 if i == j else math.log(d)
                want[i] += a * X[j]
        for tile, workers in ((512, 1), (5, 1), (5, 4)):
            got = oops.KernelOp(pts, kind, tile=tile, workers=workers).apply(X)
            np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)


def test_threaded_apply_is_bitwise_the_serial_one():
    r = np.random.default_rng(2)
    pts = r.standard_normal((300, 2))
    X = r.standard_normal((300, 7))
    a = oops.KernelOp(pts, "near", tile=64).apply(X)
    b = oops.KernelOp(pts, "near", tile=64, workers=3).apply(X)
    assert np.array_equal(a, b)


def test_perturbed_operator_amplitude():
    r = np.random.default_rng(3)
    A = r.standard_normal((200, 200))
    X = r.standard_normal((200, 5))
    op = oops.PerturbedOp(oops.DenseOp(A), 1e-13, seed=4)
    for got, exact in ((op.apply(X), A @ X), (op.apply_adjoint(X), A.T @ X)):
        d = got / exact - 1.0
        assert np.abs(d).max() <= 1e-13 * (1 + 1e-3)
        assert np.abs(d).max() > 0.5e-13          # the noise is really there
        assert abs(d.mean()) < 1e-14              # and centred


def test_cpqr_pivot_margins_on_a_diagonal_matrix():
    M = np.diag([2.9, 5.0, 1.0, 3.0])
    gaps = []
    perm, k, R = lowrank.cpqr(M, 4, None, gaps)
    assert list(perm) == [1, 3, 0, 2] and k == 4
    # residual norms are the diagonal entries; margins relative to |R_11| = 5
    np.testing.assert_allclose(gaps, [(5 - 3) / 5, (3 - 2.9) / 5, (2.9 - 1) / 5, 0.0],
                               rtol=1e-15, atol=1e-16)
