"""GPU parity at the full size of the BF16 compression workload (N = 65536
points on the random-Fourier curve, near-singular kernel 1/(|x-y| + 1e-3),
leaf 128, k = 32, p = 16), in the launch configurations the benchmark times,
checked on sampled rows that the oracle computes one by one (kernel entries of
those rows against all N columns, FP64):

* the BF16 sampler on the benchmark's structured 96-column block (narrow
  form, K split in three) and on a 288-column block of three levels' test
  matrices (wide form), and the FP64 sampler;
* the compressed operator from BF16 and from FP64 sampling (Fig. 4 + Fig. 5),
  applied to Gaussian vectors: BF16 within its sampling precision, FP64
  within the k = 32 truncation error (2e-7 to 3.4e-7 on this workload).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import operators as oops

pytestmark = pytest.mark.gpu
hm = pytest.importorskip("paper_1503_07152_amd")

N, LEAF, K, P, DELTA = 65536, 128, 32, 16, 1e-3


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def workload():
    P_ = W.fourier_curve_points(N, seed=3)
    rows = np.sort(np.random.default_rng(0).choice(N, 128, replace=False))
    Arows = oops.KernelOp(P_, "near", DELTA).entries(rows, np.arange(N))   # 128 x N, FP64
    return P_, rows, Arows


def structured(c, nblocks, seed):
    """Level-structured test block: per 2r-column block b, the rows of the
    first half of each node at depth b+1 use the second half of the columns
    and vice versa (the [Omega_2 | Omega_1] pattern)."""
    X = W.gaussian((N, c), seed=seed)
    w = c // nblocks
    for b in range(nblocks):
        odd = (np.arange(N) // (N >> (b + 1))) % 2 == 1
        X[~odd, w * b + w // 2: w * (b + 1)] = 0.0
        X[odd, w * b: w * b + w // 2] = 0.0
    return X


def test_fullsize_samplers_on_sampled_rows(workload):
    P_, rows, Arows = workload
    print(f"full-size samplers N={N}", flush=True)
    for c, nb, dt, tol in ((96, 1, hm.HM_BF16, 8e-3), (288, 3, hm.HM_BF16, 8e-3),
                           (96, 1, hm.HM_F64, 1e-12)):
        X = structured(c, nb, seed=5 + c)
        op = hm.KernelOperator(P_, "near", DELTA, dt)
        Y = hm.hm_operator_apply(op, torch.from_numpy(X)).cpu().numpy()
        e = rel(Y[rows], Arows @ X)
        print(f"  c={c} dtype={dt}: sampled-row error {e:.2e}", flush=True)
        assert e < tol
        if c == 288:
            # the wide pass and narrow passes over its 96-column slices add the
            # same exact BF16 products in different FP32 orders
            for c0 in (0, 96, 192):
                Ys = hm.hm_operator_apply(
                    op, torch.from_numpy(np.ascontiguousarray(X[:, c0:c0 + 96]))).cpu().numpy()
                assert rel(Ys, Y[:, c0:c0 + 96]) < 1e-4


def test_fullsize_compress_on_sampled_rows(workload):
    P_, rows, Arows = workload
    w = W.gaussian((N, 4), seed=21)
    exact = Arows @ w
    for dt, tol in ((hm.HM_BF16, 5e-3), (hm.HM_F64, 1e-6)):
        print(f"full-size compress N={N} dtype={dt}", flush=True)
        h = hm.hbs_compress(hm.Options(N, LEAF, K, P, seed=3),
                            hm.KernelOperator(P_, "near", DELTA, dt))
        y = h.apply(torch.from_numpy(w)).cpu().numpy()
        e = rel(y[rows], exact)
        inf = h.info()
        print(f"  sampled-row error {e:.2e}, ranks {inf['min_rank']}..{inf['max_rank']}", flush=True)
        assert e < tol
        assert inf["min_rank"] == K and inf["max_rank"] == K
