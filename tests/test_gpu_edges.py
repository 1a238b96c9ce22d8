"""Edge cases and failure handling of the HIP path, through the C ABI.

* degenerate trees: N <= leaf (L = 0: only D), one level, ragged N;
* a user callback operator (the paper's black box) gives the same result as
  the built-in dense operator;
* a failing callback -> HM_ERR_CALLBACK, NaN samples -> HM_ERR_NONFINITE,
  an operator of rank > r in tolerance mode -> HM_WARN_RANK_SATURATED
  (Sec. 2.5: the sample may have missed part of the block);
* the error estimate E of Sec. 5 on the GPU result stays at the tolerance.
All error conditions are produced on the host side of the operator (values or
return codes), never by a faulting kernel.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import hbs as ohbs
from oracle import metrics as ometrics
from oracle import operators as oops

pytestmark = pytest.mark.gpu
hm = pytest.importorskip("paper_1503_07152_amd")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n,leaf", [(100, 128), (128, 128), (200, 128), (1000, 64), (1023, 64)])
def test_degenerate_and_ragged_trees(n, leaf):
    print(f"tree n={n} leaf={leaf}", flush=True)
    k, p = 6, 6
    g = W.synthetic_hbs(n, leaf, k, seed=2) if n > leaf else None
    A = ohbs.from_generators(g).dense() if g else W.gaussian((n, n), seed=3)
    h = hm.hbs_compress(hm.Options(n, leaf, k, p, seed=4), hm.DenseOperator(A))
    ho, _, _ = ohbs.compress(oops.DenseOp(A), n, leaf, k + p, 4, rank=k)
    x = W.gaussian((n, 3), seed=5)
    y = h.apply(torch.from_numpy(x)).cpu().numpy()
    assert rel(y, A @ x) < 1e-12 and rel(y, ho.apply(x)) < 1e-12
    ya = h.apply(torch.from_numpy(x), adjoint=True).cpu().numpy()
    assert rel(ya, A.T @ x) < 1e-12


def test_callback_operator_matches_builtin():
    n, leaf, k, p = 1024, 64, 10, 8
    g = W.synthetic_hbs(n, leaf, k, seed=6)
    A = ohbs.from_generators(g).dense()
    At = torch.from_numpy(A).cuda()
    calls = []

    def matvec(adjoint, X, Y):
        calls.append(X.shape[1])
        Y.copy_((At.t() if adjoint else At) @ X)

    h1 = hm.hbs_compress(hm.Options(n, leaf, k, p, seed=9), hm.CallbackOperator(matvec))
    h2 = hm.hbs_compress(hm.Options(n, leaf, k, p, seed=9), hm.DenseOperator(A))
    x = W.gaussian((n, 3), seed=7)
    y1 = h1.apply(torch.from_numpy(x)).cpu().numpy()
    y2 = h2.apply(torch.from_numpy(x)).cpu().numpy()
    assert rel(y1, A @ x) < 1e-12 and rel(y1, y2) < 1e-12
    L = h1.info()["levels"]
    assert len(calls) == 2 * L + 1 and sum(calls) == h1.info()["sample_columns"]


@pytest.mark.parametrize("dt,tol", [(hm.HM_F32, 1e-5), (hm.HM_BF16, 5e-3)])
def test_callback_in_lower_precision_matches_oracle(dt, tol):
    """A user black box sampled in FP32 or BF16 (the callback receives its
    test block in that type and returns FP32 products): the orthonormal form
    (Fig. 4) must meet the accuracy of that sampling precision against the
    FP64 oracle, as the built-in kernel operator does."""
    n, leaf, k, p, seed = 2048, 128, 32, 16, 3
    P = W.fourier_curve_points(n, seed=3)
    K = oops.KernelOp(P, "near")
    A = torch.from_numpy(K.dense()).cuda()
    A32, A16 = A.float(), A.to(torch.bfloat16).float()
    seen = []

    def matvec(adjoint, X, Y):
        seen.append((X.dtype, Y.dtype))
        if X.dtype == torch.bfloat16:
            Y.copy_(A16 @ X.float())       # BF16 x BF16 products, FP32 sums
        else:
            Y.copy_(A32 @ X)

    h = hm.hbs_compress(hm.Options(n, leaf, k, p, seed=seed, orthonormal=True),
                        hm.CallbackOperator(matvec, dt))
    want = (torch.bfloat16 if dt == hm.HM_BF16 else torch.float32, torch.float32)
    assert seen and all(s_ == want for s_ in seen)
    ho, _, _ = ohbs.compress(K, n, leaf, k + p, seed, rank=k, to_id=False)
    x = W.gaussian((n, 8), seed=99)
    y = h.apply(torch.from_numpy(x)).cpu().numpy()
    e = rel(y, ho.apply(x))
    print(f"callback dtype {dt}: vs oracle {e:.2e}", flush=True)
    assert e < tol


def test_fp32_storage_and_conversion():
    """Factors computed in FP64 and stored in FP32 (store_dtype), and the
    conversion of a handle both ways: FP32 storage applies within FP32
    rounding of the FP64 form and of the exact operator."""
    n, leaf, k, p = 2048, 64, 12, 8
    g = W.synthetic_hbs(n, leaf, k, seed=2)
    op = hm.HBSOperator(hm.hm_hbs_from_generators(g))
    h64 = hm.hbs_compress(hm.Options(n, leaf, k, p, seed=4), op)
    h32 = hm.hbs_compress(hm.Options(n, leaf, k, p, seed=4, store_dtype=hm.HM_F32), op)
    assert h32.info()["dtype"] == hm.HM_F32 and h64.info()["dtype"] == hm.HM_F64
    x = W.gaussian((n, 4), seed=5)
    ya = ohbs.from_generators(g).apply(x)
    y64 = h64.apply(torch.from_numpy(x)).cpu().numpy()
    y32 = h32.apply(torch.from_numpy(x.astype(np.float32))).double().cpu().numpy()
    assert rel(y32, ya) < 1e-5 and rel(y32, y64) < 1e-5
    c32 = h64.convert(hm.HM_F32)
    yc = c32.apply(torch.from_numpy(x.astype(np.float32))).double().cpu().numpy()
    assert rel(yc, y32) < 1e-6
    back = c32.convert(hm.HM_F64)
    assert back.info()["dtype"] == hm.HM_F64
    assert rel(back.apply(torch.from_numpy(x)).cpu().numpy(), y64) < 1e-6
    e = c32.export()
    assert np.array_equal(e["skel_in"], h64.export()["skel_in"])
    with pytest.raises(hm.HMError):
        hm.hbs_compress(hm.Options(n, leaf, k, p, seed=4, store_dtype=7), op)


def test_failing_callback_reports_error():
    def bad(adjoint, X, Y):
        return 7
    with pytest.raises(hm.HMError) as e:
        hm.hbs_compress(hm.Options(512, 64, 8, 4, seed=1), hm.CallbackOperator(bad))
    assert e.value.code == -4


def test_nonfinite_samples_report_error():
    A = W.gaussian((512, 512), seed=1)
    A[10, 400] = np.nan
    with pytest.raises(hm.HMError) as e:
        hm.hbs_compress(hm.Options(512, 64, 8, 4, seed=1), hm.DenseOperator(A))
    assert e.value.code == -5


def test_nonfinite_kernel_points_report_error():
    # the near-singular kernel's samples are finite whenever its points are,
    # so the compression checks the points instead of every sample block: a
    # non-finite point must still end it with HM_ERR_NONFINITE (-5)
    n = 1024
    P = W.ellipse_points(n)
    P[300, 1] = np.inf
    pts = torch.from_numpy(P).cuda()
    for dt in (hm.HM_BF16, hm.HM_F64):
        op = hm.KernelOperator(pts, "near", 1e-3, dt)
        with pytest.raises(hm.HMError) as e:
            hm.hbs_compress(hm.Options(n, 64, 8, 4, seed=1), op)
        assert e.value.code == -5


def test_rank_saturation_warning():
    # a dense Gaussian matrix has full-rank off-diagonal blocks: at tol 1e-12
    # every block's revealed rank reaches the cap r - p
    n = 512
    A = W.gaussian((n, n), seed=2)
    h = hm.hbs_compress(hm.Options(n, 64, 12, 4, tol=1e-12, seed=3), hm.DenseOperator(A))
    assert h.status == hm.HM_WARN_RANK_SATURATED
    assert h.info()["saturated"] > 0
    hd = hm.hodlr_compress(hm.Options(n, 64, 12, 4, tol=1e-12, seed=3), hm.DenseOperator(A))
    assert hd.status == hm.HM_WARN_RANK_SATURATED


def test_error_estimate_E_at_tolerance():
    n, leaf, k, p, tol = 2048, 64, 40, 8, 1e-9
    P = W.ellipse_points(n)
    K = oops.KernelOp(P, "log")
    h = hm.hbs_compress(hm.Options(n, leaf, k, p, tol=tol, seed=5),
                        hm.KernelOperator(P, "log", 0.0, hm.HM_F64))
    E = ometrics.estimate_E(K.apply, lambda w: h.apply(torch.from_numpy(w)).cpu().numpy(), n)
    print(f"E = {E:.2e} (tol {tol}), ranks {h.info()['min_rank']}..{h.info()['max_rank']}")
    assert E < 10 * tol


def test_bf16_rank_deficient_blocks_fall_back_to_householder():
    """BF16 samples take the Gram-matrix node SVD; blocks whose leading r
    singular values it cannot resolve (here: two clusters of coincident
    points, every off-diagonal block exactly rank one after rounding) make the
    compression rerun on the Householder path, with the same accuracy as FP64
    sampling of the same operator."""
    n, leaf, k, p = 512, 64, 8, 4
    P = np.zeros((n, 2))
    P[n // 2:, 0] = 1.0
    K = oops.KernelOp(P, "near", 1e-3)
    x = W.gaussian((n, 3), seed=8)
    ref = K.apply(x)
    errs = {}
    for name, dt in (("bf16", hm.HM_BF16), ("f64", hm.HM_F64)):
        h = hm.hbs_compress(hm.Options(n, leaf, k, p, seed=3), hm.KernelOperator(P, "near", 1e-3, dt))
        y = h.apply(torch.from_numpy(x)).cpu().numpy()
        assert np.isfinite(y).all()
        errs[name] = rel(y, ref)
    print(f"errors {errs}")
    assert errs["f64"] < 1e-12 and errs["bf16"] < 5e-3


@pytest.mark.parametrize("case", ["synthetic", "log"])
def test_adaptive_sampling_matches_oracle(case):
    """Adaptive sampling (hbs_compress_adaptive) against the oracle's
    compress_adaptive on the same inputs and seeds: the same number of
    rounds (caps doubling while a node saturates or E > e_target), the same
    final ranks, and the same represented operator."""
    if case == "synthetic":
        n, leaf, k0, p, seed, tol, et = 2048, 64, 8, 8, 7, 1e-10, 1e-10
        g = W.synthetic_hbs(n, leaf, 20, seed=3)
        op = hm.HBSOperator(hm.hm_hbs_from_generators(g))
        oop = oops.HBSOp(ohbs.from_generators(g))
    else:
        n, leaf, k0, p, seed, tol, et = 1024, 64, 6, 8, 5, 1e-10, 1e-9
        P = W.ellipse_points(n)
        op = hm.KernelOperator(P, "log", 1e-3, hm.HM_F64)
        oop = oops.KernelOp(P, "log")
    h = hm.hbs_compress_adaptive(hm.Options(n, leaf, k0, p, tol=tol, seed=seed), op, et)
    ho, rounds = ohbs.compress_adaptive(oop, n, leaf, k0, p, seed, tol, et)
    inf = h.info()
    print(f"adaptive {case}: GPU rounds {inf['adapt_rounds']} E {inf['err_estimate']:.2e}; "
          f"oracle {rounds}", flush=True)
    assert h.status == 0
    assert inf["adapt_rounds"] == len(rounds)
    assert inf["err_estimate"] <= et
    e = h.export()
    for t in range(2, 2 ** (ho.tree.L + 1)):
        assert e["rank_u"][t] == ho.rank_u(t) and e["rank_v"][t] == ho.rank_v(t)
    x = W.gaussian((n, 8), seed=99)
    y = h.apply(torch.from_numpy(x)).cpu().numpy()
    assert rel(y, ho.apply(x)) < 1e-10
