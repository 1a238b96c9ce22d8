"""GPU parity of the HBS hot path against the CPU oracle, through the C ABI.

Every case uses the same seeded synthetic inputs and the same counter-based
test matrices on both sides.  Compressed representations are compared as the
operators they represent (factors are unique only up to rotations): densified
and compared entry by entry at N <= 4096, on Gaussian probes otherwise, plus
exact recovery where the input has off-diagonal rank exactly k.  The HBS-ID
output is also checked for the properties that define it (identity rows,
nested skeletons, B^skel = A(skel_in, skel_out)) and its skeletons against
the oracle's over the pivots the oracle decided by a clear margin.
Tolerances: FP64 1e-10 (or, where rounding decides the output, a stated
multiple of the oracle's own spread under sample noise), FP32 sampling 1e-5,
BF16 sampling 5e-3.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import hbs as ohbs
from oracle import operators as oops
from oracle import rng as orng

import parity_util as PU

pytestmark = pytest.mark.gpu

hm = pytest.importorskip("paper_1503_07152_amd")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("seed,level,phase,row0,nrows,ncols", [
    (0, 0, 0, 0, 1000, 7), (2 ** 40 + 5, 3, 0, 12345, 777, 48), (9, 2, 1, 0, 65, 1)])
def test_gauss_stream_matches_oracle(seed, level, phase, row0, nrows, ncols):
    say(f"gauss seed={seed} level={level} rows={row0}+{nrows} cols={ncols}")
    g = hm.hm_gauss(seed, level, phase, row0, nrows, ncols).cpu().numpy()
    ref = orng.gaussian_block(seed, level, np.arange(row0, row0 + nrows), ncols, phase)
    assert np.max(np.abs(g - ref) / (np.abs(ref) + 1e-300)) < 1e-14


@pytest.mark.parametrize("kernel,mode,n,c,tol", [
    ("near", hm.HM_F64, 1000, 96, 1e-13), ("log", hm.HM_F64, 777, 17, 1e-13),
    ("near", hm.HM_F32, 1000, 96, 2e-6), ("near", hm.HM_BF16, 1000, 96, 8e-3),
    ("near", hm.HM_F64, 300, 128, 1e-13), ("near", hm.HM_BF16, 1000, 192, 8e-3),
    ("log", hm.HM_BF16, 777, 288, 8e-3), ("near", hm.HM_BF16, 1500, 300, 8e-3),
    # K-split edges of the narrow BF16 form: 2 K-tiles (two parts), 1 K-tile
    # (no split), 3 K-tiles with a one-row last tile
    ("near", hm.HM_BF16, 100, 96, 8e-3), ("near", hm.HM_BF16, 50, 40, 8e-3),
    ("log", hm.HM_BF16, 129, 128, 8e-3)])
def test_kernel_sampler_matches_dense_product(kernel, mode, n, c, tol):
    say(f"sampler kernel={kernel} mode={mode} n={n} c={c}")
    P = W.fourier_curve_points(n, seed=3)
    K = oops.KernelOp(P, kernel)
    X = W.gaussian((n, c), seed=4)
    X[: n // 3, : c // 2] = 0.0            # zero blocks exercise the mask path
    op = hm.KernelOperator(P, kernel, 1e-3, mode)
    Y = hm.hm_operator_apply(op, torch.from_numpy(X)).cpu().numpy()
    ref = K.apply(X)
    assert rel(Y, ref) < tol


def test_bf16_wide_sampler_equals_column_slices():
    """The BF16 sampler holds up to 288 columns in one pass over the entries
    of A.  A wide call (one FP32 accumulator per element over all of K) and
    narrow calls on its slices (the K-tiles split in three, FP32 parts summed
    in FP64) add the same exact BF16 x BF16 products in different orders, so
    they agree to FP32 accumulation error: sqrt(n) u32 relative for random
    signs, bounded here at 2e-5 (n = 1111)."""
    n, c = 1111, 288
    say(f"wide bf16 sampler n={n} c={c}")
    P = W.fourier_curve_points(n, seed=5)
    X = W.gaussian((n, c), seed=6)
    X[: n // 2, 96:144] = 0.0
    X[n // 3:, 200:240] = 0.0
    op = hm.KernelOperator(P, "near", 1e-3, hm.HM_BF16)
    Y = hm.hm_operator_apply(op, torch.from_numpy(X)).cpu().numpy()
    for c0, c1 in ((0, 96), (96, 192), (192, 288), (48, 176)):
        Ys = hm.hm_operator_apply(op, torch.from_numpy(np.ascontiguousarray(X[:, c0:c1])))
        assert rel(Ys.cpu().numpy(), Y[:, c0:c1]) < 2e-5, (c0, c1)


def test_dense_operator_and_adjoint():
    say("dense operator n=513 c=40")
    r = np.random.default_rng(0)
    A = r.standard_normal((513, 513))
    X = r.standard_normal((513, 40))
    op = hm.DenseOperator(A)
    assert rel(hm.hm_operator_apply(op, torch.from_numpy(X)).cpu().numpy(), A @ X) < 1e-13
    assert rel(hm.hm_operator_apply(op, torch.from_numpy(X), adjoint=True).cpu().numpy(),
               A.T @ X) < 1e-13


@pytest.mark.parametrize("n,leaf,k", [(1024, 64, 10), (1000, 64, 12), (4096, 128, 32), (50, 64, 5)])
def test_apply_matches_oracle(n, leaf, k):
    say(f"apply n={n} leaf={leaf} k={k}")
    g = W.synthetic_hbs(n, leaf, k, seed=1)
    h = hm.hm_hbs_from_generators(g)
    ho = ohbs.from_generators(g)
    x = W.gaussian((n, 5), seed=2)
    y = h.apply(torch.from_numpy(x)).cpu().numpy()
    assert rel(y, ho.apply(x)) < 1e-13
    ya = h.apply(torch.from_numpy(x), adjoint=True).cpu().numpy()
    assert rel(ya, ho.apply_adjoint(x)) < 1e-13
    h32 = hm.hm_hbs_from_generators(g, dtype=hm.HM_F32)
    y32 = h32.apply(torch.from_numpy(x.astype(np.float32))).cpu().numpy()
    assert rel(y32, ho.apply(x)) < 1e-5


def _compare_compress(h, ho, n, A_apply=None, probes=8):
    x = W.gaussian((n, probes), seed=99)
    y = h.apply(torch.from_numpy(x)).cpu().numpy()
    yo = ho.apply(x)
    out = dict(vs_oracle=rel(y, yo))
    if A_apply is not None:
        out["vs_A"] = rel(y, A_apply(x))
    return out


def dense_gpu(h, n):
    """The represented operator densified on the device (N <= 4096)."""
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    return h.apply(eye).cpu().numpy()


@pytest.mark.parametrize("n,leaf,k,p,ortho", [
    (1024, 64, 10, 10, True), (1024, 64, 10, 10, False), (2000, 64, 12, 8, False),
    (4096, 128, 30, 10, False)])
def test_compress_synthetic_hbs_exact_recovery(n, leaf, k, p, ortho):
    say(f"compress synthetic n={n} leaf={leaf} k={k} p={p} ortho={ortho}")
    g = W.synthetic_hbs(n, leaf, k, seed=1)
    h_op = hm.hm_hbs_from_generators(g)
    seed = 11
    h = hm.hbs_compress(hm.Options(n, leaf, k, p, seed=seed, orthonormal=ortho),
                        hm.HBSOperator(h_op))
    ho_full = ohbs.from_generators(g)
    ho, st, ex = ohbs.compress(oops.HBSOp(ho_full), n, leaf, k + p, seed, rank=k, to_id=not ortho)
    # entry by entry: the GPU's represented operator, the oracle's and A
    A = ho_full.dense()
    Ag, Ao = dense_gpu(h, n), ho.dense()
    scale = np.abs(A).max()
    e_or, e_A = PU.max_rel(Ag, Ao, scale), PU.max_rel(Ag, A, scale)
    say(f"  max|GPU - oracle| = {e_or:.2e}, max|GPU - A| = {e_A:.2e} (of max|A|)")
    assert e_or < 1e-12 and e_A < 1e-12
    inf = h.info()
    assert inf["sample_columns"] == st.columns
    assert inf["operator_calls"] == 2 * ho.tree.L + 1
    if not ortho:
        e = h.export()
        L = ho.tree.L
        for t in range(2, 2 ** (L + 1)):
            assert e["rank_u"][t] == k and e["rank_v"][t] == k
        # HBS-ID structure on the GPU output: identity rows, nested
        # skeletons, B^skel = A(skel_in, skel_out) (eq. ben1)
        err = PU.hbs_id_structure(e, lambda r, c: A[np.ix_(r, c)])
        say(f"  max|B^skel - A(skel)| = {err:.2e} (of max|A(skel)|)")
        assert err < 1e-12


@pytest.mark.parametrize("kernel,n,leaf,k,p,tol", [
    ("log", 1024, 64, 40, 8, 1e-10), ("near", 2048, 64, 30, 10, 0.0),
    ("near", 4096, 128, 32, 16, 0.0)])
def test_compress_kernel_matches_oracle_fp64(kernel, n, leaf, k, p, tol):
    """FP64 parity on kernel operators, entry by entry on the densified
    operators.  Where the method's output is decided by rounding (pivots past
    the numerical rank of a fixed-rank ID, singular values near the cut), two
    correct runs differ by more than rounding; the bound is then the oracle's
    own spread: the largest change of its result when its samples carry
    relative noise of the size the GPU's FP64 sampler is held to (1e-13).
    Required: the 1e-10 target, or at most 3x that spread.  Skeletons must
    agree over every pivot the oracle decided by a margin above 1e-6."""
    say(f"compress kernel={kernel} n={n} k={k} p={p} tol={tol}")
    P = W.ellipse_points(n) if kernel == "log" else W.fourier_curve_points(n, seed=3)
    K = oops.KernelOp(P, kernel)
    seed = 5
    otol = tol if tol > 0 else None
    h = hm.hbs_compress(hm.Options(n, leaf, k, p, tol=tol, seed=seed),
                        hm.KernelOperator(P, kernel, 1e-3, hm.HM_F64))
    h2 = hm.hbs_compress(hm.Options(n, leaf, k, p, tol=tol, seed=seed, orthonormal=True),
                         hm.KernelOperator(P, kernel, 1e-3, hm.HM_F64))
    ho, _, ex = ohbs.compress(K, n, leaf, k + p, seed, rank=k, tol=otol)
    noisy = PU.oracle_spread(K, n, leaf, k + p, seed, k, otol, None)
    A = K.dense()
    scale = np.abs(A).max()
    Ao, Aoo = ho.dense(), ex["ortho"].dense()
    for name, hg, ref, alts in (("HBS-ID", h, Ao, [a.dense() for a, _ in noisy]),
                                ("orthonormal", h2, Aoo, [b.dense() for _, b in noisy])):
        Ag = dense_gpu(hg, n)
        gap = PU.max_rel(Ag, ref, scale)
        gap_f = rel(Ag, ref)
        spread = max(PU.max_rel(x, ref, scale) for x in alts)
        spread_f = max(rel(x, ref) for x in alts)
        acc_g, acc_o = rel(Ag, A), rel(ref, A)
        say(f"  {name}: GPU vs oracle max {gap:.2e} (Frobenius {gap_f:.2e}); oracle spread "
            f"max {spread:.2e} (Frobenius {spread_f:.2e}); vs A: GPU {acc_g:.2e}, oracle {acc_o:.2e}")
        assert gap_f < 1e-10 or (gap <= PU.SPREAD_FACTOR * spread
                                 and gap_f <= PU.SPREAD_FACTOR * spread_f)
    e = h.export()
    bad, cmp = PU.skeleton_prefix_mismatches(e, ho)
    agree = np.mean([set(e["skel_in"][t, :e["rank_u"][t]]) == set(ho.skel_in[t])
                     for t in range(2, 2 ** (ho.tree.L + 1))])
    say(f"  skeleton sets equal on {agree:.3f} of nodes; decided prefixes: {cmp - len(bad)}"
        f"/{cmp} equal {bad[:4]}")
    assert not bad
    err = PU.hbs_id_structure(e, K.entries)
    err_o = PU.oracle_bskel_error(ho, K.entries)
    say(f"  max|B^skel - A(skel)|: GPU {err:.2e}, oracle {err_o:.2e}")
    assert err <= max(10 * err_o, 1e-12)


# n = 4096 (L = 5): the block-identity product is split over the spare
# columns of four narrow second-product calls
@pytest.mark.parametrize("mode,tol,n", [(hm.HM_F64, 1e-10, 2048), (hm.HM_F32, 1e-5, 2048),
                                        (hm.HM_BF16, 5e-3, 2048), (hm.HM_BF16, 5e-3, 4096)])
def test_mixed_precision_sampling_errors(mode, tol, n):
    leaf, k, p, seed = 128, 32, 16, 3
    say(f"mixed precision mode={mode} n={n}")
    P = W.fourier_curve_points(n, seed=3)
    K = oops.KernelOp(P, "near")
    h = hm.hbs_compress(hm.Options(n, leaf, k, p, seed=seed, orthonormal=True),
                        hm.KernelOperator(P, "near", 1e-3, mode))
    ho, _, _ = ohbs.compress(K, n, leaf, k + p, seed, rank=k, to_id=False)
    r = _compare_compress(h, ho, n, K.apply)
    say(f"  {r}")
    assert r["vs_oracle"] < tol
    # BF16 kernel sampling puts the first products of G levels in one call,
    # those of the next levels into the second calls while they fit in 288
    # columns, and the block-identity product in the last level's second call
    L = ho.tree.L
    inf = h.info()
    if mode == hm.HM_BF16:
        r2, nmax = 2 * (k + p), ho.tree.nmax()
        calls, nxt = L, 0
        for lev in range(L):
            if nxt == lev:
                calls += 1
                nxt += min(288 // r2, L - lev)
            c2 = r2 + (nmax if lev == L - 1 else 0)
            nxt += min(L - nxt, (288 - c2) // r2)
        assert inf["operator_calls"] == calls
    else:
        assert inf["operator_calls"] == 2 * L + 1
    assert inf["sample_columns"] == 4 * (k + p) * L + ho.tree.nmax()


def test_low_memory_plan_matches_shared_calls():
    """HM_FLAG_LOW_MEMORY_PLAN takes the plan the compression falls back to
    when the shared sample windows would exceed 4 GiB: one operator call per
    product instead of first products riding in shared 288-column calls.  The
    test blocks are the same, so both reach the oracle's compression to the
    BF16 accuracy, with more operator calls."""
    n, leaf, k, p, seed = 4096, 128, 32, 16, 3
    say(f"low-memory plan n={n}")
    P = W.fourier_curve_points(n, seed=3)
    K = oops.KernelOp(P, "near")
    op = hm.KernelOperator(P, "near", 1e-3, hm.HM_BF16)
    h1 = hm.hbs_compress(hm.Options(n, leaf, k, p, seed=seed, orthonormal=True), op)
    h2 = hm.hbs_compress(hm.Options(n, leaf, k, p, seed=seed, orthonormal=True,
                                    low_memory_plan=True), op)
    ho, _, _ = ohbs.compress(K, n, leaf, k + p, seed, rank=k, to_id=False)
    L = ho.tree.L
    c1, c2 = h1.info()["operator_calls"], h2.info()["operator_calls"]
    say(f"  operator calls: shared {c1}, low-memory {c2}")
    assert c1 < c2 <= 2 * L + 1
    assert h2.info()["sample_columns"] == h1.info()["sample_columns"]
    for h in (h1, h2):
        r = _compare_compress(h, ho, n, K.apply)
        say(f"  {r}")
        assert r["vs_oracle"] < 5e-3


@pytest.mark.parametrize("n,leaf,k,p", [(3001, 100, 20, 8), (1537, 96, 30, 10)])
def test_bf16_gram_route_ragged_blocks(n, leaf, k, p):
    """BF16 kernel sampling takes the Gram route of the node SVD (node Gram
    matrices, pivoted Cholesky, Jacobi); sizes with node blocks of rows not a
    multiple of 32 and 2r = 56 or 80 columns (partial 16-column tiles of the
    Gram kernel) must reach the same BF16 accuracy against the oracle."""
    seed = 5
    say(f"bf16 gram route n={n} leaf={leaf} k={k} p={p}")
    P = W.fourier_curve_points(n, seed=7)
    K = oops.KernelOp(P, "near")
    h = hm.hbs_compress(hm.Options(n, leaf, k, p, seed=seed, orthonormal=True),
                        hm.KernelOperator(P, "near", 1e-3, hm.HM_BF16))
    ho, _, _ = ohbs.compress(K, n, leaf, k + p, seed, rank=k, to_id=False)
    r = _compare_compress(h, ho, n, K.apply)
    say(f"  {r}")
    assert r["vs_oracle"] < 5e-3


@pytest.mark.parametrize("n,leaf,k,p", [(1024, 64, 10, 10), (2000, 64, 12, 8)])
def test_orthonormal_bases_with_rank_deficient_blocks(n, leaf, k, p):
    """Node blocks of an operator with off-diagonal rank exactly k < r have
    numerical rank below r: the node factorisation reveals that rank and
    completes the r basis columns orthonormally (singular values 0), so the
    leaf bases of the orthonormal form (Fig. 4) stay orthonormal in all r
    columns, and the represented operator is still exact."""
    from oracle.tree import Tree
    say(f"orthonormal bases n={n} leaf={leaf} k={k} p={p}")
    g = W.synthetic_hbs(n, leaf, k, seed=4)
    h = hm.hbs_compress(hm.Options(n, leaf, k, p, seed=6, orthonormal=True),
                        hm.HBSOperator(hm.hm_hbs_from_generators(g)))
    e = h.export()
    r = k + p
    t = Tree(n, leaf)
    U, V = e["U"].cpu().numpy(), e["V"].cpu().numpy()
    worst = 0.0
    for lf in t.leaves():
        for B in (U[t.I(lf), :r], V[t.I(lf), :r]):
            worst = max(worst, np.abs(B.T @ B - np.eye(r)).max())
    say(f"  max |Q^T Q - I| = {worst:.1e}")
    assert worst < 1e-12
    ho_full = ohbs.from_generators(g)
    assert _compare_compress(h, ho_full, n, ho_full.apply)["vs_A"] < 1e-11


def _entries_from_apply(apply, n, rows, cols, chunk=1024):
    """A(rows, cols) of an operator known only through its products, one
    column chunk of the identity at a time; returns ``entries(r, c)`` over
    the given index sets."""
    rows = np.unique(rows)
    cols = np.unique(cols)
    sub = np.zeros((len(rows), len(cols)))
    for c0 in range(0, len(cols), chunk):
        cc = cols[c0:c0 + chunk]
        E = np.zeros((n, len(cc)))
        E[cc, np.arange(len(cc))] = 1.0
        sub[:, c0:c0 + len(cc)] = apply(E)[rows]
    ri = {int(r): i for i, r in enumerate(rows)}
    ci = {int(c): i for i, c in enumerate(cols)}
    return lambda r, c: sub[np.ix_([ri[int(x)] for x in r], [ci[int(x)] for x in c])]


@pytest.mark.timeout(600)
def test_synthetic_hbs_full_size_n16384():
    """The FP64 HBS workload at its full size: synthetic HBS of rank exactly
    k = 30 with nested bases (seed 1), N = 16384, leaf 64 (L = 8), p = 10.
    The GPU's HBS-ID form must equal the oracle's and A entry by entry on 8
    Gaussian probes to 1e-10 (relative to the largest entry), reveal rank
    exactly 30 at every node, and carry the HBS-ID structure (identity rows,
    nested skeletons, B^skel = A(skel_in, skel_out) on every sibling pair)."""
    n, leaf, k, p, seed = 16384, 64, 30, 10, 1
    say(f"synthetic HBS full size n={n} leaf={leaf} k={k} p={p}")
    g = W.synthetic_hbs(n, leaf, k, seed=1)
    h = hm.hbs_compress(hm.Options(n, leaf, k, p, seed=seed),
                        hm.HBSOperator(hm.hm_hbs_from_generators(g)))
    full = ohbs.from_generators(g)
    ho, st, _ = ohbs.compress(oops.HBSOp(full), n, leaf, k + p, seed, rank=k)
    x = W.gaussian((n, 8), seed=99)
    y = h.apply(torch.from_numpy(x)).cpu().numpy()
    yo, yA = ho.apply(x), full.apply(x)
    scale = np.abs(yA).max()
    e_or, e_A = PU.max_rel(y, yo, scale), PU.max_rel(y, yA, scale)
    say(f"  max entry error: vs oracle {e_or:.2e}, vs A {e_A:.2e}; Frobenius vs oracle "
        f"{rel(y, yo):.2e}")
    assert e_or < 1e-10 and e_A < 1e-10
    inf = h.info()
    assert inf["min_rank"] == k and inf["max_rank"] == k
    assert inf["sample_columns"] == st.columns == 4 * (k + p) * 8 + 64
    e = h.export()
    L = ho.tree.L
    leaves = range(2 ** L, 2 ** (L + 1))
    rows = np.concatenate([e["skel_in"][t, :k] for t in leaves])
    cols = np.concatenate([e["skel_out"][t, :k] for t in leaves])
    ent = _entries_from_apply(full.apply, n, rows, cols)
    err = PU.hbs_id_structure(e, ent)
    say(f"  max|B^skel - A(skel)| = {err:.2e}")
    assert err < 1e-11


@pytest.mark.parametrize("n,leaf,k,p", [(2048, 64, 8, 10), (1000, 64, 6, 8)])
def test_compress_hbs_product_matches_oracle(n, leaf, k, p):
    """Recompression of a product of two compressed operators (Sec. 5.2): the
    black box applies both GPU handles in turn; its HBS rank is 2k.  The
    GPU's HBS-ID form of the product equals the oracle's compression of the
    same product entry by entry and the dense product, with ranks 2k."""
    say(f"HBS product n={n} leaf={leaf} k={k} p={p}")
    g1, g2 = W.synthetic_hbs(n, leaf, k, seed=21), W.synthetic_hbs(n, leaf, k, seed=22)
    d1, d2 = hm.hm_hbs_from_generators(g1), hm.hm_hbs_from_generators(g2)
    seed, rk = 13, 2 * k
    h = hm.hbs_compress(hm.Options(n, leaf, rk, p, seed=seed), hm.HBSProductOperator(d1, d2))
    o1, o2 = ohbs.from_generators(g1), ohbs.from_generators(g2)
    A = o1.dense() @ o2.dense()
    ho, st, _ = ohbs.compress(oops.ProductOp(oops.HBSOp(o1), oops.HBSOp(o2)), n, leaf, rk + p,
                              seed, rank=rk)
    Ag, Ao = dense_gpu(h, n), ho.dense()
    scale = np.abs(A).max()
    e_or, e_A = PU.max_rel(Ag, Ao, scale), PU.max_rel(Ag, A, scale)
    say(f"  max|GPU - oracle| {e_or:.2e}, max|GPU - A| {e_A:.2e}")
    assert e_or < 1e-12 and e_A < 1e-12
    inf = h.info()
    assert inf["min_rank"] == rk and inf["max_rank"] == rk
    assert inf["sample_columns"] == st.columns
    # the product operator itself, both directions
    x = W.gaussian((n, 5), seed=3)
    op = hm.HBSProductOperator(d1, d2)
    assert rel(hm.hm_operator_apply(op, torch.from_numpy(x)).cpu().numpy(), A @ x) < 1e-13
    assert rel(hm.hm_operator_apply(op, torch.from_numpy(x), adjoint=True).cpu().numpy(),
               A.T @ x) < 1e-13


def test_autotune_picks_a_schedule_that_keeps_the_result():
    """The autotuner times every schedule of the BF16 kernel workload's
    shape (first products per call, later first products per second call,
    K-splits of the narrow sampler), keeps the fastest for later compressions
    of that shape, and the result stays within BF16 sampling accuracy of the
    oracle (the schedules differ only in the order of FP32 sums)."""
    n, leaf, k, p, seed = 4096, 128, 32, 16, 3
    P = W.fourier_curve_points(n, seed=3)
    op = hm.KernelOperator(P, "near", 1e-3, hm.HM_BF16)
    opts = hm.Options(n, leaf, k, p, seed=seed, orthonormal=True)
    try:
        t = hm.autotune(opts, op, reps=1)
        say(f"autotune: {t}")
        # defaults + (first-product groups 1-3) x (riding blocks 0-2) x (K-splits 1, 2, 3, 4, 8)
        assert t["candidates"] == 1 + 3 * 3 * 5
        assert t["t_best_ms"] <= t["t_default_ms"]
        assert 0 <= t["gfirst"] <= 3 and -1 <= t["ride"] <= 2 and t["ksplit"] in (0, 1, 2, 3, 4, 8)
        h = hm.hbs_compress(opts, op)
        ho, _, _ = ohbs.compress(oops.KernelOp(P, "near"), n, leaf, k + p, seed, rank=k,
                                 to_id=False)
        r = _compare_compress(h, ho, n)
        say(f"  tuned compress vs oracle {r['vs_oracle']:.2e}")
        assert r["vs_oracle"] < 5e-3
    finally:
        hm.autotune(opts, op, reps=0)      # back to the defaults for this shape
