"""GPU parity of the batched many-instance compression: uneven instances
(sizes, ranks, depths) compressed in one level-synchronous pass must each
equal the oracle's compression of that instance alone (same seed, same test
matrices) and recover their exact-rank operator."""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import hbs as ohbs
from oracle import operators as oops

pytestmark = pytest.mark.gpu
hm = pytest.importorskip("paper_1503_07152_amd")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("ortho", [False, True])
def test_batched_matches_per_instance_oracle(ortho):
    specs = [(640, 8), (1280, 12), (2112, 20), (576, 16), (1024, 10), (4096, 30), (128, 6)]
    leaf, p = 128, 8
    print(f"batched {len(specs)} instances ortho={ortho}", flush=True)
    gens = [W.synthetic_hbs(n, leaf, k, seed=100 + i) for i, (n, k) in enumerate(specs)]
    ops_h = [hm.hm_hbs_from_generators(g) for g in gens]
    opts = [hm.Options(n, leaf, k, p, seed=7 + i, orthonormal=ortho)
            for i, (n, k) in enumerate(specs)]
    outs = hm.hbs_compress_batched(opts, [hm.HBSOperator(h) for h in ops_h])
    for i, ((n, k), g, h) in enumerate(zip(specs, gens, outs)):
        full = ohbs.from_generators(g)
        ho, st, _ = ohbs.compress(oops.HBSOp(full), n, leaf, k + p, 7 + i, rank=k, to_id=not ortho)
        x = W.gaussian((n, 4), seed=3)
        y = h.apply(torch.from_numpy(x)).cpu().numpy()
        e_or, e_a = rel(y, ho.apply(x)), rel(y, full.apply(x))
        print(f"  instance {i} n={n} k={k}: vs oracle {e_or:.2e} vs A {e_a:.2e}", flush=True)
        assert e_or < 1e-11 and e_a < 1e-11
        assert h.info()["sample_columns"] == st.columns


def test_batched_bf16_kernel_uneven_depths():
    """Built-in kernel operators sampled in BF16 over a forest whose instances
    have different depths: the first products of several levels share calls
    (instances that stop peeling earlier get zero test blocks), and the
    block-identity product keeps its own call.  Each instance must reach the
    BF16 accuracy of its single-instance compression."""
    specs = [(2048, 3), (512, 5), (1024, 7)]
    leaf, k, p = 128, 16, 8
    print(f"batched bf16 kernel {len(specs)} instances", flush=True)
    pts = [W.fourier_curve_points(n, seed=s) for n, s in specs]
    mk = lambda P: hm.KernelOperator(P, "near", 1e-3, hm.HM_BF16)
    opts = [hm.Options(n, leaf, k, p, seed=11 + i) for i, (n, _) in enumerate(specs)]
    outs = hm.hbs_compress_batched(opts, [mk(P) for P in pts])
    for i, ((n, _), P, h) in enumerate(zip(specs, pts, outs)):
        K = oops.KernelOp(P, "near", 1e-3)
        x = W.gaussian((n, 3), seed=5)
        ref = K.apply(x)
        e_b = rel(h.apply(torch.from_numpy(x)).cpu().numpy(), ref)
        h1 = hm.hbs_compress(opts[i], mk(P))
        e_1 = rel(h1.apply(torch.from_numpy(x)).cpu().numpy(), ref)
        print(f"  instance {i} n={n}: batched {e_b:.2e} single {e_1:.2e}", flush=True)
        assert e_b < 1e-2 and e_b < 1.5 * e_1 + 1e-4


def test_batched_bf16_kernel_equal_depths():
    """Built-in kernel operators sampled in BF16 over a forest of instances of
    one depth (n = 4096, L = 5, r = 48): the second products carry first
    products of later levels, and the block-identity product is split over
    the spare columns of the narrow second-product calls.  Each instance must
    reach the BF16 accuracy of its single-instance compression."""
    n, leaf, k, p = 4096, 128, 32, 16
    seeds = [3, 8, 13]
    print(f"batched bf16 kernel {len(seeds)} instances n={n}", flush=True)
    pts = [W.fourier_curve_points(n, seed=s) for s in seeds]
    mk = lambda P: hm.KernelOperator(P, "near", 1e-3, hm.HM_BF16)
    opts = [hm.Options(n, leaf, k, p, seed=21 + i) for i in range(len(seeds))]
    outs = hm.hbs_compress_batched(opts, [mk(P) for P in pts])
    for i, (P, h) in enumerate(zip(pts, outs)):
        K = oops.KernelOp(P, "near", 1e-3)
        x = W.gaussian((n, 3), seed=5)
        ref = K.apply(x)
        e_b = rel(h.apply(torch.from_numpy(x)).cpu().numpy(), ref)
        h1 = hm.hbs_compress(opts[i], mk(P))
        e_1 = rel(h1.apply(torch.from_numpy(x)).cpu().numpy(), ref)
        print(f"  instance {i}: batched {e_b:.2e} single {e_1:.2e}", flush=True)
        assert e_b < 1e-2 and e_b < 1.5 * e_1 + 1e-4


def c3_oversample(k, r_max=48):
    """Oversampling of a batch instance: 10 where k + 10 fits the library's
    sample limit r <= 48, else 48 - k (k = 39, 40)."""
    return min(10, r_max - k)


@pytest.mark.timeout(600)
def test_batched_c3_instances_match_oracle():
    """The first 32 instances of the uneven batch (N log-uniform in
    [512, 8192] in multiples of 64, k uniform in 8..40, leaf 128, seed 2),
    compressed together: every instance equals the oracle's compression of it
    alone and recovers its exact-rank operator, with revealed ranks exactly
    k at every node."""
    specs = W.batched_instances(256, seed=2)[:32]
    leaf = 128
    print(f"batched C3 subset: {len(specs)} instances, total N {sum(n for n, _ in specs)}",
          flush=True)
    gens = [W.synthetic_hbs(n, leaf, k, seed=1000 + i) for i, (n, k) in enumerate(specs)]
    ops_h = [hm.hm_hbs_from_generators(g) for g in gens]
    opts = [hm.Options(n, leaf, k, c3_oversample(k), seed=2000 + i)
            for i, (n, k) in enumerate(specs)]
    outs = hm.hbs_compress_batched(opts, [hm.HBSOperator(h) for h in ops_h])
    worst_or, worst_a = 0.0, 0.0
    for i, ((n, k), g, h) in enumerate(zip(specs, gens, outs)):
        full = ohbs.from_generators(g)
        ho, st, _ = ohbs.compress(oops.HBSOp(full), n, leaf, k + c3_oversample(k), 2000 + i,
                                  rank=k)
        x = W.gaussian((n, 4), seed=3)
        y = h.apply(torch.from_numpy(x)).cpu().numpy()
        e_or, e_a = rel(y, ho.apply(x)), rel(y, full.apply(x))
        worst_or, worst_a = max(worst_or, e_or), max(worst_a, e_a)
        assert e_or < 1e-11 and e_a < 1e-11, (i, n, k, e_or, e_a)
        inf = h.info()
        assert inf["sample_columns"] == st.columns
        assert inf["min_rank"] == k and inf["max_rank"] == k
    print(f"  worst: vs oracle {worst_or:.2e}, vs A {worst_a:.2e}", flush=True)
    # FP32 storage of the same batch: factors computed in FP64, stored and
    # applied in FP32, within 1e-5 of the oracle
    opts32 = [hm.Options(n, leaf, k, c3_oversample(k), seed=2000 + i, store_dtype=hm.HM_F32)
              for i, (n, k) in enumerate(specs)]
    outs32 = hm.hbs_compress_batched(opts32, [hm.HBSOperator(h) for h in ops_h])
    worst32 = 0.0
    for i, ((n, k), g, h) in enumerate(zip(specs, gens, outs32)):
        assert h.info()["dtype"] == hm.HM_F32
        x = W.gaussian((n, 4), seed=3)
        y = h.apply(torch.from_numpy(x.astype(np.float32))).double().cpu().numpy()
        worst32 = max(worst32, rel(y, ohbs.from_generators(g).apply(x)))
    print(f"  FP32 storage: worst vs A {worst32:.2e}", flush=True)
    assert worst32 < 1e-5


def test_persistent_id_sweep_equals_level_synchronous():
    """The Fig. 5 sweep as one persistent launch over every level, side and
    instance (HM_FLAG_PERSISTENT_ID: work items taken from a device counter,
    a parent after both its children) and level by level (the default, one
    launch per level and side): on exact-rank instances of the uneven batch
    both give the same ranks and the same represented operators, each equal
    to the operator itself."""
    specs = W.batched_instances(256, seed=2)[:16]
    leaf = 128
    print(f"persistent vs level-synchronous ID sweep, {len(specs)} instances", flush=True)
    gens = [W.synthetic_hbs(n, leaf, k, seed=3000 + i) for i, (n, k) in enumerate(specs)]
    ops_h = [hm.hm_hbs_from_generators(g) for g in gens]
    mk = lambda pers: [hm.Options(n, leaf, k, c3_oversample(k), seed=4000 + i, persistent_id=pers)
                       for i, (n, k) in enumerate(specs)]
    outs_p = hm.hbs_compress_batched(mk(True), [hm.HBSOperator(h) for h in ops_h])
    outs_l = hm.hbs_compress_batched(mk(False), [hm.HBSOperator(h) for h in ops_h])
    worst = 0.0
    for (n, k), g, hp, hl in zip(specs, gens, outs_p, outs_l):
        ep, el = hp.export(), hl.export()
        assert np.array_equal(ep["rank_u"], el["rank_u"]) and np.array_equal(ep["rank_v"], el["rank_v"])
        x = W.gaussian((n, 4), seed=3)
        yp = hp.apply(torch.from_numpy(x)).cpu().numpy()
        yl = hl.apply(torch.from_numpy(x)).cpu().numpy()
        ya = ohbs.from_generators(g).apply(x)
        worst = max(worst, rel(yp, yl))
        assert rel(yp, ya) < 1e-11 and rel(yl, ya) < 1e-11
    print(f"  worst persistent vs level-synchronous: {worst:.2e}", flush=True)
    assert worst < 1e-12
