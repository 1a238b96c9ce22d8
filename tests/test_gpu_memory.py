"""Memory interfaces of the C ABI on the GPU: zero-copy generator views
(hm_hbs_generators) and a caller's allocator (hm_set_allocator), here torch's
caching allocator.

* the views alias the handle's memory and hold the same values as the copying
  export, and keep the handle alive after its last Python reference is gone;
* compression, apply, backward and batched compression under the caller's
  allocator give the same results as under hipMalloc (same kernels, same
  inputs), their memory shows up in torch's pool while the handles live and
  goes back to it when they are freed.
"""
import gc

import numpy as np
import pytest
import torch

import workloads as W
from oracle import hbs as ohbs

pytestmark = pytest.mark.gpu
hm = pytest.importorskip("paper_1503_07152_amd")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_generator_views_alias_export():
    n, leaf, k, p = 2000, 64, 12, 8
    print(f"views n={n} leaf={leaf} k={k} p={p}", flush=True)
    g = W.synthetic_hbs(n, leaf, k, seed=3)
    h = hm.hbs_compress(hm.Options(n, leaf, k, p, seed=5),
                        hm.HBSOperator(hm.hm_hbs_from_generators(g)))
    v = h.generators()
    e = h.export()
    R, nodes = v["R"], v["nodes"]
    assert nodes == 2 ** (v["L"] + 1) - 1 and R == e["R"]
    for name in ("U", "V", "D"):
        assert torch.equal(v[name], e[name])
    for name in ("Ut", "Vt", "B"):
        assert v[name].shape[0] == nodes
        assert torch.equal(v[name], e[name][1:])
    # zero copy: the views are the handle's memory
    ptr = v["U"].data_ptr()
    assert hm.HBS.generators(h)["U"].data_ptr() == ptr
    x = torch.from_numpy(W.gaussian((n, 2), seed=4)).cuda()
    y = h.apply(x)
    # the views keep the handle alive
    U_sum = float(v["U"].sum())
    del h, e
    gc.collect()
    torch.cuda.synchronize()
    assert float(v["U"].sum()) == U_sum
    assert v["U"].data_ptr() == ptr
    A = ohbs.from_generators(g).dense()
    assert rel(y.cpu().numpy(), A @ x.cpu().numpy()) < 1e-11


def _run_all(g, n, leaf, k, p):
    """Compress, apply, adjoint apply, backward and batched compress."""
    h_op = hm.hm_hbs_from_generators(g)
    h = hm.hbs_compress(hm.Options(n, leaf, k, p, seed=7), hm.HBSOperator(h_op))
    x = torch.from_numpy(W.gaussian((n, 3), seed=8)).cuda()
    gy = torch.from_numpy(W.gaussian((n, 3), seed=9)).cuda()
    y = h.apply(x)
    ya = h.apply(x, adjoint=True)
    gx, gg = hm.hss_apply_backward(h, x, gy)
    hb = hm.hbs_compress_batched([hm.Options(n, leaf, k, p, seed=7)] * 2,
                                 [hm.HBSOperator(h_op)] * 2)
    yb = hb[1].apply(x)
    torch.cuda.synchronize()
    out = dict(y=y, ya=ya, gx=gx, gU=gg["U"], gB=gg["B"], yb=yb)
    return {kk: vv.cpu() for kk, vv in out.items()}, (h_op, h, hb)


def test_torch_caching_allocator_backs_library_memory():
    n, leaf, k, p = 2048, 64, 10, 6
    print(f"allocator n={n} leaf={leaf} k={k} p={p}", flush=True)
    g = W.synthetic_hbs(n, leaf, k, seed=2)
    ref, handles = _run_all(g, n, leaf, k, p)
    del handles
    gc.collect()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    try:
        hm.use_torch_allocator(True)
        got, handles = _run_all(g, n, leaf, k, p)
        held = torch.cuda.memory_allocated() - base
        # handle memory (at least U, V and D of the compressed matrix) sits in
        # torch's pool while the handles live
        assert held >= 3 * n * 8 * min(leaf, k + p)
        for kk in ref:
            assert torch.allclose(got[kk], ref[kk], rtol=1e-13, atol=1e-13 * float(ref[kk].abs().max())), kk
        del handles
        gc.collect()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() - base <= held // 4
    finally:
        hm.use_torch_allocator(False)
    # and back on hipMalloc
    again, handles = _run_all(g, n, leaf, k, p)
    for kk in ref:
        assert torch.allclose(again[kk], ref[kk], rtol=1e-13, atol=1e-13 * float(ref[kk].abs().max())), kk


def test_operator_apply_back_to_back_under_torch_allocator():
    """hm_operator_apply returns without waiting; its scratch (packed X, the
    K-split partial products) goes back to torch's pool on the stream, so calls
    enqueued back to back, each with fresh scratch, must all give the first
    call's result."""
    n, c = 3000, 96
    print(f"back-to-back operator applies n={n} c={c}", flush=True)
    P = W.fourier_curve_points(n, seed=8)
    X = torch.from_numpy(W.gaussian((n, c), seed=9)).cuda()
    try:
        hm.use_torch_allocator(True)
        op = hm.KernelOperator(P, "near", 1e-3, hm.HM_BF16)
        ys = [hm.hm_operator_apply(op, X) for _ in range(6)]
        torch.cuda.synchronize()
        for y in ys[1:]:
            assert torch.equal(y, ys[0])
    finally:
        hm.use_torch_allocator(False)
