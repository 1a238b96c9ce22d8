"""The apply that allocates nothing (hss_apply_noalloc), through the C ABI:
its output must equal hss_apply's on the same handle and input, on two calls
in a row, the second with a smaller input (the scratch array keeps the first
call's contents), and it must make no allocation through the library's
allocator hook."""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
hm = pytest.importorskip("paper_1503_07152_amd")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _call(h, x):
    y = hm.fortran(x.shape[0], x.shape[1], x.dtype)
    y.fill_(float("nan"))
    rc = hm.lib.hss_apply_noalloc(h.handle, x.shape[1], C.c_void_p(x.data_ptr()), x.shape[0],
                                  C.c_void_p(y.data_ptr()), y.shape[0],
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, hm.lib.hm_last_error().decode()
    return y


def test_noalloc_apply_equals_hss_apply_on_two_calls():
    calls = []

    def alloc(ctx, nbytes, stream):
        calls.append(nbytes)
        return None            # any allocation attempt would fail the call

    def free(ctx, ptr, stream):
        calls.append(-1)

    # first call: the apply benchmark's shape (FP32, N = 262144, k = 32, 64
    # right-hand sides; 2.1 MB of scratch per column, so several passes)
    n1, leaf1, k1 = 262144, 128, 32
    say(f"noalloc apply call 1: n={n1} k={k1} FP32, 64 columns")
    h1 = hm.hm_hbs_from_generators(W.synthetic_hbs(n1, leaf1, k1, seed=4), dtype=hm.HM_F32)
    x1 = hm.to_fortran(W.gaussian((n1, 64), seed=5), torch.float32)
    ref1 = hm.hss_apply(h1, x1)
    # second call: smaller (FP64, N = 1000, k = 12, 7 columns)
    n2, leaf2, k2 = 1000, 64, 12
    h2 = hm.hm_hbs_from_generators(W.synthetic_hbs(n2, leaf2, k2, seed=6))
    x2 = hm.to_fortran(W.gaussian((n2, 7), seed=7), torch.float64)
    ref2 = hm.hss_apply(h2, x2)
    torch.cuda.synchronize()
    hooks = (hm.ALLOC_FN(alloc), hm.FREE_FN(free))
    assert hm.lib.hm_set_allocator(hooks[0], hooks[1], None) == 0
    try:
        y1 = _call(h1, x1)
        say("noalloc apply call 2: n=1000 k=12 FP64, 7 columns")
        y2 = _call(h2, x2)
        torch.cuda.synchronize()
    finally:
        hm.lib.hm_set_allocator(hm.ALLOC_FN(), hm.FREE_FN(), None)
    assert calls == [], calls
    e1 = rel(y1.double().cpu().numpy(), ref1.double().cpu().numpy())
    e2 = rel(y2.cpu().numpy(), ref2.cpu().numpy())
    say(f"  noalloc vs hss_apply: {e1:.2e} (FP32, n={n1}), {e2:.2e} (FP64, n={n2})")
    assert e1 < 1e-6 and e2 < 1e-14
    # a third call, narrower than the passes of the first, on the same handle
    y3 = _call(h1, x1[:, :3])
    assert rel(y3.double().cpu().numpy(), ref1[:, :3].double().cpu().numpy()) < 1e-6


def test_noalloc_apply_rejects_bad_arguments():
    h = hm.hm_hbs_from_generators(W.synthetic_hbs(512, 64, 8, seed=1))
    x = hm.to_fortran(W.gaussian((512, 2), seed=1))
    y = hm.fortran(512, 2)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = hm.lib.hss_apply_noalloc(h.handle, 2, C.c_void_p(x.data_ptr()), 100,
                                  C.c_void_p(y.data_ptr()), 512, s)
    assert rc == -1 and b"ld" in hm.lib.hm_last_error()
    assert hm.lib.hss_apply_noalloc(None, 2, C.c_void_p(x.data_ptr()), 512,
                                    C.c_void_p(y.data_ptr()), 512, s) == -1


def test_noalloc_apply_replays_in_a_captured_graph():
    """The allocation-free apply captured in a HIP graph (torch.cuda.graph on
    its capture stream) and replayed three times, with new right-hand sides
    copied in and eager work between the replays: every replay equals the
    eager hss_apply of the same input."""
    n, leaf, k, c = 8192, 128, 32, 16
    h = hm.hm_hbs_from_generators(W.synthetic_hbs(n, leaf, k, seed=8))
    x = hm.fortran(n, c)
    y = hm.fortran(n, c)
    x.copy_(torch.from_numpy(W.gaussian((n, c), seed=1)))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        hm.hss_apply_noalloc(h, x, y, stream=torch.cuda.current_stream())
    for rep in range(3):
        xn = W.gaussian((n, c), seed=10 + rep)
        x.copy_(torch.from_numpy(xn))
        g.replay()
        torch.cuda.synchronize()
        want = hm.hss_apply(h, torch.from_numpy(xn)).cpu().numpy()
        _ = torch.ones(1000, device="cuda").sum().item()      # eager work between replays
        e = rel(y.cpu().numpy(), want)
        say(f"  graph replay {rep}: vs eager apply {e:.2e}")
        assert e < 1e-14
