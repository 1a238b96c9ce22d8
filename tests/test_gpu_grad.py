"""GPU checks of the backward of the compressed apply (hss_apply_backward
and the torch.autograd.Function built on it):

* every gradient equals the FP64 reference gradient of the oracle (a plain
  dense assembly of A_H differentiated by torch CPU autograd), to 1e-12;
* central finite differences of <gy, A_H x> through the GPU forward, along
  random directions of every input, to 1e-7 (FP64, N = 2048);
* gx equals hss_apply_adjoint(gy);
* the FP32 path against the FP64 reference, to 1e-5.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import grad as ograd

pytestmark = pytest.mark.gpu
hm = pytest.importorskip("paper_1503_07152_amd")

KEYS = ("U", "V", "Ut", "Vt", "B", "D")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def tensors(g, dtype=torch.float64):
    return {k: torch.from_numpy(np.ascontiguousarray(g[k])).to("cuda", dtype) for k in KEYS}


# (2048, 32, 32, 64/65): the shape of the benchmark's apply (k = 32, 64
# right-hand sides, one more for a ragged column tile) at L = 6 levels:
# two or three 32-column groups in the tree kernels and K-chunks in the
# gradient outer products
@pytest.mark.parametrize("n,leaf,k,c", [(2048, 128, 8, 3), (1000, 64, 6, 2), (2048, 32, 32, 64),
                                        (2048, 32, 32, 65)])
def test_backward_matches_reference_fp64(n, leaf, k, c):
    say(f"backward fp64 n={n} leaf={leaf} k={k} c={c}")
    g = W.synthetic_hbs(n, leaf, k, seed=3)
    x = W.gaussian((n, c), seed=4)
    gy = W.gaussian((n, c), seed=5)
    ref, yref = ograd.reference_gradients(g, x, gy)
    T = {kk: v.clone().requires_grad_(True) for kk, v in tensors(g).items()}
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    y = hm.hbs_apply(xt, T["U"], T["V"], T["Ut"], T["Vt"], T["B"], T["D"], n, leaf)
    assert rel(y.detach().cpu().numpy(), yref) < 1e-13
    y.backward(torch.from_numpy(gy).cuda())
    assert rel(xt.grad.cpu().numpy(), ref["x"]) < 1e-12
    L = g["L"]
    for kk in KEYS:
        got = T[kk].grad.cpu().numpy()
        want = ref[kk]
        if kk in ("Ut", "Vt"):        # only non-root, non-leaf blocks exist
            got, want = got[2:2 ** L], want[2:2 ** L]
        if kk == "B":
            got, want = got[2:], want[2:]
        if kk == "D":
            mask = g["D"] != 0
            got, want = got * mask, want * mask
        e = rel(got, want)
        say(f"  grad {kk}: {e:.2e}")
        assert e < 1e-12, kk
    # gx is the adjoint apply of gy
    h = hm.hm_hbs_from_generators(g)
    ga = hm.hss_apply_adjoint(h, torch.from_numpy(gy)).cpu().numpy()
    assert rel(xt.grad.cpu().numpy(), ga) < 1e-14


def test_finite_differences_fp64_n2048():
    n, leaf, k, c = 2048, 128, 8, 2
    say("finite differences n=2048")
    g = W.synthetic_hbs(n, leaf, k, seed=6)
    x = W.gaussian((n, c), seed=7)
    gy = torch.from_numpy(W.gaussian((n, c), seed=8)).cuda()
    T = tensors(g)
    h = hm.hbs_from_tensors(n, leaf, *[T[kk] for kk in KEYS])
    gx, grads = hm.hss_apply_backward(h, torch.from_numpy(x), gy)

    def f(TT, xx):
        hh = hm.hbs_from_tensors(n, leaf, *[TT[kk] for kk in KEYS])
        return float((gy * hm.hss_apply(hh, xx)).sum())

    rng = np.random.default_rng(0)
    hstep = 1e-6
    L = g["L"]
    for key in ("x",) + KEYS:
        base = x if key == "x" else g[key]
        d = rng.standard_normal(base.shape)
        if key in ("Ut", "Vt"):
            d[:2] = 0.0; d[2 ** L:] = 0.0
        if key == "B":
            d[:2] = 0.0
        if key == "D":
            d = d * (g["D"] != 0)
        def at(s):
            if key == "x":
                return f(T, torch.from_numpy(x + s * d).cuda())
            TT = dict(T)
            TT[key] = T[key] + s * torch.from_numpy(d).cuda()
            return f(TT, torch.from_numpy(x).cuda())
        fd = (at(hstep) - at(-hstep)) / (2 * hstep)
        gk = gx if key == "x" else grads[key]
        an = float((gk.cpu() * torch.from_numpy(d)).sum())
        say(f"  FD {key}: fd={fd:.10e} an={an:.10e}")
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), key


def test_backward_fp32_against_fp64_reference():
    n, leaf, k, c = 4096, 128, 16, 8
    say("backward fp32 n=4096")
    g = W.synthetic_hbs(n, leaf, k, seed=9)
    x = W.gaussian((n, c), seed=10)
    gy = W.gaussian((n, c), seed=11)
    h64 = hm.hm_hbs_from_generators(g)
    h32 = hm.hm_hbs_from_generators(g, dtype=hm.HM_F32)
    gx64, g64 = hm.hss_apply_backward(h64, torch.from_numpy(x), torch.from_numpy(gy))
    gx32, g32 = hm.hss_apply_backward(h32, torch.from_numpy(x.astype(np.float32)),
                                      torch.from_numpy(gy.astype(np.float32)))
    assert rel(gx32.double().cpu().numpy(), gx64.cpu().numpy()) < 1e-5
    for kk in KEYS:
        e = rel(g32[kk].double().cpu().numpy(), g64[kk].cpu().numpy())
        say(f"  fp32 grad {kk}: {e:.2e}")
        assert e < 1e-5, kk


def test_backward_fp32_full_size_against_oracle():
    """The benchmark's shape (synthetic HBS N = 262144, leaf 128, k = 32, 64
    FP32 right-hand sides, L = 11), checked where the oracle can follow at
    that size: gx = A_H^* gy against the oracle's FP64 adjoint apply (Fig. 7
    with U and V exchanged), and gD_t = gy_t x_t^T, the definition, entry by
    entry on every leaf."""
    from oracle import hbs as ohbs
    n, leaf, k, c = 262144, 128, 32, 64
    say(f"backward fp32 full size n={n} k={k} c={c}")
    g = W.synthetic_hbs(n, leaf, k, seed=4)
    x = W.gaussian((n, c), seed=5).astype(np.float32)
    gy = W.gaussian((n, c), seed=6).astype(np.float32)
    h = hm.hm_hbs_from_generators(g, dtype=hm.HM_F32)
    gx, gr = hm.hss_apply_backward(h, torch.from_numpy(x), torch.from_numpy(gy))
    gx = gx.double().cpu().numpy()
    ho = ohbs.from_generators(g)
    want = ho.apply_adjoint(gy.astype(np.float64))
    e = rel(gx, want)
    say(f"  gx vs oracle adjoint apply: {e:.2e}")
    assert e < 1e-5
    gD = gr["D"].double().cpu().numpy()
    worst = 0.0
    for t in ho.tree.leaves():
        I = ho.tree.I(t)
        m = ho.tree.size(t)
        ref = gy[I].astype(np.float64) @ x[I].astype(np.float64).T
        worst = max(worst, float(np.abs(gD[I, :m] - ref).max() / np.abs(ref).max()))
    say(f"  gD max entry error {worst:.2e}")
    assert worst < 1e-5


def test_backward_writes_every_output_entry():
    """The outputs need no initialisation: with every output prefilled with NaN,
    the blocks no node owns (gB of the root, gUt / gVt of the root and the
    leaves, block 0) and the D columns past a ragged leaf's size come back as
    exact zeros, and the owned entries equal those of a call on zeroed outputs."""
    n, leaf, k, c = 1000, 64, 6, 3
    say("backward writes every entry n=1000")
    g = W.synthetic_hbs(n, leaf, k, seed=9)
    h = hm.hm_hbs_from_generators(g)
    inf = h.info()
    R, L = inf["rank_pad"], inf["levels"]
    nn = 2 ** (L + 1)
    nmax = hm.HBS._nmax(n, leaf, L)
    x = hm.to_fortran(torch.from_numpy(W.gaussian((n, c), seed=1)))
    gy = hm.to_fortran(torch.from_numpy(W.gaussian((n, c), seed=2)))

    def run(fill):
        out = dict(gx=hm.fortran(n, c), U=hm.fortran(n, R), V=hm.fortran(n, R),
                   Ut=torch.empty((nn, R, 2 * R), dtype=torch.float64, device="cuda"),
                   Vt=torch.empty((nn, R, 2 * R), dtype=torch.float64, device="cuda"),
                   B=torch.empty((nn, R, R), dtype=torch.float64, device="cuda"),
                   D=hm.fortran(n, nmax))
        for t in out.values():
            t.fill_(fill)
        p = hm._ptr
        hm._check(hm.lib.hss_apply_backward(
            h.handle, c, p(x), hm._ld(x), p(gy), hm._ld(gy), p(out["gx"]), hm._ld(out["gx"]),
            p(out["U"]), p(out["V"]), p(out["Ut"]), p(out["Vt"]), p(out["B"]), p(out["D"]),
            hm._stream(None)))
        torch.cuda.synchronize()
        return {kk: v.cpu().numpy() for kk, v in out.items()}

    a, z = run(float("nan")), run(0.0)
    for kk in a:
        assert np.isfinite(a[kk]).all(), kk
        np.testing.assert_array_equal(a[kk], z[kk], err_msg=kk)
    for kk in ("Ut", "Vt"):
        assert not a[kk][:2].any() and not a[kk][2 ** L:].any(), kk
    assert not a["B"][:2].any()
