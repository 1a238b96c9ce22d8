"""GPU parity of the frontal-matrix black box of nested dissection (Sec. 5.4)
against the oracle (SciPy sparse LU solves with B11 and B22), through the C
ABI: element by element on grids from one row to several thousand, ragged
reduction levels, the narrowest and widest supported strips, column counts
across the kernels' chunk and pass boundaries; the full 102400-row grid on
every row of four columns; and the HODLR / HBS-ID compressions of the
operator (ε = 1e-9, ℓ = 25 as in Tables 8 and 9) against the oracle's.

Tolerance: both sides solve B11 and B22 in FP64 with different elimination
orders (block cyclic reduction against SuperLU's), so they agree to the
rounding of a solve with cond(B11) <= 1e4 here: 1e-11 relative."""
import sys

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import frontal as ofr
from oracle import hbs as ohbs
from oracle import hodlr as ohodlr

pytestmark = pytest.mark.gpu
hm = pytest.importorskip("paper_1503_07152_amd")

TOL = 1e-11


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _apply(f, X):
    return f.apply(torch.from_numpy(X).cuda()).cpu().numpy()


@pytest.mark.parametrize("H,W,m", [
    (1, 41, 3),        # a single row: A = 0
    (2, 41, 5),        # one reduction level
    (3, 5, 1),
    (37, 41, 7),       # ragged levels (37 -> 19 -> 10 -> 5 -> 3 -> 2 -> 1)
    (257, 41, 50),
    (1000, 41, 103),   # past one chunk of the step kernel (102 columns)
    (300, 3, 9),       # one column per side
    (129, 65, 60),     # the widest sides (32 columns; 50-column chunks)
    (513, 41, 130),    # two passes of 128 columns
])
def test_frontal_apply_matches_oracle(H, W, m):
    say(f"frontal apply H={H} W={W} m={m}")
    ch, cv = wl.grid_conductivities(H, W, seed=H + W)
    f = hm.frontal_create(ch, cv)
    X = wl.gaussian((H, m), seed=m)
    Y = _apply(f, X)
    Yo = ofr.FrontalOp(ch, cv).apply(X)
    e = rel(Y, Yo) if H > 1 else float(np.abs(Y).max())
    say(f"  rel err {e:.2e}")
    if H == 1:
        assert np.abs(Y).max() < 1e-13 * np.abs(X).max() * 8
    else:
        assert e < TOL


def test_frontal_apply_leading_dimensions_and_properties():
    H, W = 600, 41
    ch, cv = wl.grid_conductivities(H, W, seed=5)
    f = hm.frontal_create(ch, cv)
    # column-major blocks with leading dimensions H + 9 (X) and H + 3 (Y):
    # row-major (6, ld) buffers, transposed
    Xb = torch.from_numpy(wl.gaussian((6, H + 9), seed=2)).cuda()
    Yb = torch.full((6, H + 3), float("nan"), dtype=torch.float64, device="cuda")
    rc = hm.lib.hm_frontal_apply(f.handle, 6, Xb.data_ptr(), H + 9, Yb.data_ptr(), H + 3, None)
    assert rc == 0
    torch.cuda.synchronize()
    Yo = ofr.FrontalOp(ch, cv).apply(Xb.T[:H].cpu().numpy())
    assert rel(Yb.T[:H].cpu().numpy(), Yo) < TOL
    assert torch.isnan(Yb[:, H:]).all()      # rows past n are not written
    # a Laplacian: A 1 = 0; symmetric
    ones = _apply(f, np.ones((H, 1)))
    assert np.abs(ones).max() < 1e-12 * 8
    U = wl.gaussian((H, 3), seed=11)
    AU = _apply(f, U)
    G = U.T @ AU
    assert np.abs(G - G.T).max() < 1e-12 * np.abs(G).max()


def test_frontal_full_size_every_row():
    # the workload of the measurements: 102400 rows, width 41
    H = 102400
    say(f"frontal full size H={H}")
    ch, cv = wl.grid_conductivities(H, 41, seed=7)
    f = hm.frontal_create(ch, cv)
    X = wl.gaussian((H, 4), seed=3)
    Y = _apply(f, X)
    Yo = ofr.FrontalOp(ch, cv).apply(X)
    e = rel(Y, Yo)
    say(f"  rel err {e:.2e}")
    assert e < TOL


def test_frontal_operator_calls_match():
    H = 700
    ch, cv = wl.grid_conductivities(H, 41, seed=9)
    f = hm.frontal_create(ch, cv)
    X = wl.gaussian((H, 10), seed=4)
    Yo = ofr.FrontalOp(ch, cv).apply(X)
    for adj in (False, True):
        Y = hm.hm_operator_apply(hm.FrontalOperator(f), torch.from_numpy(X).cuda(),
                                 adjoint=adj).cpu().numpy()
        assert rel(Y, Yo) < TOL


@pytest.mark.parametrize("kind", ["hodlr", "hbs"])
def test_frontal_compression_matches_oracle(kind):
    # Tables 8 / 9 workload at N = 3200: leaf 100, eps = 1e-9, l = 25 samples
    # per level (HODLR: rank cap 20, p = 5; HBS-ID: its row blocks rank twice
    # the HODLR's, so cap 28 and p = 8)
    H, leaf, seed, tol = 3200, 100, 11, 1e-9
    k, p = (20, 5) if kind == "hodlr" else (28, 8)
    say(f"frontal {kind} compression H={H}")
    ch, cv = wl.grid_conductivities(H, 41, seed=7)
    f = hm.frontal_create(ch, cv)
    op = ofr.FrontalOp(ch, cv)
    opts = hm.Options(H, leaf, k, p, tol=tol, seed=seed)
    if kind == "hodlr":
        h = hm.hodlr_compress(opts, hm.FrontalOperator(f))
        ho, _ = ohodlr.compress(op, H, leaf, k + p, seed, rank=k, tol=tol)
        apply_o = ho.apply
    else:
        h = hm.hbs_compress(opts, hm.FrontalOperator(f))
        ho = ohbs.compress(op, H, leaf, k + p, seed, rank=k, tol=tol)[0]
        apply_o = lambda x: ohbs.apply_hbs(ho, x)
    X = wl.gaussian((H, 8), seed=12)
    AX = op.apply(X)
    Y = h.apply(torch.from_numpy(X)).cpu().numpy()
    Yo = apply_o(X)
    inf = h.info()
    say(f"  ranks {inf['min_rank']}..{inf['max_rank']}  gpu vs A {rel(Y, AX):.2e}"
        f"  oracle vs A {rel(Yo, AX):.2e}  gpu vs oracle {rel(Y, Yo):.2e}")
    assert inf["max_rank"] < k                 # no block saturated its cap
    # both meet the tolerance; they agree to within it (rank decisions at the
    # threshold may differ by rounding)
    assert rel(Y, AX) < 20 * tol and rel(Yo, AX) < 20 * tol
    assert rel(Y, Yo) < 20 * tol


def test_frontal_rejects_a_grid_without_conductance():
    # every bar at zero: D = 0, the first pivot is not positive -> HM_ERR_SINGULAR,
    # reported by the factor's own pivot check (no fault, no handle)
    import ctypes as C
    H, W = 16, 41
    ch = torch.zeros((H, W - 1), dtype=torch.float64, device="cuda")
    cv = torch.zeros((H - 1, W), dtype=torch.float64, device="cuda")
    f = C.c_void_p()
    rc = hm.lib.hm_frontal_create(H, W, ch.data_ptr(), cv.data_ptr(), None, C.byref(f))
    assert rc == -7 and f.value is None
    assert b"pivot" in hm.lib.hm_last_error()


def test_frontal_handle_outlives_its_inputs():
    # the conductivities are read during create only; the handle keeps what it needs
    H = 300
    ch, cv = wl.grid_conductivities(H, 41, seed=13)
    chd, cvd = torch.from_numpy(ch).cuda(), torch.from_numpy(cv).cuda()
    f = hm.frontal_create(chd, cvd)
    chd.fill_(float("nan"))
    cvd.fill_(float("nan"))
    del chd, cvd
    torch.cuda.synchronize()
    X = wl.gaussian((H, 5), seed=2)
    assert rel(_apply(f, X), ofr.FrontalOp(ch, cv).apply(X)) < TOL
