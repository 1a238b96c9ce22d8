"""Helpers of the GPU parity tests (imported by them; no tests here).

* ``hbs_id_structure``: the properties that define an HBS-ID form (Sec. 3.3,
  Sec. 4.3, eq. ben0-ben2), checked on the library's exported output:
  identity rows of the interpolation bases at the skeleton, nested skeletons,
  and ``B^skel_ab = A(skel_in_a, skel_out_b)`` entry by entry.
* ``skeleton_prefix_mismatches``: compares the GPU's skeleton sequences with
  the oracle's over the leading pivots that the oracle's ID decided by a
  margin above a rounding floor (later pivots are near ties that rounding
  decides, so any correct implementation may differ there).
* ``oracle_spread``: reruns the oracle with relative noise on its samples and
  returns how far that alone moves its result -- the yardstick for a GPU
  result whose products round differently from the oracle's.
"""
from __future__ import annotations

import numpy as np

from oracle import hbs as ohbs
from oracle import operators as oops

# relative error the GPU's FP64 kernel sampler is held to in its own tests
# (test_kernel_sampler_matches_dense_product): noise of that size on the
# oracle's samples is what the parity bound is calibrated against
SAMPLE_NOISE = 1e-13
# margin (relative to the first pivot's residual norm) above which a pivot
# is decided, far above rounding of the ID's input (~1e-10 relative)
GAP_FLOOR = 1e-6
# stated multiple of the oracle's own spread within which a GPU result
# counts as equal to it
SPREAD_FACTOR = 3.0


def hbs_id_structure(e, entries, nodes_max=None):
    """Check the exported HBS-ID form ``e`` (``HBS.export()``) against the
    operator's entries (``entries(rows, cols)``, instance-local indices).
    Returns the largest ``|B^skel - A(skel_in, skel_out)|`` relative to the
    largest entry of A met, after asserting identity rows and nestedness."""
    L, R = e["L"], e["R"]
    nn = 2 ** (L + 1)
    ru, rv, si, so = e["rank_u"], e["rank_v"], e["skel_in"], e["skel_out"]
    U = e["U"].cpu().numpy()
    V = e["V"].cpu().numpy()
    Ut = e["Ut"].cpu().numpy()
    Vt = e["Vt"].cpu().numpy()
    B = e["B"].cpu().numpy()
    first_leaf = 2 ** L
    worst, amax = 0.0, 0.0
    for t in range(2, nn):
        for rk, sk, leafb, tr in ((ru, si, U, Ut), (rv, so, V, Vt)):
            k = int(rk[t])
            s = sk[t, :k]
            assert np.all(s >= 0) and np.all(sk[t, k:] == -1), t
            assert len(set(s.tolist())) == k, f"node {t}: repeated skeleton"
            if t >= first_leaf:
                # leaf basis: rows at the skeleton are the identity
                np.testing.assert_array_equal(leafb[s, :k], np.eye(k), err_msg=f"leaf {t}")
                np.testing.assert_array_equal(leafb[s, k:], 0.0)
            else:
                a, b = 2 * t, 2 * t + 1
                ka, kb = int(rk[a]), int(rk[b])
                cand = np.full(2 * R, -1)
                cand[:ka] = sk[a, :ka]
                cand[R:R + kb] = sk[b, :kb]
                # nested: the parent's skeleton is drawn from its children's
                pos = [int(np.flatnonzero(cand == x)[0]) if np.any(cand == x) else -1 for x in s]
                assert min(pos) >= 0, f"node {t}: skeleton not nested in its children's"
                np.testing.assert_array_equal(tr[t][pos, :k], np.eye(k), err_msg=f"node {t}")
                pad = np.r_[np.arange(ka, R), np.arange(R + kb, 2 * R)]
                assert np.all(tr[t][pad] == 0.0)
        # B^skel_{sib(t), t} = A(skel_in[sib], skel_out[t])
        s_in = si[t ^ 1, :int(ru[t ^ 1])]
        s_out = so[t, :int(rv[t])]
        A = entries(s_in, s_out)
        worst = max(worst, float(np.abs(B[t][:len(s_in), :len(s_out)] - A).max()))
        amax = max(amax, float(np.abs(A).max()))
    return worst / amax


def oracle_bskel_error(ho, entries):
    """The same ``B^skel`` check on the oracle's own HBS-ID form."""
    worst, amax = 0.0, 0.0
    for (a, b), Bab in ho.B.items():
        A = entries(ho.skel_in[a], ho.skel_out[b])
        worst = max(worst, float(np.abs(Bab - A).max()))
        amax = max(amax, float(np.abs(A).max()))
    return worst / amax


def skeleton_prefix_mismatches(e, ho, floor=GAP_FLOOR):
    """Nodes whose GPU skeleton sequence differs from the oracle's within
    the oracle's decided prefix.  Leaves always count; a parent counts when
    both children's skeletons agree as sets (else its candidates differ).
    Returns ``(mismatches, compared)``."""
    L = ho.tree.L
    bad, compared = [], 0
    for side in ("in", "out"):
        gsk = e["skel_" + side]
        grk = e["rank_u" if side == "in" else "rank_v"]
        osk = getattr(ho, "skel_" + side)
        gaps = getattr(ho, "gaps_" + side)
        same_set = {}
        for lev in range(L, 0, -1):
            for t in ho.tree.level_nodes(lev):
                g = gsk[t, :int(grk[t])]
                o = np.asarray(osk[t])
                same_set[t] = set(g.tolist()) == set(o.tolist())
                if lev < L and not (same_set[2 * t] and same_set[2 * t + 1]):
                    continue
                below = np.flatnonzero(np.asarray(gaps[t]) < floor)
                d = int(below[0]) if below.size else len(gaps[t])
                compared += 1
                if not np.array_equal(g[:d], o[:d]):
                    bad.append((side, t, d))
    return bad, compared


def oracle_spread(op, n, leaf, r, seed, rank, tol, probe, runs=2, amp=SAMPLE_NOISE):
    """Rerun the oracle with relative noise ``amp`` on every sample entry;
    returns the list of ``(hbs_id, orthonormal)`` results of the runs."""
    out = []
    for s in range(1, runs + 1):
        h, _, ex = ohbs.compress(oops.PerturbedOp(op, amp, s), n, leaf, r, seed, rank=rank,
                                 tol=tol)
        out.append((h, ex["ortho"]))
    return out


def max_rel(a, b, scale):
    """Largest entrywise difference relative to ``scale``."""
    return float(np.abs(a - b).max() / scale)
