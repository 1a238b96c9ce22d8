"""Write the FP64 oracle fixture of the near-singular kernel workload at full
size: N = 65536 points on the random-Fourier curve (seed 3), kernel
1/(|x - y| + 1e-3) (1000 on the diagonal), leaf 128, k = 32, p = 16,
test-matrix seed 3, fixed-rank mode (Fig. 4 then Fig. 5).

Calls only ``oracle/`` and ``workloads/``.  One clean compression, then the
same compression with relative noise on every sample entry (the products a
sampler with rounding error of that size could return), which measures how
far rounding of the samples alone moves the result.  Stored (``.npz``, no
pickles):

* ``rows``: 1024 sampled row indices (``numpy.random.default_rng(0)``);
  probes are ``workloads.gaussian((N, 8), seed=99)``;
* ``y_A``: exact A times the probes on those rows (kernel entries of the
  rows against all N columns);
* ``y_id``, ``y_ortho``: the oracle's HBS-ID form (Fig. 5) and orthonormal
  form (Fig. 4) times the probes, on those rows; ``y_id_noise``,
  ``y_ortho_noise``: the same for each noisy run (``noise_amp``);
* ``rank_u``, ``rank_v``, ``skel_in``, ``skel_out`` (node-indexed, -1
  padded) and ``prefix_in``, ``prefix_out``: the number of leading pivots of
  each node's ID decided by a margin above ``gap_floor`` (``lowrank.cpqr``);
  ``skel_in_noise``/``skel_out_noise``: the noisy runs' skeletons;
* ``meta``: JSON text with the configuration, wall times, thread counts, the
  errors against A and spreads, and ``bskel_err``: the largest
  ``|B^skel - A(skel_in, skel_out)|`` of the clean run's HBS-ID form over all
  sibling pairs, relative to the largest entry of A met (eq. ben1).

Usage: ``python tests/golden/make_oracle_fixture.py [--n N] [--out PATH]``
(about 10 minutes per compression on 8 cores at N = 65536).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W                                   # noqa: E402
from oracle import hbs as ohbs                          # noqa: E402
from oracle import operators as oops                    # noqa: E402

LEAF, K, P, SEED, DELTA = 128, 32, 16, 3, 1e-3
ROWS, PROBES, PROBE_SEED = 1024, 8, 99
GAP_FLOOR = 1e-6
# (amplitude, generator seed) of each noisy run; 1e-13 is the relative
# error the GPU's FP64 sampler is held to in its own tests, 1e-12 ten times it
NOISE = ((1e-13, 1), (1e-13, 2), (1e-12, 3))


def decided_prefix(gaps, floor):
    below = np.flatnonzero(np.asarray(gaps) < floor)
    return int(below[0]) if below.size else len(gaps)


def node_tables(h, nn):
    ru = np.zeros(nn, np.int32)
    rv = np.zeros(nn, np.int32)
    si = np.full((nn, K), -1, np.int32)
    so = np.full((nn, K), -1, np.int32)
    pi = np.zeros(nn, np.int32)
    po = np.zeros(nn, np.int32)
    for t in range(2, nn):
        ru[t], rv[t] = h.rank_u(t), h.rank_v(t)
        si[t, :len(h.skel_in[t])] = h.skel_in[t]
        so[t, :len(h.skel_out[t])] = h.skel_out[t]
        pi[t] = decided_prefix(h.gaps_in[t], GAP_FLOOR)
        po[t] = decided_prefix(h.gaps_out[t], GAP_FLOOR)
    return ru, rv, si, so, pi, po


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    n = a.n
    out = a.out or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                f"near_n{n}_oracle.npz")
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        limit = threadpool_limits(1)      # threads go to the row tiles instead
        blas = [(i["internal_api"], i["num_threads"]) for i in threadpool_info()]
    except ImportError:                   # pragma: no cover
        limit, blas = None, []
    pts = W.fourier_curve_points(n, seed=SEED)
    op = oops.KernelOp(pts, "near", DELTA, workers=a.workers)
    rows = np.sort(np.random.default_rng(0).choice(n, min(ROWS, n), replace=False))
    x = W.gaussian((n, PROBES), seed=PROBE_SEED)
    y_A = op.entries(rows, np.arange(n)) @ x
    meta = dict(n=n, leaf=LEAF, k=K, p=P, seed=SEED, kernel="near", delta=DELTA,
                point_seed=SEED, probe_seed=PROBE_SEED, probes=PROBES, gap_floor=GAP_FLOOR,
                noise=[list(z) for z in NOISE], workers=a.workers, blas=blas,
                host=platform.processor() or platform.machine(),
                cpus=len(os.sched_getaffinity(0)))
    res = {}

    def run(o, tag):
        t0 = time.perf_counter()
        h, st, ex = ohbs.compress(o, n, LEAF, K + P, SEED, rank=K)
        dt = time.perf_counter() - t0
        print(f"{tag}: compress {dt:.1f} s, {st.calls} calls, {st.columns} columns", flush=True)
        return h, ex, dt

    h0, ex0, t_clean = run(op, "clean")
    meta["t_compress_s"] = t_clean
    worst, amax = 0.0, 0.0
    for (a_, b_), Bab in h0.B.items():
        Aab = op.entries(h0.skel_in[a_], h0.skel_out[b_])
        worst = max(worst, float(np.abs(Bab - Aab).max()))
        amax = max(amax, float(np.abs(Aab).max()))
    meta["bskel_err"] = worst / amax
    print(f"B^skel vs A(skel): {worst / amax:.2e}", flush=True)
    nn = 2 ** (h0.tree.L + 1)
    res["rows"] = rows.astype(np.int64)
    res["y_A"] = y_A
    res["y_id"] = h0.apply(x)[rows]
    res["y_ortho"] = ex0["ortho"].apply(x)[rows]
    (res["rank_u"], res["rank_v"], res["skel_in"], res["skel_out"], res["prefix_in"],
     res["prefix_out"]) = node_tables(h0, nn)
    del ex0
    yi, yo, si, so = [], [], [], []
    for amp, s in NOISE:
        h1, ex1, _ = run(oops.PerturbedOp(op, amp, s), f"noise {amp:.0e} seed {s}")
        yi.append(h1.apply(x)[rows])
        yo.append(ex1["ortho"].apply(x)[rows])
        _, _, a_in, a_out, _, _ = node_tables(h1, nn)
        si.append(a_in)
        so.append(a_out)
        del h1, ex1
    res["y_id_noise"] = np.stack(yi)
    res["y_ortho_noise"] = np.stack(yo)
    res["skel_in_noise"] = np.stack(si)
    res["skel_out_noise"] = np.stack(so)
    rel = lambda u, v: float(np.linalg.norm(u - v) / np.linalg.norm(v))
    meta["oracle_vs_A_id"] = rel(res["y_id"], y_A)
    meta["oracle_vs_A_ortho"] = rel(res["y_ortho"], y_A)
    meta["spread_id"] = [rel(y, res["y_id"]) for y in yi]
    meta["spread_ortho"] = [rel(y, res["y_ortho"]) for y in yo]
    print(json.dumps({k: meta[k] for k in ("oracle_vs_A_id", "oracle_vs_A_ortho", "spread_id",
                                           "spread_ortho")}), flush=True)
    np.savez_compressed(out, meta=np.array(json.dumps(meta)), **res)
    print(f"wrote {out}", flush=True)
    if limit is not None:
        limit.unregister() if hasattr(limit, "unregister") else None


if __name__ == "__main__":
    main()
