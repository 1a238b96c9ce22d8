"""Benchmark of the randomized HBS compression on one MI355X.

Workload (the mixed-precision configuration): HBS compression of the kernel
matrix A(i,j) = 1/(|x_i - x_j| + 1e-3) on N = 65536 points of a smooth
random-Fourier closed curve (8 modes, amplitude 0.2, seed 3), leaf 128
(L = 9 levels), rank k = 32, oversampling p = 16 (r = 48 samples per level),
HBS-ID output.  The operator is sampled on BF16 MFMA with FP32 accumulation;
node factorisations (Householder TSQR, Jacobi SVD, pivoted-QR ID) run in FP64.

One step = one full ``hbs_compress`` call (test matrices, operator samples,
telescoping subtraction, node factorisations, transfers, diagonal blocks,
HBS-ID sweep) with the points already resident in HBM.

Reported: ``value`` = GFLOP/s of the compression, counting the operator
products as dense N x N x c products (2 N^2 per sampled column, the paper's
T_mult cost) plus nothing else (the net factorisation work is ~1% and is not
counted); compress seconds of the BF16, FP32 and FP64 forms; accuracy of each
form on sampled rows against the exact matrix; the dominant kernel's
roofline; the CPU oracle on a bounded sample of the same products.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N, LEAF, K, P, DELTA, SEED_PTS, SEED = 65536, 128, 32, 16, 1e-3, 3, 3

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_TF = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}
# Peak of plain vector ALU work on MI355X: 256 CUs x 4 SIMDs x 32 FP32 lanes
# x 2.4 GHz = 78.6e12 lane-slots/s for non-packed FP32 operations (the FP32
# vector peak of 157.3 TFLOP/s counts an FMA as two); transcendentals (sqrt,
# rcp) issue at a quarter of that rate and count 4 slots (measured on the
# device: 61.6 T adds/s, 17.2 T reciprocals/s in a full-chip issue test).
PEAK_ALU_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12
# instruction slots per kernel entry in the BF16 sampler (from its code):
# 2 FP32 subtractions, mul, fma (d^2), sqrt (4), add (+delta), rcp (4), half a
# packed BF16 conversion = 13.5 slots
SLOTS_PER_ENTRY = 13.5

# HBM bytes of one BF16 operator apply (k_pack + k_sampler + k_sum_parts,
# N = 65536, 96 columns) from two rocprofv3 --pmc passes (FETCH_SIZE,
# WRITE_SIZE in KiB per dispatch, summed over the three kernels), scaled by
# what the same counters read for a plain 256 MiB device copy (FETCH_SIZE
# reads 0.5x the bytes moved, WRITE_SIZE 1.0x).  Most of it is the three
# K-split partial products (written, read back, summed).  Valid only for the
# sampler source they were taken on (SHA-1 below); otherwise unknown.
SAMPLER_TRAFFIC = {"sha1": "ccd8b683386b3325e55a31dcc936cac39c3c7669",
                   "fetch_kib": 24590.8 + 96446.5 + 73746.7,
                   "write_kib": 12320.0 + 148705.4 + 49152.0,
                   "fetch_scale": 2.0, "write_scale": 1.0}


def sampler_traffic_bytes():
    import hashlib
    src = os.path.join(ROOT, "paper_1503_07152_amd", "csrc", "sampler.hip")
    with open(src, "rb") as f:
        if hashlib.sha1(f.read()).hexdigest() != SAMPLER_TRAFFIC["sha1"]:
            return None
    t = SAMPLER_TRAFFIC
    return int((t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024)


def levels(n, leaf):
    return 0 if n <= leaf else int(math.ceil(math.log2(n / leaf)))


def sample_columns(n, leaf, r):
    L = levels(n, leaf)
    return 4 * r * L + -(-n // 2 ** L)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=N)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the timed BF16 steps (for profiling runs)")
    ap.add_argument("--sampler-only", action="store_true",
                    help="only the BF16 sampler on one structured N x 96 block, 3 launches "
                         "(hardware-counter runs)")
    ap.add_argument("--apply-only", action="store_true",
                    help="only the forward and backward compressed apply of the "
                         "differentiation workload (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only a plain device copy of 256 MiB, 3 times (scale of the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is design-only)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1503_07152_amd as hm
    import workloads as W

    n = args.n
    r = K + P
    torch.cuda.set_device(0)
    # the library's device memory (compress workspaces, handles, apply scratch)
    # comes from torch's caching allocator, as in a PyTorch program: no
    # hipMalloc / hipFree (which synchronises) inside the timed calls
    hm.use_torch_allocator(True)
    if args.copy_calibration:
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print("copy calibration: 3 x 268435456 bytes read and written", flush=True)
        return
    if args.apply_only:
        print(json.dumps(backward_measurement(hm, W, torch)), flush=True)
        return
    if args.sampler_only:
        pts = torch.from_numpy(W.fourier_curve_points(n, seed=SEED_PTS)).cuda()
        c = 2 * r
        X = hm.fortran(n, c)
        X.copy_(torch.from_numpy(W.gaussian((n, c), seed=5)))
        X[: n // 2, : c // 2] = 0.0
        X[n // 2:, c // 2:] = 0.0
        op = hm.KernelOperator(pts, "near", DELTA, hm.HM_BF16)
        for _ in range(3):
            hm.hm_operator_apply(op, X)
        torch.cuda.synchronize()
        print(f"sampler-only: 3 launches, N={n}, {c} columns", flush=True)
        return
    pts = torch.from_numpy(W.fourier_curve_points(n, seed=SEED_PTS)).cuda()
    op_bf16 = hm.KernelOperator(pts, "near", DELTA, hm.HM_BF16)
    opts = hm.Options(n, LEAF, K, P, seed=SEED)
    print(f"bench: HBS compress N={n} leaf={LEAF} k={K} p={P} BF16 sampling; "
          f"warmup {args.warmup}, steps {args.steps}", flush=True)

    for i in range(args.warmup):
        h = hm.hbs_compress(opts, op_bf16)
        print(f"warmup {i}: {h.info()['t_compress_ms']:.1f} ms", flush=True)
        del h
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    h = None
    for i in range(args.steps):
        del h
        h = hm.hbs_compress(opts, op_bf16)
        infos.append(h.info())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    cols = sample_columns(n, LEAF, r)
    assert infos[-1]["sample_columns"] == cols, (infos[-1]["sample_columns"], cols)
    flops = 2.0 * n * n * cols
    value = flops / (ms * 1e-3) / 1e9
    print(f"timed: {ms:.1f} ms/step, {value:.0f} GFLOP/s; operator share "
          f"{infos[-1]['t_operator_ms'] / infos[-1]['t_compress_ms']:.2f}", flush=True)

    out = {
        "metric": "HBS compress s + GFLOP/s at N=65536,k=32 vs FP64 GPU; rel error; bwd apply GB/s",
        "value": round(value, 1), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic (random-Fourier curve points, seed 3; Philox test matrices, seed 3)",
        "config": {"workload": f"HBS-ID compression N={n} leaf={LEAF} k={K} p={P}, "
                               "kernel 1/(|x-y|+1e-3) on a random-Fourier curve, BF16 MFMA "
                               "sampling, FP64 factorisations",
                   "n": n, "leaf": LEAF, "rank": K, "oversample": P,
                   "levels": levels(n, LEAF), "sample_columns": cols},
        "compress_s_bf16": round(ms / 1e3, 4),
        "t_net_s_bf16": round((infos[-1]["t_compress_ms"] - infos[-1]["t_operator_ms"]) / 1e3, 4),
        "jacobi_sweeps_max": infos[-1]["jacobi_sweeps"],
    }
    if not args.no_extra:
        out.update(extra_measurements(hm, W, torch, pts, n, h, ms))
        out.update(backward_measurement(hm, W, torch))
        out.update(batched_measurement(hm, W, torch))
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(W, n)
    print(json.dumps(out), flush=True)


def extra_measurements(hm, W, torch, pts, n, h_bf16, ms_bf16):
    from oracle import operators as oops   # exact entries of A on sampled rows only
    res = {}
    # ---- other precisions, one compress each ---------------------------------
    forms = {"bf16": h_bf16}
    times = {"bf16": ms_bf16 / 1e3}
    for name, dt in (("f32", hm.HM_F32), ("f64", hm.HM_F64)):
        op = hm.KernelOperator(pts, "near", DELTA, dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hh = hm.hbs_compress(hm.Options(n, LEAF, K, P, seed=SEED), op)
        torch.cuda.synchronize()
        times[name] = time.perf_counter() - t0
        forms[name] = hh
        print(f"{name} form: {times[name] * 1e3:.1f} ms", flush=True)
    res["compress_s_f32"] = round(times["f32"], 4)
    res["compress_s_f64"] = round(times["f64"], 4)
    res["speedup_bf16_vs_f64_gpu"] = round(times["f64"] / times["bf16"], 2)
    res["speedup_f32_vs_f64_gpu"] = round(times["f64"] / times["f32"], 2)
    # ---- accuracy on sampled rows against the exact matrix --------------------
    Kop = oops.KernelOp(pts.cpu().numpy(), "near", DELTA)
    rows = np.random.default_rng(0).choice(n, 256, replace=False)
    w = W.gaussian((n, 4), seed=21)
    exact = Kop.entries(rows, np.arange(n)) @ w
    for name, hh in forms.items():
        y = hh.apply(torch.from_numpy(w)).cpu().numpy()[rows]
        res[f"rel_err_{name}_vs_A_sampled_rows"] = float(np.linalg.norm(y - exact) /
                                                          np.linalg.norm(exact))
    yb = forms["bf16"].apply(torch.from_numpy(w)).cpu().numpy()
    y64 = forms["f64"].apply(torch.from_numpy(w)).cpu().numpy()
    y32 = forms["f32"].apply(torch.from_numpy(w)).cpu().numpy()
    res["rel_err_bf16_vs_f64_gpu"] = float(np.linalg.norm(yb - y64) / np.linalg.norm(y64))
    res["rel_err_f32_vs_f64_gpu"] = float(np.linalg.norm(y32 - y64) / np.linalg.norm(y64))
    inf = forms["bf16"].info()
    res["ranks"] = [inf["min_rank"], inf["max_rank"]]
    res["storage_reals_per_dof"] = round(inf["storage_reals"] / n, 1)
    # ---- dominant kernel: the BF16 sampler, timed live with HIP events --------
    c = 2 * (K + P)
    X = hm.fortran(n, c)
    X.copy_(torch.from_numpy(W.gaussian((n, c), seed=5)))
    half = n // 2
    X[:half, :c // 2] = 0.0          # structured like [Omega_2 | Omega_1]
    X[half:, c // 2:] = 0.0
    s = torch.cuda.current_stream()
    hm.hm_operator_apply(hm.KernelOperator(pts, "near", DELTA, hm.HM_BF16), X)
    reps = 5
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    op = hm.KernelOperator(pts, "near", DELTA, hm.HM_BF16)
    e0.record(s)
    for _ in range(reps):
        hm.hm_operator_apply(op, X, stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    t_launch = e0.elapsed_time(e1) / reps * 1e-3
    entries = float(n) * n
    achieved = entries * SLOTS_PER_ENTRY / t_launch / 1e12
    res["roofline"] = {"bound": "alu", "achieved": round(achieved, 2), "peak": round(PEAK_ALU_TOPS, 1),
                       "unit": "Tslot/s", "frac": round(achieved / PEAK_ALU_TOPS, 3),
                       "traffic": sampler_traffic_bytes() if n == N else None,
                       "kernel": "k_sampler<BF16, near> (+ k_pack, k_sum_parts)",
                       "launch_ms": round(t_launch * 1e3, 3),
                       "mfma_frac": round(2 * n * (n * c / 2) / t_launch / 1e12 /
                                          PEAK_TF["bf16"], 4)}
    # FP64 form of the same kernel, MFMA-bound
    op64 = hm.KernelOperator(pts, "near", DELTA, hm.HM_F64)
    hm.hm_operator_apply(op64, X, stream=s)
    e0.record(s)
    for _ in range(2):
        hm.hm_operator_apply(op64, X, stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    t64 = e0.elapsed_time(e1) / 2 * 1e-3
    res["roofline_f64_sampler"] = {"bound": "mfma", "achieved": round(2 * n * (n * c / 2) / t64 / 1e12, 2),
                                   "peak": PEAK_TF["f64"], "unit": "TFLOP/s",
                                   "frac": round(2 * n * (n * c / 2) / t64 / 1e12 / PEAK_TF["f64"], 3),
                                   "launch_ms": round(t64 * 1e3, 3),
                                   "note": "flops of the nonzero half of the structured block"}
    return res


def backward_measurement(hm, W, torch, n=262144, leaf=128, k=32, c=64):
    """Backward of the compressed apply y = A_H x (the differentiation
    workload): synthetic HBS N=262144, leaf 128, k=32 (seed 4), 64 FP32
    right-hand sides (seed 5).  Algorithmic bytes = every input read once
    (x, gy, U, V, D, transfers, B) + every output written once (gx, gU, gV,
    gD, gUt, gVt, gB)."""
    g = W.synthetic_hbs(n, leaf, k, seed=4, dtype=np.float32)
    h = hm.hm_hbs_from_generators(g, dtype=hm.HM_F32)
    x = hm.to_fortran(torch.from_numpy(W.gaussian((n, c), seed=5, dtype=np.float32)))
    gy = hm.to_fortran(torch.from_numpy(W.gaussian((n, c), seed=6, dtype=np.float32)))
    s = torch.cuda.current_stream()
    hm.hss_apply_backward(h, x, gy)
    hm.hss_apply(h, x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record(s)
    for _ in range(reps):
        hm.hss_apply_backward(h, x, gy, stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    tb = e0.elapsed_time(e1) / reps * 1e-3
    e0.record(s)
    for _ in range(reps):
        hm.hss_apply(h, x, stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    tf = e0.elapsed_time(e1) / reps * 1e-3
    L = int(math.ceil(math.log2(n / leaf)))
    nn = 2 ** (L + 1)
    nmax = -(-n // 2 ** L)
    small = nn * (2 * 2 * k * k + k * k)          # Ut, Vt, B
    elems_in = 2 * n * c + 2 * n * k + n * nmax + small
    elems_out = n * c + 2 * n * k + n * nmax + small
    bwd_bytes = 4.0 * (elems_in + elems_out)
    fwd_bytes = 4.0 * (n * c + 2 * n * k + n * nmax + small + n * c)
    bw = bwd_bytes / tb / 1e9
    return {"bwd_apply_GBps": round(bw, 1), "bwd_apply_ms": round(tb * 1e3, 3),
            "bwd_apply_hbm_frac": round(bw / PEAK_HBM_GBS, 3),
            "fwd_apply_GBps": round(fwd_bytes / tf / 1e9, 1), "fwd_apply_ms": round(tf * 1e3, 3),
            "apply_config": f"synthetic HBS N={n} leaf={leaf} k={k}, {c} FP32 right-hand sides"}


def batched_measurement(hm, W, torch, count=256, leaf=128, p=8):
    """Many uneven instances: N_i log-uniform in [512, 8192] (multiples of 64),
    k_i uniform in [8, 40] (seed 2), synthetic HBS operators; one batched call
    against one call per instance."""
    specs = W.batched_instances(count, seed=2)
    ops_h = [hm.hm_hbs_from_generators(W.synthetic_hbs(n, leaf, k, seed=1000 + i))
             for i, (n, k) in enumerate(specs)]
    opts = [hm.Options(n, leaf, k, p, seed=2 + i) for i, (n, k) in enumerate(specs)]
    ops = [hm.HBSOperator(h) for h in ops_h]
    hm.hbs_compress_batched(opts[:8], ops[:8])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = hm.hbs_compress_batched(opts, ops)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    del outs
    t0 = time.perf_counter()
    for o, op in zip(opts, ops):
        h = hm.hbs_compress(o, op)
        del h
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    return {"batched_instances": count, "batched_total_n": int(sum(n for n, _ in specs)),
            "batched_s": round(tb, 4), "batched_instances_per_s": round(count / tb, 1),
            "sequential_s": round(ts, 4), "batched_speedup": round(ts / tb, 2)}


def cpu_baseline(W, n):
    """The FP64 oracle's operator product (the dominant step of the
    compression) on a bounded sample: 1024 of the N rows against all N columns
    and 96 sampled columns; scaled to GFLOP/s with the same 2 N^2 per column
    count as ``value``."""
    from oracle import operators as oops
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:  # noqa: BLE001
        threads = 1
    pts = W.fourier_curve_points(n, seed=SEED_PTS)
    Kop = oops.KernelOp(pts, "near", DELTA, tile=256)
    X = W.gaussian((n, 96), seed=5)
    rows = 1024
    sub = oops.KernelOp(pts, "near", DELTA, tile=256)
    t0 = time.perf_counter()
    done = 0
    for i0 in range(0, rows, 256):
        idx = np.arange(i0, min(i0 + 256, rows))
        _ = sub.entries(idx, np.arange(n)) @ X
        done += len(idx)
    dt = time.perf_counter() - t0
    gflops = 2.0 * done * n * 96 / dt / 1e9
    return {"value": round(gflops, 2), "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle kernel-matrix product, {done} of {n} rows x {n} columns x 96 "
                      f"columns ({dt:.1f} s); FP64 NumPy"}


if __name__ == "__main__":
    main()
