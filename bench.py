"""Benchmark of the randomized HBS compression on one MI355X.

Workload (the mixed-precision configuration): HBS compression of the kernel
matrix A(i,j) = 1/(|x_i - x_j| + 1e-3) on N = 65536 points of a smooth
random-Fourier closed curve (8 modes, amplitude 0.2, seed 3), leaf 128
(L = 9 levels), rank k = 32, oversampling p = 16 (r = 48 samples per level),
HBS-ID output.  The operator is sampled on BF16 MFMA with FP32 accumulation;
node factorisations (Gram/Householder, Jacobi SVD, pivoted-QR ID) run in FP64.

One step = one full ``hbs_compress`` call (test matrices, operator samples,
telescoping subtraction, node factorisations, transfers, diagonal blocks,
HBS-ID sweep) with the points already resident in HBM.

Reported: ``value`` = GFLOP/s of the compression counting the method's own
operator work: each structured test block [Omega_2 | Omega_1] of 2r columns
has N/2 nonzero rows per column (N^2 flops per column), 4 r L such columns in
all, plus the block identity (2 N^2 in all): (4 r L + 2) N^2 flops per step
(the net factorisation work, ~1 %, is not counted); the dense-equivalent
figure (2 N^2 per sampled column) is reported beside it.  Compress seconds of
the BF16, FP32 and FP64 forms (median of timed calls after a warm-up call);
accuracy of each form against the FP64 oracle's compression of the same
workload (``tests/golden/near_n65536_oracle.npz``, written by the oracle) and
against the exact matrix on sampled rows; the dominant kernel's roofline;
the differentiation, synthetic-HBS and batched workloads; the CPU oracle's
full compression of the same workload at N = 32768.
"""
from __future__ import annotations

import argparse
import ctypes as C
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

# HBM bytes of one BF16 operator apply at N = 65536 (96 columns: k_pack,
# k_sampler, k_sum_parts; 288 columns: k_pack, k_sampler) from two rocprofv3
# --pmc passes (FETCH_SIZE, WRITE_SIZE in KiB per dispatch, summed over the
# kernels of the call), scaled by what the same counters read for a plain
# 256 MiB device copy (FETCH_SIZE reads 0.5x the bytes moved, WRITE_SIZE 1.0x).
# Valid only for the sampler source they were taken on (SHA-1); otherwise
# reported as unknown (null).
SAMPLER_TRAFFIC = {
    96: {"sha1": "d3cb4a07aceb989cc85533415719783fa98d9c8a",
         "fetch_kib": 24591.2 + 93679.6 + 36882.5,
         "write_kib": 12320.0 + 73728.0 + 49152.0,
         "fetch_scale": 2.0, "write_scale": 1.0},
    288: {"sha1": "d3cb4a07aceb989cc85533415719783fa98d9c8a",
          "fetch_kib": 73743.4 + 152244.5,
          "write_kib": 36896.4 + 150127.3,
          "fetch_scale": 2.0, "write_scale": 1.0},
}


def sampler_traffic_bytes(c):
    import hashlib
    t = SAMPLER_TRAFFIC.get(c)
    if t is None:
        return None
    src = os.path.join(ROOT, "paper_1503_07152_amd", "csrc", "sampler.hip")
    with open(src, "rb") as f:
        if hashlib.sha1(f.read()).hexdigest() != t["sha1"]:
            return None
    return int((t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024)


def levels(n, leaf):
    return 0 if n <= leaf else int(math.ceil(math.log2(n / leaf)))


def sample_columns(n, leaf, r):
    L = levels(n, leaf)
    return 4 * r * L + -(-n // 2 ** L)


def method_flops(n, leaf, r):
    """Operator work of one compression as the method defines it: the
    structured blocks (N/2 nonzero rows per column, 4 r L columns) and the
    block identity (one nonzero per leaf per column: 2 N^2 in all)."""
    return (4.0 * r * levels(n, leaf) + 2.0) * float(n) * n


def structured_block(W, n, c, nblocks, seed):
    """A test block of `nblocks` levels' [Omega_2 | Omega_1] patterns side by
    side (levels 0, 1, 2, ...): per 2r-column block b, rows in the first half
    of each node at depth b+1 use the block's second half of the columns."""
    X = W.gaussian((n, c), seed=seed)
    w = c // nblocks
    for b in range(nblocks):
        odd = (np.arange(n) // (n >> (b + 1))) % 2 == 1
        X[~odd, w * b + w // 2: w * (b + 1)] = 0.0
        X[odd, w * b: w * b + w // 2] = 0.0
    return X


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=N)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the timed BF16 steps (for profiling runs)")
    ap.add_argument("--sampler-only", type=int, default=0, metavar="C",
                    help="only the BF16 sampler on one structured N x C block (C = 96: one "
                         "level, narrow form; 288: three levels, wide form), 3 launches "
                         "(hardware-counter runs)")
    ap.add_argument("--apply-only", action="store_true",
                    help="only the forward and backward compressed apply of the "
                         "differentiation workload (profiling runs)")
    ap.add_argument("--frontal-only", action="store_true",
                    help="only the frontal-matrix black box and its compressions "
                         "(profiling runs)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (built-in schedule)")
    ap.add_argument("--torch-alloc", action="store_true",
                    help="route the library's device memory through torch's caching "
                         "allocator instead of the library's own block cache")
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
    # the library's device memory (compress workspaces, handles) comes from
    # its own block cache (after the warm-up no hipMalloc / hipFree inside the
    # timed calls), or from torch's caching allocator on request
    if args.torch_alloc:
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
    if args.frontal_only:
        print(json.dumps(frontal_measurement(hm, W, torch)), flush=True)
        return
    if args.sampler_only:
        pts = torch.from_numpy(W.fourier_curve_points(n, seed=SEED_PTS)).cuda()
        c = args.sampler_only
        X = hm.to_fortran(structured_block(W, n, c, max(1, c // (2 * r)), seed=5))
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
    tune = None
    if not args.no_tune:
        # schedule chosen by the library's autotuner for this shape (not timed)
        tune = hm.autotune(opts, op_bf16, reps=2)
        print(f"autotune: {tune}", flush=True)

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
    value = method_flops(n, LEAF, r) / (ms * 1e-3) / 1e9
    dense_equiv = 2.0 * n * n * cols / (ms * 1e-3) / 1e9
    t_net = float(np.median([i["t_compress_ms"] - i["t_operator_ms"] for i in infos]))
    t_cmp = float(np.median([i["t_compress_ms"] for i in infos]))
    print(f"timed: {ms:.1f} ms/step, {value:.0f} GFLOP/s (method flops), "
          f"{dense_equiv:.0f} dense-equivalent; net share {t_net / t_cmp:.2f}", flush=True)

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
        "flop_model": "(4 r L + 2) N^2 per compress: structured test blocks with N/2 nonzero "
                      "rows per column, plus the block identity",
        "dense_equiv_GFLOPs": round(dense_equiv, 1),
        "compress_s_bf16": round(ms / 1e3, 4),
        "t_net_s_bf16": round(t_net / 1e3, 4),
        "net_share_bf16": round(t_net / t_cmp, 3),
        "operator_calls_bf16": infos[-1]["operator_calls"],
        "jacobi_sweeps_max": infos[-1]["jacobi_sweeps"],
        "autotune": tune,
    }
    if not args.no_extra:
        # the Fig. 5 sweep as one persistent launch (device work queue over
        # levels and sides) instead of level by level
        tp, hp = _median_compress(hm, torch, hm.Options(n, LEAF, K, P, seed=SEED,
                                                        persistent_id=True), op_bf16, 5)
        out["compress_s_bf16_persistent_id"] = round(tp, 4)
        print(f"persistent ID sweep: {tp * 1e3:.1f} ms (median of 5)", flush=True)
        del hp
        out.update(extra_measurements(hm, W, torch, pts, n, h, ms))
        out.update(solver_measurement(hm, W, torch, h, n))
        out.update(frontal_measurement(hm, W, torch))
        out.update(backward_measurement(hm, W, torch))
        out.update(synthetic_hbs_measurement(hm, W, torch))
        out.update(product_measurement(hm, W, torch))
        out.update(batched_measurement(hm, W, torch))
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(W)
        out["cpu_product_sample"] = cpu_product_sample(W, n)
    print(json.dumps(out), flush=True)


def _median_compress(hm, torch, opts, op, calls):
    """Median wall time of `calls` compress calls after one warm-up call
    (first launches of each kernel, workspace growth)."""
    h = hm.hbs_compress(opts, op)
    del h
    ts = []
    for _ in range(calls):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = hm.hbs_compress(opts, op)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), h


def _event_time(torch, s, fn, reps):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def extra_measurements(hm, W, torch, pts, n, h_bf16, ms_bf16):
    from oracle import operators as oops   # exact entries of A on sampled rows only
    res = {}
    # ---- other precisions: median of 10 calls each after a warm-up -----------
    forms = {"bf16": h_bf16}
    times = {"bf16": ms_bf16 / 1e3}
    for name, dt in (("f32", hm.HM_F32), ("f64", hm.HM_F64)):
        op = hm.KernelOperator(pts, "near", DELTA, dt)
        times[name], forms[name] = _median_compress(hm, torch, hm.Options(n, LEAF, K, P, seed=SEED),
                                                    op, 10)
        print(f"{name} form: {times[name] * 1e3:.1f} ms (median of 10)", flush=True)
    res["compress_s_f32"] = round(times["f32"], 4)
    res["compress_s_f64"] = round(times["f64"], 4)
    res["speedup_bf16_vs_f64_gpu"] = round(times["f64"] / times["bf16"], 2)
    res["speedup_f32_vs_f64_gpu"] = round(times["f64"] / times["f32"], 2)
    r = K + P
    for name in ("f32", "f64"):
        res[f"GFLOPs_{name}"] = round(method_flops(n, LEAF, r) / times[name] / 1e9, 1)
    # ---- accuracy: against the FP64 oracle's compression of this workload
    # (stored by the oracle) and against the exact matrix, on its sampled rows
    fx = os.path.join(ROOT, "tests", "golden", "near_n65536_oracle.npz")
    if n == N and os.path.exists(fx):
        z = np.load(fx, allow_pickle=False)
        meta = json.loads(str(z["meta"]))
        rows = z["rows"]
        w = W.gaussian((n, meta["probes"]), seed=meta["probe_seed"])
        rl = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
        spread = max(rl(a, z["y_id"]) for a in z["y_id_noise"])
        for name, hh in forms.items():
            y = hh.apply(torch.from_numpy(w)).cpu().numpy()[rows]
            res[f"rel_err_{name}_vs_oracle"] = rl(y, z["y_id"])
            res[f"rel_err_{name}_vs_A"] = rl(y, z["y_A"])
        res["oracle_vs_A"] = rl(z["y_id"], z["y_A"])
        res["oracle_rounding_spread"] = spread
        res["accuracy_sample"] = (f"{len(rows)} sampled rows x {meta['probes']} Gaussian probes; "
                                  "oracle spread = its change under 1e-13 relative sample noise")
    else:
        Kop = oops.KernelOp(pts.cpu().numpy(), "near", DELTA)
        rows = np.random.default_rng(0).choice(n, 256, replace=False)
        w = W.gaussian((n, 4), seed=21)
        exact = Kop.entries(rows, np.arange(n)) @ w
        for name, hh in forms.items():
            y = hh.apply(torch.from_numpy(w)).cpu().numpy()[rows]
            res[f"rel_err_{name}_vs_A"] = float(np.linalg.norm(y - exact) / np.linalg.norm(exact))
    inf = forms["bf16"].info()
    res["ranks"] = [inf["min_rank"], inf["max_rank"]]
    res["storage_reals_per_dof"] = round(inf["storage_reals"] / n, 1)
    # ---- dominant kernel: the BF16 sampler in its wide form (three levels'
    # test blocks, 288 columns: the calls that take most of a step), timed
    # live with HIP events on the stream it is launched on ------------------
    s = torch.cuda.current_stream()
    op = hm.KernelOperator(pts, "near", DELTA, hm.HM_BF16)
    entries = float(n) * n
    for c, key in ((6 * r, "roofline"), (2 * r, "roofline_narrow_sampler")):
        nb = c // (2 * r)
        X = hm.to_fortran(structured_block(W, n, c, nb, seed=5))
        t = _event_time(torch, s, lambda: hm.hm_operator_apply(op, X, stream=s), 5)
        achieved = entries * SLOTS_PER_ENTRY / t / 1e12
        mflops = 2.0 * entries * c / 2          # nonzero half of every structured block
        res[key] = {"bound": "alu", "achieved": round(achieved, 2),
                    "peak": round(PEAK_ALU_TOPS, 1), "unit": "Tslot/s",
                    "frac": round(achieved / PEAK_ALU_TOPS, 3),
                    "traffic": sampler_traffic_bytes(c) if n == N else None,
                    "kernel": f"k_sampler<BF16, near> {c} columns (+ k_pack"
                              f"{', k_sum_parts' if c <= 128 else ''})",
                    "launch_ms": round(t * 1e3, 3),
                    "mfma_frac": round(mflops / t / 1e12 / PEAK_TF["bf16"], 4),
                    "algorithmic_bytes": int(2 * 8 * n * c + 8 * n)}
        print(f"sampler {c} columns: {t * 1e3:.3f} ms, ALU frac {achieved / PEAK_ALU_TOPS:.3f}",
              flush=True)
    # FP64 form of the same kernel (one level), MFMA-bound
    X = hm.to_fortran(structured_block(W, n, 2 * r, 1, seed=5))
    op64 = hm.KernelOperator(pts, "near", DELTA, hm.HM_F64)
    t64 = _event_time(torch, s, lambda: hm.hm_operator_apply(op64, X, stream=s), 2)
    fl = 2.0 * entries * r
    res["roofline_f64_sampler"] = {"bound": "mfma", "achieved": round(fl / t64 / 1e12, 2),
                                   "peak": PEAK_TF["f64"], "unit": "TFLOP/s",
                                   "frac": round(fl / t64 / 1e12 / PEAK_TF["f64"], 3),
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
    tb = _event_time(torch, s, lambda: hm.hss_apply_backward(h, x, gy, stream=s), 10)
    tf = _event_time(torch, s, lambda: hm.hss_apply(h, x, stream=s), 10)
    # the allocation-free forward apply captured once in a HIP graph and replayed
    y = hm.fortran(n, c, torch.float32)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        hm.hss_apply_noalloc(h, x, y, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    tg = _event_time(torch, s, g.replay, 10)
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
            "fwd_apply_hbm_frac": round(fwd_bytes / tf / 1e9 / PEAK_HBM_GBS, 3),
            "fwd_apply_graph_ms": round(tg * 1e3, 3),
            "apply_config": f"synthetic HBS N={n} leaf={leaf} k={k}, {c} FP32 right-hand sides"}


def solver_measurement(hm, W, torch, h, n):
    """The direct solver on the compressed kernel matrix of the headline
    step (HBS-ID form, N = 65536, leaf 128, k = 32): factor (median of 5),
    solve with 1 and 64 right-hand sides (event-timed on the current stream,
    10 repetitions), and the residual |A_H x - b| / |b| through the apply."""
    f = hm.hbs_factor(h)
    del f
    ts = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = hm.hbs_factor(h)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    s = torch.cuda.current_stream()
    res = {"solver_factor_s": round(float(np.median(ts)), 4)}
    for c in (1, 64):
        b = torch.from_numpy(W.gaussian((n, c), seed=5)).cuda()
        t = _event_time(torch, s, lambda: f.solve(b), 10)
        x = f.solve(b)
        r = float(torch.linalg.norm(h.apply(x) - b) / torch.linalg.norm(b))
        res[f"solver_solve_ms_rhs{c}"] = round(t * 1e3, 3)
        res[f"solver_residual_rhs{c}"] = r
    res["solver_config"] = (f"HBS direct solver on the BF16-sampled HBS-ID form, N={n} "
                            f"leaf={LEAF} k={K}, FP64")
    print(f"solver: factor {res['solver_factor_s'] * 1e3:.1f} ms, solve "
          f"{res['solver_solve_ms_rhs1']:.2f} / {res['solver_solve_ms_rhs64']:.2f} ms "
          f"(1 / 64 rhs), residual {res['solver_residual_rhs64']:.1e}", flush=True)
    return res


def frontal_apply_bytes(H, w, m):
    """Algorithmic bytes of one apply of the frontal black box (Sec. 5.4) to m
    columns: block cyclic reduction over H grid rows on each side, every array
    a kernel touches counted once per kernel.  x read twice (transposed copy,
    output) and its transposed copy written and read once, y written once.
    Per side (wp = w rounded up to 4, right-hand sides wp entries per column):
    levels 1 and 2 run through operators built with the factor -- the
    level-3 right-hand sides come from fifteen x values per row (15 wp FP64
    of operator per row, written once), the level-2 back substitution reads
    its 7 wp operator, gam and del and the level-3 rows' solutions, writes
    the 4-entry projection P and the six projections NP its level-1
    neighbours need (no x: nothing finer reads it); the level-1 back
    substitution reads 9 operator values and its neighbours' NP halves,
    writes P; each level >= 3 reads its active rows' right-hand sides once
    and two w x w matrices per kept row, writes the kept rows; the root and
    each back substitution there read Dinv, gam, del, the right-hand sides,
    the neighbours' solutions and 6 wp of level-1 operator once, write x, P
    and NP; the output kernel reads P, writes y.  (Two levels only: the
    level-2 right-hand sides from seven x values each.)"""
    wp = (w + 3) // 4 * 4
    R, Mb, Pb, NPb, Qb = 8 * wp * m, 8 * w * w, 32 * m, 48 * m, 8 * 6 * wp
    nl = [H]
    while nl[-1] > 1:
        nl.append((nl[-1] + 1) // 2)
    L = len(nl) - 1
    total = 2 * 8 * H * m + 2 * 8 * H * m + 8 * H * m     # x twice, XT, y
    side = 0
    if L == 1:
        side += 8 * (6 * wp + 9) + Pb
    elif L >= 2:
        n1 = nl[1]
        odd1 = n1 // 2
        l1bwd = ((n1 + 1) // 2) * NPb + odd1 * (8 * 9 + Pb)
        if L == 2:
            side += ((n1 + 1) // 2) * (8 * 7 * wp + R) + (R + Mb + Qb + R + Pb + NPb) + l1bwd
        else:
            n2 = nl[2]
            kept2, odd2 = (n2 + 1) // 2, n2 // 2
            side += kept2 * (8 * 15 * wp + R)
            for l in range(3, L):
                kept = (nl[l] + 1) // 2
                side += nl[l] * R + 2 * Mb * kept + kept * R
            side += R + Mb + Qb + R + Pb + NPb
            for l in range(3, L):
                odd = nl[l] // 2
                side += nl[l] * R + odd * (3 * Mb + Qb) + odd * (R + Pb + NPb)
            side += kept2 * R + odd2 * (8 * 7 * wp + 2 * Mb + Qb + Pb + NPb)
            side += l1bwd
    total += 2 * side + 2 * ((H + 1) // 2) * Pb   # both sides; P read by the output
    return float(total)


# Tables 8 and 9 (N = 102400, eps = 1e-9, l = 25): the paper's figures on its
# machine (MATLAB, UMFPACK for the sparse solves), context only
PAPER_FRONTAL = {"hodlr": {"T_compress_s": 468.981, "M_MB": 203.0, "E": 1.30e-14, "k": 9},
                 "hbs": {"T_compress_s": 465.309, "M_MB": 103.1, "E": 4.07e-14, "k": 18}}


def frontal_measurement(hm, W, torch, H=102400, width=41, leaf=100):
    """The frontal matrix of nested dissection (Sec. 5.4): conduction grid of
    H rows and 41 columns, conductivities U[1, 2] (seed 7).  The factor of
    B11 and B22 (median of 3 after a warm-up), one apply to 50 columns (the
    compressions' 2 l columns; event-timed, 10 repetitions) against
    `frontal_apply_bytes`, and the HODLR and HBS-ID compressions of the black
    box at eps = 1e-9, leaf 100 (HODLR: rank cap 20, p = 5, l = 25 samples per
    level as in Table 8; HBS-ID: cap 28, p = 8, its row blocks ranking twice
    the HODLR's): median of 3, the share inside the black box, ranks, storage
    and E = |(A - A_H) X| / |A X| on 10 Gaussian probes, A applied through
    the black box itself."""
    ch, cv = W.grid_conductivities(H, width, seed=7)
    chd = torch.from_numpy(ch).cuda()
    cvd = torch.from_numpy(cv).cuda()
    f = hm.frontal_create(chd, cvd)
    ts = []
    for _ in range(3):
        del f
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = hm.frontal_create(chd, cvd)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    res = {"frontal_factor_ms": round(float(np.median(ts)) * 1e3, 2)}
    m = 50
    s = torch.cuda.current_stream()
    X = torch.randn(m, H, dtype=torch.float64, device="cuda").T
    Y = torch.empty(m, H, dtype=torch.float64, device="cuda").T
    run = lambda: hm.lib.hm_frontal_apply(f.handle, m, X.data_ptr(), H, Y.data_ptr(), H,
                                          C.c_void_p(s.cuda_stream))
    t = _event_time(torch, s, run, 10)
    byts = frontal_apply_bytes(H, (width - 1) // 2, m)
    res["frontal_apply_ms_50cols"] = round(t * 1e3, 3)
    res["frontal_roofline"] = {"bound": "hbm", "achieved": round(byts / t / 1e9, 1),
                               "peak": PEAK_HBM_GBS, "unit": "GB/s",
                               "frac": round(byts / t / 1e9 / PEAK_HBM_GBS, 3),
                               "algorithmic_bytes": byts}
    op = hm.FrontalOperator(f)
    probes = torch.from_numpy(W.gaussian((H, 10), seed=12)).cuda()
    AX = f.apply(probes)
    for kind, k, p in (("hodlr", 20, 5), ("hbs", 28, 8)):
        opts = hm.Options(H, leaf, k, p, tol=1e-9, seed=11)
        comp = hm.hodlr_compress if kind == "hodlr" else hm.hbs_compress
        h = comp(opts, op)
        tt = []
        for _ in range(3):
            del h
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = comp(opts, op)
            torch.cuda.synchronize()
            tt.append(time.perf_counter() - t0)
        inf = h.info()
        e = float(torch.linalg.norm(h.apply(probes) - AX) / torch.linalg.norm(AX))
        res[f"frontal_{kind}"] = {
            "T_compress_s": round(float(np.median(tt)), 4),
            "T_operator_share": round(inf["t_operator_ms"] / inf["t_compress_ms"], 3),
            "operator_calls": inf["operator_calls"], "sample_columns": inf["sample_columns"],
            "k_max": inf["max_rank"], "M_MB": round(inf["storage_reals"] * 8 / 1e6, 1),
            "M_per_N": round(inf["storage_reals"] / H, 1), "E": e,
            "paper": PAPER_FRONTAL[kind]}
        print(f"frontal {kind}: {res[f'frontal_{kind}']['T_compress_s'] * 1e3:.1f} ms, "
              f"k {inf['max_rank']}, E {e:.1e}", flush=True)
        del h
    res["frontal_config"] = (f"conduction grid {H} x {width}, U[1,2] bars (seed 7), FP64; "
                             f"leaf {leaf}, eps 1e-9")
    print(f"frontal: factor {res['frontal_factor_ms']:.1f} ms, apply "
          f"{res['frontal_apply_ms_50cols']:.2f} ms per 50 columns "
          f"({res['frontal_roofline']['frac']:.2f} of HBM)", flush=True)
    return res


def synthetic_hbs_measurement(hm, W, torch, n=16384, leaf=64, k=30, p=10):
    """The FP64 HBS workload: synthetic HBS of rank exactly 30 with nested
    bases (seed 1), N = 16384, leaf 64, p = 10, applied in O(N k) as the
    black box; median of 10 compress calls, exact-recovery error on 8
    Gaussian probes against the operator itself."""
    g = W.synthetic_hbs(n, leaf, k, seed=1)
    op_h = hm.hm_hbs_from_generators(g)
    opts = hm.Options(n, leaf, k, p, seed=1)
    t, h = _median_compress(hm, torch, opts, hm.HBSOperator(op_h), 10)
    x = torch.from_numpy(W.gaussian((n, 8), seed=99))
    y = h.apply(x).cpu().numpy()
    ya = op_h.apply(x).cpu().numpy()
    inf = h.info()
    return {"hbs_f64_n16384_compress_s": round(t, 4),
            "hbs_f64_n16384_t_net_s": round((inf["t_compress_ms"] - inf["t_operator_ms"]) / 1e3, 4),
            "hbs_f64_n16384_rel_err_vs_A": float(np.linalg.norm(y - ya) / np.linalg.norm(ya)),
            "hbs_f64_n16384_ranks": [inf["min_rank"], inf["max_rank"]],
            "hbs_f64_n16384_config": f"synthetic HBS N={n} leaf={leaf} k={k} p={p}, FP64"}


def product_measurement(hm, W, torch, n=16384, leaf=64, k=15, p=10):
    """Recompression of a product of two compressed operators (Sec. 5.2):
    two synthetic HBS of rank 15 (seeds 21, 22), N = 16384, leaf 64; the
    black box applies both in turn, its HBS rank is 30 (compressed with
    k = 30, p = 10); median of 5 calls, error on 8 probes against the
    product itself."""
    d1 = hm.hm_hbs_from_generators(W.synthetic_hbs(n, leaf, k, seed=21))
    d2 = hm.hm_hbs_from_generators(W.synthetic_hbs(n, leaf, k, seed=22))
    op = hm.HBSProductOperator(d1, d2)
    t, h = _median_compress(hm, torch, hm.Options(n, leaf, 2 * k, p, seed=13), op, 5)
    x = torch.from_numpy(W.gaussian((n, 8), seed=99))
    y = h.apply(x)
    ya = hm.hm_operator_apply(op, x)
    inf = h.info()
    return {"hbs_product_n16384_compress_s": round(t, 4),
            "hbs_product_n16384_rel_err": float(torch.linalg.norm(y - ya) / torch.linalg.norm(ya)),
            "hbs_product_n16384_ranks": [inf["min_rank"], inf["max_rank"]],
            "hbs_product_n16384_config": f"product of two synthetic HBS N={n} leaf={leaf} "
                                         f"k={k}, recompressed at k={2 * k} p={p}, FP64"}


def batched_measurement(hm, W, torch, count=256, leaf=128):
    """Many uneven instances: N_i log-uniform in [512, 8192] (multiples of 64),
    k_i uniform in [8, 40] (seed 2), synthetic HBS operators, p_i = min(10,
    48 - k_i), factors stored in FP32; one batched call against one call per
    instance; exact-recovery error of every instance on 4 Gaussian probes."""
    specs = W.batched_instances(count, seed=2)
    ops_h = [hm.hm_hbs_from_generators(W.synthetic_hbs(n, leaf, k, seed=1000 + i))
             for i, (n, k) in enumerate(specs)]
    opts = [hm.Options(n, leaf, k, min(10, 48 - k), seed=2000 + i, store_dtype=hm.HM_F32)
            for i, (n, k) in enumerate(specs)]
    ops = [hm.HBSOperator(h) for h in ops_h]
    hm.hbs_compress_batched(opts[:8], ops[:8])
    res = {}
    for tag, pers in (("", False), ("_persistent_id", True)):
        for o in opts:
            o.c.flags = hm.HM_FLAG_PERSISTENT_ID if pers else 0
        hm.hbs_compress_batched(opts, ops)       # warm-up of this form
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = hm.hbs_compress_batched(opts, ops)
        torch.cuda.synchronize()
        res["batched_s" + tag] = round(time.perf_counter() - t0, 4)
        errs = []
        for (n, _), hh, ho in zip(specs, outs, ops_h):
            x = torch.from_numpy(W.gaussian((n, 4), seed=3))
            y = hh.apply(x).double()
            ya = ho.apply(x)
            errs.append(float(torch.linalg.norm(y - ya) / torch.linalg.norm(ya)))
        res["batched_rel_err_max" + tag] = max(errs)
        if not tag:
            res["batched_rel_err_median"] = float(np.median(errs))
        del outs
    for o in opts:
        o.c.flags = 0
    tb = res["batched_s"]
    t0 = time.perf_counter()
    for o, op in zip(opts, ops):
        h = hm.hbs_compress(o, op)
        del h
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    res.update({"batched_instances": count, "batched_total_n": int(sum(n for n, _ in specs)),
                "batched_instances_per_s": round(count / tb, 1),
                "sequential_s": round(ts, 4), "batched_speedup": round(ts / tb, 2),
                "batched_storage": "fp32"})
    return res


def _threads():
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:  # noqa: BLE001
        return 1


def cpu_baseline(W, n=32768):
    """The FP64 oracle's full compression (Fig. 4 + Fig. 5, NumPy/LAPACK) of
    the benchmark workload at N = 32768 (same curve law, kernel, leaf, k, p,
    seeds; L = 8), one run, on the host's cores (row tiles of the kernel
    product on one thread each, BLAS single-threaded inside them); GFLOP/s by
    the same method flop count as ``value``."""
    from oracle import hbs as ohbs
    from oracle import operators as oops
    from threadpoolctl import threadpool_limits
    cores = len(os.sched_getaffinity(0))
    pts = W.fourier_curve_points(n, seed=SEED_PTS)
    op = oops.KernelOp(pts, "near", DELTA, workers=cores)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        ohbs.compress(op, n, LEAF, K + P, SEED, rank=K)
        dt = time.perf_counter() - t0
    return {"value": round(method_flops(n, LEAF, K + P) / dt / 1e9, 2), "unit": "GFLOP/s",
            "cores": cores, "kind": "oracle",
            "sample": f"oracle's full HBS-ID compression of the benchmark workload at N={n} "
                      f"(leaf {LEAF}, k {K}, p {P}; {dt:.1f} s, {cores} threads); FP64 NumPy"}


def cpu_product_sample(W, n):
    """The oracle's operator product (the dominant step) on a bounded sample:
    1024 of the N rows against all N columns and 96 columns, in GFLOP/s of
    a dense product."""
    from oracle import operators as oops
    pts = W.fourier_curve_points(n, seed=SEED_PTS)
    X = W.gaussian((n, 96), seed=5)
    sub = oops.KernelOp(pts, "near", DELTA, tile=256)
    t0 = time.perf_counter()
    done = 0
    for i0 in range(0, 1024, 256):
        idx = np.arange(i0, min(i0 + 256, 1024))
        _ = sub.entries(idx, np.arange(n)) @ X
        done += len(idx)
    dt = time.perf_counter() - t0
    return {"value": round(2.0 * done * n * 96 / dt / 1e9, 2), "unit": "GFLOP/s",
            "cores": int(_threads()),
            "sample": f"{done} of {n} rows x {n} columns x 96 columns ({dt:.1f} s)"}


if __name__ == "__main__":
    main()
