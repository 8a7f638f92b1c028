#!/usr/bin/env python3
"""Benchmark of the CP-ALS hot path on one MI355X.

Workload: order-4 dense tensor 128^4 in FP32 (synthetic: planted rank-64
factors iid Uniform[0,1) plus Gaussian noise at 1% of the norm), CP rank
R = 64, factors initialised iid Uniform[0,1), all generated from a seed.

One step = one pass of the whole hot path from the same initial factors:
  DT    3 sweeps with the standard dimension tree (2 first-level TTMs each)
  MSDT  3 sweeps with the multi-sweep dimension tree (one whole tree: 4 TTMs)
  PP    PP-ALS on the MSDT plan: 1 regular sweep, PP initialization plus one
        approximated sweep, then 3 approximated sweeps (a fixed schedule)
Every sweep runs Gamma / inverse / solve / Gram / residual in FP64 on the
GPU.  `value` is the step's effective throughput: each sweep is credited the
flops of one standard-DT sweep of this workload, divided by the step time.

Prints one JSON line on stdout; everything else goes to stderr.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}  # MI355X dense matrix-core peaks
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def dt_sweep_flops(dims, R):
    """Flops of one standard dimension-tree sweep (2 flops per multiply-add):
    replay the tree's paths with node reuse, charging 2*numel(T)*R for a
    first-level contraction and 2*numel(X) for a batched TTV out of node X."""
    N = len(dims)

    def prod(xs):
        out = 1
        for x in xs:
            out *= x
        return out

    def path(n):
        lo, hi, out = 0, N - 1, []
        while lo < hi:
            mid = lo + (hi - lo + 2) // 2 - 1
            if n <= mid:
                out += list(range(hi, mid, -1))
                hi = mid
            else:
                out += list(range(lo, mid + 1))
                lo = mid + 1
        return out

    numel = prod(dims)
    ver = [0] * N
    cache = {}
    flops = 0
    for n in range(N):
        seq = path(n)
        sets, kept = [], frozenset(range(N))
        for m in seq:
            kept = kept - {m}
            sets.append(kept)

        def stamp(s):
            return tuple(ver[c] for c in range(N) if c not in s)

        start = -1
        for d in range(len(sets) - 2, -1, -1):
            if cache.get(sets[d]) == stamp(sets[d]):
                start = d
                break
        prev = frozenset(range(N)) if start < 0 else sets[start]
        for d in range(start + 1, len(sets)):
            flops += 2 * numel * R if d == 0 else 2 * R * prod(dims[k] for k in prev)
            prev = sets[d]
            if d < len(sets) - 1:
                cache[sets[d]] = stamp(sets[d])
        ver[n] += 1
    return flops


# the source that decides the first-level contraction's HBM traffic: its two
# kernels and their launchers (text from each marker to the end of that function)
TTM_SOURCE_MARKERS = (
    "__global__ __launch_bounds__(512) void k_ttm_kc(",
    "__global__ __launch_bounds__(512) void k_ttm_kc32(",
    "__global__ __launch_bounds__(512) void k_ttm_q(",
    "hipError_t launch_ttm_kc(",
    "hipError_t launch_ttm_kc32(",
    "hipError_t launch_ttm_q(",
    "hipError_t launch_ttm(const T* X",
)


def kernel_sha():
    """SHA-256 of the first-level contraction's kernels and launchers in
    kernels.hip (counters taken on other source stay valid when the rest of
    the file changes)."""
    with open(os.path.join(ROOT, "paper_2010_12056_amd", "csrc", "kernels.hip")) as f:
        src = f.read()
    h = hashlib.sha256()
    for m in TTM_SOURCE_MARKERS:
        i = src.find(m)
        if i < 0:
            raise RuntimeError(f"kernels.hip: {m!r} not found")
        j = src.find("\n}\n", i)
        h.update(src[i:j + 3].encode())
    return h.hexdigest()


def load_traffic(sha):
    """HBM bytes per first-level-contraction launch from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "ttm_o4_s128_r64_f32_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("ttm_source_sha256") != sha:
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(w, budget_s, dt_flops):
    """The FP64 oracle (test infrastructure) on the host cores: exact ALS
    sweeps (naive explicit-KRP MTTKRP) on the same tensor and init, as many
    as fit in the budget (at least one)."""
    import numpy as np

    import oracle

    try:
        from threadpoolctl import threadpool_info

        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    T64 = w.T.astype(np.float64)
    st = oracle.AlsState.start(T64, w.init)
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.als_sweep(st)
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= 8:
            break
    dt = time.perf_counter() - t0
    return {
        "value": n * dt_flops / dt / 1e12,
        "unit": "TFLOP/s (DT-equivalent)",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"{n} exact FP64 ALS sweep(s) of the oracle (explicit-KRP MTTKRP) on the same "
                  f"128^4 tensor and init, {dt:.2f} s, {dt / n * 1e3:.1f} ms/sweep",
        "ms_per_sweep": dt / n * 1e3,
    }


PRECISION_WORKLOAD = "o3_s1024_r128_bf16"


def precision_bench(args):
    """The precision path: order-3 1024^3 tensor stored in BF16 (planted
    rank-128 N(0,1) factors with column norms spread log-uniformly over
    [1e-2, 1], noise 1e-3 of the norm; the FP32 copy is the FP32 plan's
    input), R = 128.  Times DT and MSDT sweeps for FP32, BF16 and BF16X2
    plans, reports the first-contraction kernel against the HBM roofline, and
    states the error of each BF16 path against the FP64 oracle run on the same
    BF16 values: the oracle's exact fitness of the GPU's own factors after each
    of the first sweeps (resynced), and sampled MTTKRP rows."""
    import numpy as np
    import torch

    import oracle
    from oracle import core
    from paper_2010_12056_amd import cpals, synth

    dev = torch.device("cuda:0")
    dims, R = (1024, 1024, 1024), 128
    t_gen = time.perf_counter()
    w = synth.planted_tensor(dims, R, 3001, kind="lognorm", noise_rel=1e-3, dtype=np.float32)
    bits = synth.bf16_bits(w.T)
    fp8_scale = synth.fp8_scale(w.T)  # the FP8 copy is the tensor times this power of two
    bits8 = synth.fp8_bits(w.T, scale=fp8_scale)
    log(f"[bench] generated {PRECISION_WORKLOAD} in {time.perf_counter() - t_gen:.1f}s")
    T32 = torch.from_numpy(w.T).to(dev)
    Tb = torch.from_numpy(bits.view(np.int16)).to(dev).view(torch.bfloat16)
    T8 = torch.from_numpy(bits8).to(dev).view(torch.float8_e4m3fn)
    tensors = {"f32": T32, "bf16": Tb, "bf16x2": Tb, "fp8": T8, "fp8x2": T8}
    A0 = [torch.from_numpy(a).to(dev) for a in w.init]
    numel = int(np.prod(dims))
    stream = torch.cuda.current_stream(dev)
    res = {}
    for prec in ("f32", "bf16", "bf16x2", "fp8", "fp8x2"):
        T = tensors[prec]
        out = {}
        for tree, nsw in (("dt", 3), ("msdt", 4)):
            plan = cpals.Plan(dims, R, prec=prec, tree=tree, device=dev)
            plan.set_tensor(T)
            A = [a.clone() for a in A0]
            for a, a0 in zip(A, A0):
                a.copy_(a0)
            plan.reset()
            plan.als_sweep(A, info=False)  # warm
            for a, a0 in zip(A, A0):
                a.copy_(a0)
            plan.reset()
            plan.profile(True, phases=("ttm",))
            plan.profile_read()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(nsw):
                plan.als_sweep(A, info=False)
            e1.record(stream)
            torch.cuda.synchronize()
            ph = plan.profile_read()
            plan.profile(False)
            ttm_ms, ttm_n = ph["ttm"]
            out[tree] = {"ms_per_sweep": round(e0.elapsed_time(e1) / nsw, 4),
                         "ttm_avg_ms": round(ttm_ms / max(ttm_n, 1), 5), "ttm_launches": ttm_n}
            plan.close()
        res[prec] = out
        log(f"[bench] {prec}: {out}")
    # roofline of the BF16 first contraction: tensor read once, FP32 output written once
    esz = 2
    out_bytes = (numel // dims[0]) * R * 4
    ttm_ms = res["bf16x2"]["dt"]["ttm_avg_ms"]
    achieved = (numel * esz + out_bytes) / (ttm_ms * 1e-3) / 1e9
    ttm8_ms = res["fp8x2"]["dt"]["ttm_avg_ms"]
    achieved8 = (numel + out_bytes) / (ttm8_ms * 1e-3) / 1e9
    ttm8s_ms = res["fp8"]["dt"]["ttm_avg_ms"]
    achieved8s = (numel + out_bytes) / (ttm8s_ms * 1e-3) / 1e9
    # error against the FP64 oracle on the stored BF16 / FP8 values, resynced per sweep
    log("[bench] oracle checks")
    errs = {}
    for prec in ("bf16", "bf16x2", "fp8", "fp8x2"):
        if prec == "bf16":
            T64 = synth.bf16_to_f32(bits).astype(np.float64)
            del bits
            normT2 = float(np.sum(T64 * T64))
        elif prec == "fp8":
            del T64
            T64 = synth.fp8_to_f32(bits8).astype(np.float64)
            del bits8
            normT2 = float(np.sum(T64 * T64))
        plan = cpals.Plan(dims, R, prec=prec, tree="dt", device=dev)
        plan.set_tensor(tensors[prec])
        A = [a.clone() for a in A0]
        rows = np.random.default_rng(0).choice(dims[0], 4, replace=False)
        M = plan.mttkrp(A, 0).cpu().numpy()[rows]
        K = core.krp([w.init[1], w.init[2]])
        X0 = T64.reshape(dims[0], -1)
        ref = X0[rows] @ K
        refabs = np.abs(X0[rows]) @ core.krp([np.abs(w.init[1]), np.abs(w.init[2])])
        del K
        unit = 2.0 ** -8 if prec in ("bf16", "fp8") else 2.0 ** -16  # the factor's rounding; the tensor is exact
        rec = {"mttkrp_rows_relerr": float(np.linalg.norm(M - ref) / np.linalg.norm(ref)),
               "mttkrp_rows_err_over_bound": float(np.max(np.abs(M - ref) / (unit * refabs))),
               "sweeps": []}
        plan.reset()
        for sweep in range(3):
            info = plan.als_sweep(A)
            Ah = [a.cpu().numpy() for a in A]
            S = [core.gram(a) for a in Ah]
            M0 = X0 @ core.krp([Ah[1], Ah[2]])
            r_or = core.residual_fast(normT2, core.gamma(S, 0), S[0], M0, Ah[0])
            rec["sweeps"].append({"gpu_fitness": info["fitness"], "oracle_fitness_same_factors": 1.0 - r_or,
                                  "abs_err": abs(info["fitness"] - (1.0 - r_or))})
            del M0
        errs[prec] = rec
        log(f"[bench] {prec} error vs oracle: {rec}")
        plan.close()
    line = {
        "metric": "ALS sweep ms, order-3 1024^3 R=128: BF16 / split-BF16 first contraction vs FP32",
        "value": res["bf16x2"]["msdt"]["ms_per_sweep"],
        "unit": "ms per MSDT sweep (BF16X2)",
        "n_gpus": 1,
        "higher_is_better": False,
        "vs_baseline": None,
        "dtype": "bf16x2 (first contraction), f32 levels, f64 solve",
        "data": "synthetic",
        "config": {"workload": "order-3 dense 1024x1024x1024 stored BF16 (and FP8 E4M3 after a power-of-two scale), planted rank-128 N(0,1) factors with "
                               "log-uniform column norms in [1e-2, 1], noise 1e-3, CP rank 128",
                   "dims": list(dims), "rank": R, "fp8_tensor_scale": fp8_scale},
        "by_precision": res,
        "speedup_bf16x2_vs_f32_msdt": round(res["f32"]["msdt"]["ms_per_sweep"] / res["bf16x2"]["msdt"]["ms_per_sweep"], 3),
        "speedup_fp8x2_vs_f32_msdt": round(res["f32"]["msdt"]["ms_per_sweep"] / res["fp8x2"]["msdt"]["ms_per_sweep"], 3),
        "roofline_fp8": {"kernel": "k_ttm_bf16 (FP8 tensor, BF16 factor, first contraction)", "bound": "hbm",
                         "achieved": round(achieved8s, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(achieved8s / PEAK_HBM_GBS, 4), "traffic": None,
                         "bytes_per_launch": numel + out_bytes, "avg_launch_ms": ttm8s_ms},
        "roofline_fp8x2": {"kernel": "k_ttm_bf16 (FP8 tensor, split factor, first contraction)", "bound": "hbm",
                           "achieved": round(achieved8, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                           "frac": round(achieved8 / PEAK_HBM_GBS, 4), "traffic": None,
                           "bytes_per_launch": numel + out_bytes, "avg_launch_ms": ttm8_ms},
        "roofline": {"kernel": "k_ttm_bf16 (BF16X2, first contraction)", "bound": "hbm",
                     "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                     "bytes_per_launch": numel * esz + out_bytes, "avg_launch_ms": ttm_ms},
        "error_vs_fp64_oracle": errs,
    }
    print(json.dumps(line), flush=True)


BATCH_WORKLOAD = "batch512_o3"


def batch_bench(args):
    """The batched path: 512 independent order-3 FP32 tensors, each mode size
    iid uniform on [16, 96], rank uniform over {4, 8, 16, 32}, planted iid
    Uniform[0,1) factors plus noise 1e-3 of the norm; 30 ALS sweeps of every
    tensor per step in one persistent launch, replayed from a captured HIP
    graph (factors reset from the initial ones before each replay, outside the
    graph).  Launch shape from the autotuner's cache (tuned now if absent)."""
    import numpy as np
    import torch

    from paper_2010_12056_amd import autotune, cpals, synth

    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    ws = synth.batch_workload(512, seed=5001)
    log(f"[bench] generated {BATCH_WORKLOAD} in {time.perf_counter() - t_gen:.1f}s")
    dims = [w.dims for w in ws]
    ranks = [w.R for w in ws]
    tuned = autotune.lookup(dims, ranks)
    source = "cache"
    if tuned is None:
        tuned = autotune.tune(ws, write=False, log=log)
        source = "tuned now"
    log(f"[bench] launch shape {tuned['waves']} waves x {tuned['groups_per_cu']} groups/CU ({source})")
    sweeps = 30
    b = cpals.Batch(dims, ranks, device=dev, waves=tuned["waves"], groups_per_cu=tuned["groups_per_cu"])
    T = b.pack_tensors([w.T for w in ws])
    A0 = b.pack_factors([w.init for w in ws])
    A = A0.clone()
    fit = torch.empty((len(ws), sweeps), dtype=torch.float64, device=dev)
    status = torch.empty(len(ws), dtype=torch.int32, device=dev)
    ticks = torch.empty((len(ws), 2), dtype=torch.int64, device=dev)
    b.sweeps(T, A, sweeps, fitness=fit, status=status, ticks=ticks)  # eager warm-up
    torch.cuda.synchronize()
    s = torch.cuda.Stream(dev)
    s.wait_stream(torch.cuda.current_stream(dev))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        bg = cpals.Batch(dims, ranks, device=dev, waves=tuned["waves"], groups_per_cu=tuned["groups_per_cu"])
        with torch.cuda.graph(g, stream=s):
            bg.sweeps(T, A, sweeps, fitness=fit, status=status, ticks=ticks)
    torch.cuda.current_stream(dev).wait_stream(s)
    for _ in range(args.warmup):
        A.copy_(A0)
        g.replay()
    torch.cuda.synchronize()
    ms = []
    for _ in range(args.steps):
        A.copy_(A0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    ms_step = float(np.mean(ms))
    hz = b.tick_rate()
    tk = ticks.cpu().numpy()
    lat_us = (tk[:, 1] - tk[:, 0]) / hz / sweeps * 1e6  # per-tensor sweep latency
    st = status.cpu().numpy()
    f = fit.cpu().numpy()
    # algorithmic work per launch: every sweep reads each tensor twice (two first-level
    # contractions) and does 2 * 2 * s0 s1 s2 R matrix-core flops
    bytes_launch = sum(2 * w.T.size * 4 for w in ws) * sweeps
    flops_launch = sum(4 * w.T.size * w.R for w in ws) * sweeps
    achieved_gbs = bytes_launch / (ms_step * 1e-3) / 1e9
    # oracle spot check: 4 tensors, fitness after the first 3 sweeps of this run
    import oracle

    chk = []
    for i in (0, 100, 300, 511):
        sto = oracle.AlsState.start(ws[i].T.astype(np.float64), ws[i].init)
        r = [oracle.als_sweep(sto) for _ in range(3)]
        chk.append(max(abs(f[i, k] - (1.0 - r[k])) for k in range(3)))
    line = {
        "metric": "batched CP-ALS: tensors/s and per-tensor sweep latency, 512 order-3 tensors s in [16,96], "
                  "R in {4,8,16,32}, 30 sweeps each",
        "value": round(len(ws) / (ms_step * 1e-3), 1),
        "unit": "tensors/s (30 sweeps each)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "vs_baseline": None,
        "dtype": "f32 (contractions), f64 (solve, Gram, residual)",
        "data": "synthetic",
        "config": {"workload": "512 independent order-3 dense FP32 tensors, modes iid U[16,96], R iid from "
                               "{4,8,16,32}, planted U[0,1) factors + 1e-3 noise, 30 sweeps, one persistent "
                               "launch replayed from a HIP graph",
                   "launch": {"waves_per_group": tuned["waves"], "groups_per_cu": tuned["groups_per_cu"],
                              "source": source}},
        "latency_us_per_sweep": {"p50": round(float(np.percentile(lat_us, 50)), 2),
                                 "p99": round(float(np.percentile(lat_us, 99)), 2),
                                 "max": round(float(lat_us.max()), 2)},
        "status_nonzero": int(np.count_nonzero(st)),
        "oracle_fitness_max_abs_err_first3": float(max(chk)),
        "roofline": {"kernel": "k_batch (persistent, all sweeps of all tensors)", "bound": "hbm",
                     "achieved": round(achieved_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved_gbs / PEAK_HBM_GBS, 4), "traffic": None,
                     "bytes_per_launch": bytes_launch, "flops_per_launch": flops_launch,
                     "mfma_tflops": round(flops_launch / (ms_step * 1e-3) / 1e12, 2)},
    }
    b.close()
    bg.close()
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="o4_s128_r64_f32")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--counters-workload", action="store_true",
                    help="run only what the HBM-counter passes read: one MTTKRP per first-level layout "
                         "on the workload, then a plain 512 MiB device copy as the calibration kernel")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the multi-GPU decomposition (a processor grid with "
              "collectives) is not implemented, so --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2010_12056_amd import cpals, synth

    if not os.path.exists(cpals.LIB_PATH):
        from paper_2010_12056_amd import build_lib

        build_lib.build()
    if args.workload == PRECISION_WORKLOAD:
        precision_bench(args)
        return
    if args.workload == BATCH_WORKLOAD:
        batch_bench(args)
        return
    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    w = synth.workload(args.workload)
    log(f"[bench] generated {args.workload} dims={w.dims} R={w.R} in {time.perf_counter() - t_gen:.1f}s")
    prec = "f32" if w.T.dtype == np.float32 else "f64"
    T = torch.from_numpy(w.T).to(dev)
    A0 = [torch.from_numpy(a).to(dev) for a in w.init]
    N = len(w.dims)
    R = w.R
    F_dt = dt_sweep_flops(w.dims, R)
    numel = int(np.prod(w.dims))
    ttm_flops = 2 * numel * R
    if args.counters_workload:
        plan = cpals.Plan(w.dims, R, prec=prec, tree="dt", device=dev)
        plan.set_tensor(T)
        for mode in (0, N - 1):  # first-level contraction over the last mode, then over mode 0
            plan.mttkrp(A0, mode)
        torch.cuda.synchronize()
        src = torch.empty(128 * 2**20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)  # calibration: reads and writes exactly 512 MiB each
        torch.cuda.synchronize()
        log("[bench] counters workload done")
        return

    plans = {
        "dt": cpals.Plan(w.dims, R, prec=prec, tree="dt", device=dev),
        "msdt": cpals.Plan(w.dims, R, prec=prec, tree="msdt", device=dev),
    }
    plans["pp"] = plans["msdt"]
    for k in ("dt", "msdt"):
        plans[k].set_tensor(T)
    A = {k: [a.clone() for a in A0] for k in ("dt", "msdt", "pp")}
    pp_sched = ["exact", "init", "approx", "approx", "approx"]
    sweeps = {"dt": 3, "msdt": N - 1, "pp": len(pp_sched)}
    stream = torch.cuda.current_stream(dev)

    def one_step(ev=None):
        for k in ("dt", "msdt", "pp"):
            plan = plans[k]
            for a, a0 in zip(A[k], A0):
                a.copy_(a0)
            plan.reset()
            if ev is not None:
                ev[k][0].record(stream)
            if k == "pp":
                for kind in pp_sched:
                    plan.pp_sweep(A[k], mode=kind, info=False)
            else:
                for _ in range(sweeps[k]):
                    plan.als_sweep(A[k], info=False)
            if ev is not None:
                ev[k][1].record(stream)

    log("[bench] warmup")
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    # per-kind timing of single sweeps (reported breakdown, separate from the timed steps)
    log("[bench] timed region")
    # inside the timed region only the first-level contractions of the last
    # timed step carry event pairs (their average launch time feeds the
    # roofline; each pair costs device time); the other phases are timed on
    # one more step afterwards
    for k in ("dt", "msdt"):
        plans[k].profile(False)
        plans[k].profile_read()
    evs = [{k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for k in ("dt", "msdt", "pp")} for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        if s == args.steps - 1:
            for k in ("dt", "msdt"):
                plans[k].profile(True, phases=("ttm",))
        one_step(evs[s])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    timed_phase = {}
    for k in ("dt", "msdt"):
        for ph, (ms, cnt) in plans[k].profile_read().items():
            a, b = timed_phase.get(ph, (0.0, 0))
            timed_phase[ph] = (a + ms, b + cnt)
        plans[k].profile(True)  # every phase, for the breakdown step
        plans[k].profile_read()
    one_step()
    phase = {}
    for k in ("dt", "msdt"):
        for ph, (ms, cnt) in plans[k].profile_read().items():
            a, b = phase.get(ph, (0.0, 0))
            phase[ph] = (a + ms, b + cnt)
        plans[k].profile(False)
    var_ms = {k: sum(e[k][0].elapsed_time(e[k][1]) for e in evs) / args.steps for k in ("dt", "msdt", "pp")}
    log(f"[bench] {args.steps} steps, {ms_step:.3f} ms/step; variants {var_ms}")

    # fitness check of the last step's factors against the DT run (same math)
    infos = {}
    for k in ("dt", "msdt"):
        plans[k].reset()
        for a, a0 in zip(A[k], A0):
            a.copy_(a0)
        infos[k] = [plans[k].als_sweep(A[k])["fitness"] for _ in range(3)]
    log(f"[bench] fitness dt {infos['dt']} msdt {infos['msdt']}")

    # PP: one timed breakdown per sweep kind on the MSDT plan
    plan = plans["pp"]
    plan.reset()
    for a, a0 in zip(A["pp"], A0):
        a.copy_(a0)
    kind_ms = {}
    for kind in pp_sched:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.pp_sweep(A["pp"], mode=kind, info=False)
        e1.record(stream)
        torch.cuda.synchronize()
        kind_ms.setdefault(kind, []).append(e0.elapsed_time(e1))

    # the dimension tree with its upper two levels combined (order >= 4): timed
    # on its own, outside the step, against the DT plan's sweeps
    comb = None
    if N >= 4:
        pc = cpals.Plan(w.dims, R, prec=prec, tree="dt_combined", device=dev)
        pc.set_tensor(T)
        Ac = [a.clone() for a in A0]
        c_ms = []
        for rep in range(1 + args.steps):
            pc.reset()
            for a, a0 in zip(Ac, A0):
                a.copy_(a0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(3):
                pc.als_sweep(Ac, info=False)
            e1.record(stream)
            torch.cuda.synchronize()
            if rep:
                c_ms.append(e0.elapsed_time(e1) / 3)
        pc.reset()
        for a, a0 in zip(Ac, A0):
            a.copy_(a0)
        c_fit = [pc.als_sweep(Ac)["fitness"] for _ in range(3)]
        pc.close()
        comb = {"ms_per_sweep": float(np.mean(c_ms)), "fitness": c_fit}
        log(f"[bench] dt_combined {comb}")

    n_sweeps = sum(sweeps.values())
    value = n_sweeps * F_dt / (ms_step * 1e-3) / 1e12
    ttm_ms, ttm_n = timed_phase["ttm"]
    ttm_avg_ms = ttm_ms / max(ttm_n, 1)
    achieved = ttm_flops / (ttm_avg_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
    sha = kernel_sha()
    traffic = load_traffic(sha) if args.workload == "o4_s128_r64_f32" else None
    variants = {}
    for k in ("dt", "msdt", "pp"):
        per = var_ms[k] / sweeps[k]
        variants[k] = {"sweeps": sweeps[k], "ms_per_sweep": round(per, 4),
                       "effective_tflops": round(F_dt / (per * 1e-3) / 1e12, 3)}
    variants["pp"]["ms_by_kind"] = {k: round(float(np.mean(v)), 4) for k, v in kind_ms.items()}
    variants["msdt"]["speedup_vs_dt"] = round(variants["dt"]["ms_per_sweep"] / variants["msdt"]["ms_per_sweep"], 3)
    variants["pp"]["approx_speedup_vs_dt"] = round(
        variants["dt"]["ms_per_sweep"] / variants["pp"]["ms_by_kind"]["approx"], 3)
    if comb is not None:
        variants["dt_combined"] = {
            "sweeps": 3, "ms_per_sweep": round(comb["ms_per_sweep"], 4),
            "effective_tflops": round(F_dt / (comb["ms_per_sweep"] * 1e-3) / 1e12, 3),
            "speedup_vs_dt": round(variants["dt"]["ms_per_sweep"] / comb["ms_per_sweep"], 3),
            "fitness_3_sweeps": comb["fitness"][-1],
            "timed": "separately, not part of the step"}

    headline = args.workload == "o4_s128_r64_f32"
    cfg = synth.WORKLOADS[args.workload]
    desc = (f"order-{N} dense {'x'.join(map(str, w.dims))} {prec.upper()}, planted rank-{R} {cfg['kind']} factors"
            f" + {cfg['noise_rel']:g} noise{', clipped at zero' if cfg.get('nonneg') else ''}, CP rank {R}")
    out = {
        "metric": ("ALS sweep ms & effective TFLOP/s, order-4 s=128 R=64: MSDT/PP vs plain DT" if headline else
                   f"ALS sweep ms & effective TFLOP/s, {args.workload} ({'x'.join(map(str, w.dims))}, R={R}):"
                   " MSDT/PP vs plain DT"),
        "value": round(value, 3),
        "unit": "TFLOP/s (effective: DT-sweep flops per sweep / time)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": desc,
                   "dims": list(w.dims), "rank": R, "sweeps_per_step": n_sweeps,
                   "dt_sweep_gflop": round(F_dt / 1e9, 3), "parallelism": "1 GPU"},
        "variants": variants,
        "phase_ms_per_step": {k: round(v[0], 4) for k, v in phase.items()},
        "phase_note": "one extra step with every phase timed (its event pairs make it slower than a timed step)",
        "fitness_3_sweeps": {"dt": infos["dt"][-1], "msdt": infos["msdt"][-1]},
        "roofline": {
            "kernel": "k_ttm (first-level contraction, FP32 MFMA)",
            "bound": "mfma",
            "achieved": round(achieved, 3),
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": traffic,
            "avg_launch_ms": round(ttm_avg_ms, 5),
            "launches": ttm_n,
            "flops_per_launch": ttm_flops,
        },
        "cpu_baseline": None,
    }
    for p in (plans["dt"], plans["msdt"]):
        p.close()
    del T
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget, F_dt)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
