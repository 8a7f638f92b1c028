#!/usr/bin/env python3
"""Benchmark of the CP-ALS hot path on one MI355X.

Workload: order-4 dense tensor 128^4 in FP32 (synthetic: planted rank-64
factors iid Uniform[0,1) plus Gaussian noise at 1% of the norm), CP rank
R = 64, factors initialised iid Uniform[0,1), all generated from a seed.

One step = one pass of the whole hot path from the same initial factors, the
three methods run to the same fitness:
  DT    10 sweeps with the standard dimension tree (2 first-level TTMs each)
  MSDT  10 sweeps with the multi-sweep dimension tree (N TTMs per N-1 sweeps),
        the same update order, so the same fitness up to rounding
  PP    PP-ALS (Alg. 2 with its own activation test, tolerance 0.1) on the
        MSDT plan, for the outer steps it needs to reach the DT run's final
        exact fitness less 1e-4 (counted once by an audited, untimed run)
Every sweep runs Gamma / inverse / solve / Gram / residual in FP64 on the
GPU.  `value` is the step's effective throughput: each run is credited the
flops the standard DT needs to reach the common fitness, divided by the step
time.  Other workloads (--workload): the order-3 64^3 FP64 tensor (20
sweeps), the precision path, the batched path, shape stand-ins.

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
    "__global__ __launch_bounds__(512) void k_ttm_kc32f(",
    "hipError_t launch_ttm_kc_fused(",
    "__global__ __launch_bounds__(512) void k_ttm_qg(",
    "hipError_t launch_ttm_qg_ncb(",
    "hipError_t launch_ttm_qg(",
    "hipError_t launch_kc32f(",
    "__global__ __launch_bounds__(512) void k_ttm_qr(",
    "hipError_t launch_ttm_qr_ncb(",
    "hipError_t launch_ttm_qr(",
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


# sweeps of the DT and MSDT runs per workload (the PP run goes on until it
# reaches the DT run's final exact fitness less TARGET_SLACK)
TREE_SWEEPS = {"o4_s128_r64_f32": 10, "o3_s64_r16_f64": 20}
# a longer run for the PP comparison, timed outside the step
LONG_SWEEPS = {"o4_s128_r64_f32": 30}
PP_TOL = 0.1  # Alg. 2 tolerance (the paper's value for its application tensors, Sec. V-C)
TARGET_SLACK = 1e-4
PP_MAX_STEPS = 60


def oracle_timings(w, budget_s, pp_start, target_sweeps):
    """The FP64 oracle (test infrastructure) on the host cores, on bounded
    samples of the same workload: naive explicit-KRP ALS sweeps from the same
    init (their fitness is compared with the GPU's), oracle-DT and
    oracle-MSDT sweeps (MTTKRPs through its tree cache), and one PP
    initialization plus one approximated step of its Alg. 2, started from the
    GPU run's factors where Alg. 2 entered PP."""
    import numpy as np

    import oracle
    from oracle import pp, trees

    try:
        from threadpoolctl import threadpool_info

        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    T64 = w.T.astype(np.float64)
    N = T64.ndim
    out = {"threads": int(threads)}
    st = oracle.AlsState.start(T64, w.init)
    rs = []
    t0 = time.perf_counter()
    while len(rs) < target_sweeps and (not rs or time.perf_counter() - t0 < budget_s):
        rs.append(oracle.als_sweep(st))
    out["naive"] = {"sweeps": len(rs), "ms_per_sweep": (time.perf_counter() - t0) / len(rs) * 1e3,
                    "fitness": [1.0 - r for r in rs]}
    del st
    for kind in ("dt", "msdt"):
        st = oracle.AlsState.start(T64, w.init)
        cache = trees.DTCache(T64, st.A)
        n_sw, u = 0, 0
        t0 = time.perf_counter()
        while n_sw < 3 and (n_sw == 0 or time.perf_counter() - t0 < budget_s / 2):
            paths = [trees.dt_path(N, n) if kind == "dt" else trees.msdt_path(N, u + n) for n in range(N)]
            trees.als_sweep_tree(st, cache, paths)
            u += N
            n_sw += 1
        out[kind] = {"sweeps": n_sw, "ms_per_sweep": (time.perf_counter() - t0) / n_sw * 1e3}
        del st, cache
    if pp_start is not None:
        st = pp.PPState.start(T64, pp_start)
        st.dA = [np.zeros_like(a) for a in st.A]  # entered from a passing test: no carried change
        t0 = time.perf_counter()
        pp.pp_als_step(st, force="init")
        t1 = time.perf_counter()
        pp.pp_als_step(st, force="approx")
        t2 = time.perf_counter()
        out["pp"] = {"init_step_ms": (t1 - t0) * 1e3, "approx_step_ms": (t2 - t1) * 1e3,
                     "note": "the oracle's approximated step includes its exact-fitness audit (one naive MTTKRP)"}
    return out


def tree_bench(args):
    """DT, MSDT and PP (Alg. 2) on one workload, at equal final fitness.

    One step, from the same initial factors each time:
      DT    TREE_SWEEPS sweeps with the standard dimension tree (Sec. II-C);
      MSDT  as many sweeps with the multi-sweep dimension tree (Sec. III),
            bit-for-bit the same update order;
      PP    Alg. 2 (tolerance PP_TOL, its own activation test) on the MSDT
            plan, for the number of outer steps it needs to reach the DT run's
            final exact fitness less TARGET_SLACK (found once beforehand by an
            untimed run whose every step is audited with cp_fitness; the timed
            runs repeat that trajectory bit for bit, checked at the end).
    `value` credits each run with the DT flops that reach the target fitness
    (TREE_SWEEPS DT sweeps for DT and MSDT; the DT sweeps to target for PP),
    divided by the step time."""
    import numpy as np
    import torch

    from paper_2010_12056_amd import cpals, synth

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
        # each first-level kernel of the step: the standard tree's fused
        # halves (a DT plan's MTTKRPs of modes 0 and N-1), the first-level-only
        # kernels (rooted MTTKRPs whose second contraction no fused kernel
        # takes: the last mode then mode 1, mode 0 then mode 2), and MSDT's
        # fused roots that also store the node (three MSDT sweeps: roots N-1,
        # the middle modes and 0)
        plan = cpals.Plan(w.dims, R, prec=prec, tree="dt", device=dev)
        plan.set_tensor(T)
        for mode in (0, N - 1):
            plan.mttkrp(A0, mode)
        plan.mttkrp(A0, 0, root=N - 1)
        plan.mttkrp(A0, 1, root=0)
        torch.cuda.synchronize()
        plan.close()
        plan = cpals.Plan(w.dims, R, prec=prec, tree="msdt", device=dev)
        plan.set_tensor(T)
        Am = [a.clone() for a in A0]
        for _ in range(N - 1):
            plan.als_sweep(Am, info=False)
        torch.cuda.synchronize()
        plan.close()
        src = torch.empty(128 * 2**20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)  # calibration: reads and writes exactly 512 MiB each
        torch.cuda.synchronize()
        log("[bench] counters workload done")
        return
    n_sw = TREE_SWEEPS.get(args.workload, 10)
    plans = {"dt": cpals.Plan(w.dims, R, prec=prec, tree="dt", device=dev),
             "msdt": cpals.Plan(w.dims, R, prec=prec, tree="msdt", device=dev)}
    for p in plans.values():
        p.set_tensor(T)
    audit = cpals.Plan(w.dims, R, prec=prec, tree="dt", device=dev)
    audit.set_tensor(T)
    A = {k: [a.clone() for a in A0] for k in ("dt", "msdt", "pp")}

    def restart(k):
        plan = plans["dt" if k == "dt" else "msdt"]
        for a, a0 in zip(A[k], A0):
            a.copy_(a0)
        plan.reset()
        return plan

    def calibrate(nsw):
        """Untimed: DT and MSDT fitness over nsw sweeps, the target (the DT
        run's final fitness less TARGET_SLACK), the sweeps each needs to reach
        it, and PP's outer steps to it, every step audited with cp_fitness."""
        c = {"fit": {}}
        for k in ("dt", "msdt"):
            plan = restart(k)
            c["fit"][k] = [plan.als_sweep(A[k])["fitness"] for _ in range(nsw)]
        target = c["fit"]["dt"][-1] - TARGET_SLACK
        c["target"] = target
        c["to_target"] = {k: next(i + 1 for i, f in enumerate(c["fit"][k]) if f >= target) for k in ("dt", "msdt")}
        plan = restart("pp")
        kinds, est, exact, clamped = [], [], [], []
        c["pp_start"] = None
        while len(kinds) < PP_MAX_STEPS:
            if c["pp_start"] is None:
                before = [a.cpu().numpy() for a in A["pp"]]
            info = plan.pp_sweep(A["pp"], tol=PP_TOL, mode="auto")
            if info["kind"] == "init" and c["pp_start"] is None:
                c["pp_start"] = before
            kinds.append(info["kind"])
            est.append(info["fitness"])
            clamped.append(info["r_clamped"])
            exact.append(audit.fitness(A["pp"]))
            if exact[-1] >= target:
                break
        c.update(pp_kinds=kinds, pp_est=est, pp_exact=exact, pp_clamped=clamped, k_pp=len(kinds),
                 pp_reached=exact[-1] >= target, pp_final=[a.clone() for a in A["pp"]])
        log(f"[bench] {nsw}-sweep target {target:.8f}: dt {c['to_target']['dt']} sweeps, msdt "
            f"{c['to_target']['msdt']}, pp {len(kinds)} steps {kinds} reached={c['pp_reached']}")
        return c

    log("[bench] calibration")
    cal = calibrate(n_sw)
    fit, target, to_target = cal["fit"], cal["target"], cal["to_target"]
    pp_kinds, pp_est, pp_exact, pp_clamped = cal["pp_kinds"], cal["pp_est"], cal["pp_exact"], cal["pp_clamped"]
    k_pp, pp_reached, pp_final, pp_start = cal["k_pp"], cal["pp_reached"], cal["pp_final"], cal["pp_start"]

    stream = torch.cuda.current_stream(dev)

    def one_step(ev=None, nsw=n_sw, kpp=None):
        """ev: per run, a list of events recorded after each sweep (index 0 before the first)."""
        kpp = k_pp if kpp is None else kpp
        for k in ("dt", "msdt", "pp"):
            plan = restart(k)
            if ev is not None:
                ev[k][0].record(stream)
            nk = kpp if k == "pp" else nsw
            for i in range(nk):
                if k == "pp":
                    plan.pp_sweep(A[k], tol=PP_TOL, mode="auto", info=False)
                else:
                    plan.als_sweep(A[k], info=False)
                if ev is not None:
                    ev[k][i + 1].record(stream)

    log("[bench] warmup")
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    log("[bench] timed region")
    # inside the timed region only the first-level contractions of the last
    # timed step carry event pairs (their average launch time feeds the
    # roofline; each pair costs device time); the other phases are timed on
    # one more step afterwards
    for p in plans.values():
        p.profile(False)
        p.profile_read()

    def mk(n):
        return [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]

    evs = [{"dt": mk(n_sw), "msdt": mk(n_sw), "pp": mk(k_pp)} for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        if s == args.steps - 1:
            for p in plans.values():
                p.profile(True, phases=("ttm",))
        one_step(evs[s])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    timed_phase = {}
    for p in plans.values():
        for ph, (ms, cnt) in p.profile_read().items():
            a, b = timed_phase.get(ph, (0.0, 0))
            timed_phase[ph] = (a + ms, b + cnt)
        p.profile(True)  # every phase, for the breakdown step
        p.profile_read()
    # the timed PP runs followed the calibrated trajectory bit for bit
    same = all(torch.equal(a, b) for a, b in zip(A["pp"], pp_final))
    one_step()
    phase = {}
    for p in plans.values():
        for ph, (ms, cnt) in p.profile_read().items():
            a, b = phase.get(ph, (0.0, 0))
            phase[ph] = (a + ms, b + cnt)
        p.profile(False)

    def sweep_ms(k):
        """Mean over timed steps of each sweep's duration (ms), per sweep index."""
        n = len(evs[0][k]) - 1
        return [float(np.mean([e[k][i].elapsed_time(e[k][i + 1]) for e in evs])) for i in range(n)]

    per = {k: sweep_ms(k) for k in ("dt", "msdt", "pp")}
    log(f"[bench] {args.steps} steps, {ms_step:.3f} ms/step; per-run ms "
        f"{ {k: round(sum(v), 3) for k, v in per.items()} }")
    methods = {}
    for k in ("dt", "msdt"):
        methods[k] = {"sweeps": n_sw, "ms_per_sweep": round(sum(per[k]) / n_sw, 4),
                      "effective_tflops": round(F_dt * n_sw / (sum(per[k]) * 1e-3) / 1e12, 3),
                      "sweeps_to_target": to_target[k], "ms_to_target": round(sum(per[k][:to_target[k]]), 4),
                      "final_fitness": fit[k][-1]}
    kinds = {kk: [per["pp"][i] for i, x in enumerate(pp_kinds) if x == kk] for kk in ("exact", "init", "approx")}
    methods["pp"] = {
        "tolerance": PP_TOL, "steps_to_target": k_pp, "reached_target": bool(pp_reached),
        "schedule": pp_kinds,
        "steps_by_kind": {kk: len(v) for kk, v in kinds.items()},
        "ms_by_kind": {kk: round(float(np.mean(v)), 4) for kk, v in kinds.items() if v},
        "ms_to_target": round(sum(per["pp"]), 4),
        "final_exact_fitness": pp_exact[-1],
        "estimate_clamped_steps": int(sum(pp_clamped)),
        "max_abs_estimate_minus_exact": float(max(abs(a - b) for a, b in zip(pp_est, pp_exact))),
        "timed_runs_bitwise_equal_calibration": bool(same),
    }
    methods["msdt"]["speedup_vs_dt_per_sweep"] = round(methods["dt"]["ms_per_sweep"] / methods["msdt"]["ms_per_sweep"], 3)
    for k in ("msdt", "pp"):
        methods[k]["speedup_vs_dt_to_target"] = round(methods["dt"]["ms_to_target"] / methods[k]["ms_to_target"], 3)
    methods["pp"]["speedup_vs_msdt_to_target"] = round(methods["msdt"]["ms_to_target"] / methods["pp"]["ms_to_target"], 3)

    def side_plan(prec_v, tree_v):
        """Three sweeps of another plan from the same initial factors, timed
        on their own (outside the step); ms per sweep and fitness after the
        three sweeps."""
        pc = cpals.Plan(w.dims, R, prec=prec_v, tree=tree_v, device=dev)
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
        return float(np.mean(c_ms)), c_fit[-1]

    # the dimension tree with its upper two levels combined (order >= 4)
    if N >= 4:
        cms, cfit = side_plan(prec, "dt_combined")
        methods["dt_combined"] = {
            "sweeps": 3, "ms_per_sweep": round(cms, 4),
            "effective_tflops": round(F_dt / (cms * 1e-3) / 1e12, 3),
            "speedup_vs_dt_per_sweep": round(methods["dt"]["ms_per_sweep"] / cms, 3),
            "fitness_3_sweeps": cfit, "dt_fitness_3_sweeps": fit["dt"][2],
            "timed": "separately, not part of the step"}
        log(f"[bench] dt_combined {methods['dt_combined']}")
    # the FP32 tensor with the first contraction as three-part BF16 products
    if prec == "f32":
        if N >= 4:
            xms, xfit = side_plan("f32x3", "dt_combined")
            methods["dt_combined_f32x3"] = {
                "sweeps": 3, "ms_per_sweep": round(xms, 4),
                "effective_tflops": round(F_dt / (xms * 1e-3) / 1e12, 3),
                "speedup_vs_dt_per_sweep": round(methods["dt"]["ms_per_sweep"] / xms, 3),
                "fitness_3_sweeps": xfit, "dt_fitness_3_sweeps": fit["dt"][2],
                "timed": "separately, not part of the step"}
            log(f"[bench] dt_combined_f32x3 {methods['dt_combined_f32x3']}")
        for tree_v in ("dt", "msdt"):
            xms, xfit = side_plan("f32x3", tree_v)
            methods[f"{tree_v}_f32x3"] = {
                "sweeps": 3, "ms_per_sweep": round(xms, 4),
                "speedup_vs_f32_per_sweep": round(methods[tree_v]["ms_per_sweep"] / xms, 3),
                "fitness_3_sweeps": xfit, "f32_fitness_3_sweeps": fit[tree_v][2],
                "timed": "separately, not part of the step"}
            log(f"[bench] {tree_v}_f32x3 {methods[f'{tree_v}_f32x3']}")

    # PP against DT and MSDT over a longer run (outside the step): the target
    # is the DT run's fitness after LONG_SWEEPS sweeps, where ALS converges
    # slowly and Alg. 2 stays longer in its PP phase
    long_cmp = None
    if args.workload in LONG_SWEEPS:
        nl = LONG_SWEEPS[args.workload]
        cl = calibrate(nl)
        reps = 2
        evl = [{"dt": mk(nl), "msdt": mk(nl), "pp": mk(cl["k_pp"])} for _ in range(reps)]
        for r in range(reps):
            one_step(evl[r], nsw=nl, kpp=cl["k_pp"])
        torch.cuda.synchronize()
        same_l = all(torch.equal(a, b) for a, b in zip(A["pp"], cl["pp_final"]))

        def ms_of(k):
            n = len(evl[0][k]) - 1
            return [float(np.mean([e[k][i].elapsed_time(e[k][i + 1]) for e in evl])) for i in range(n)]

        pl = {k: ms_of(k) for k in ("dt", "msdt", "pp")}
        tt = {k: sum(pl[k][:cl["to_target"][k]]) for k in ("dt", "msdt")}
        tt["pp"] = sum(pl["pp"])
        kinds_l = {kk: [pl["pp"][i] for i, x in enumerate(cl["pp_kinds"]) if x == kk] for kk in ("exact", "init", "approx")}
        long_cmp = {
            "sweeps": nl, "target_fitness": cl["target"],
            "dt": {"sweeps_to_target": cl["to_target"]["dt"], "ms_to_target": round(tt["dt"], 4)},
            "msdt": {"sweeps_to_target": cl["to_target"]["msdt"], "ms_to_target": round(tt["msdt"], 4),
                     "speedup_vs_dt_to_target": round(tt["dt"] / tt["msdt"], 3)},
            "pp": {"steps_to_target": cl["k_pp"], "reached_target": bool(cl["pp_reached"]),
                   "steps_by_kind": {kk: len(v) for kk, v in kinds_l.items()},
                   "ms_by_kind": {kk: round(float(np.mean(v)), 4) for kk, v in kinds_l.items() if v},
                   "ms_to_target": round(tt["pp"], 4), "final_exact_fitness": cl["pp_exact"][-1],
                   "estimate_clamped_steps": int(sum(cl["pp_clamped"])),
                   "speedup_vs_dt_to_target": round(tt["dt"] / tt["pp"], 3),
                   "speedup_vs_msdt_to_target": round(tt["msdt"] / tt["pp"], 3),
                   "timed_runs_bitwise_equal_calibration": bool(same_l)},
            "timed": f"separately, not part of the step ({reps} repetitions)"}
        log(f"[bench] long comparison {long_cmp}")
    audit.close()

    credited = F_dt * (2 * n_sw + to_target["dt"])
    value = credited / (ms_step * 1e-3) / 1e12
    ttm_ms, ttm_n = timed_phase["ttm"]
    ttm_avg_ms = ttm_ms / max(ttm_n, 1)
    achieved = ttm_flops / (ttm_avg_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
    traffic = load_traffic(kernel_sha()) if args.workload == "o4_s128_r64_f32" else None
    headline = args.workload == "o4_s128_r64_f32"
    cfg = synth.WORKLOADS[args.workload]
    desc = (f"order-{N} dense {'x'.join(map(str, w.dims))} {prec.upper()}, planted rank-{R} {cfg['kind']} factors"
            f" + {cfg['noise_rel']:g} noise{', clipped at zero' if cfg.get('nonneg') else ''}, CP rank {R}")
    out = {
        "metric": ("ALS sweep ms & effective TFLOP/s, order-4 s=128 R=64: MSDT/PP vs plain DT" if headline else
                   f"ALS sweep ms & effective TFLOP/s, {args.workload} ({'x'.join(map(str, w.dims))}, R={R}):"
                   " MSDT/PP vs plain DT"),
        "value": round(value, 3),
        "unit": "TFLOP/s (effective: DT flops to the common target fitness / step time)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": desc, "dims": list(w.dims), "rank": R,
                   "step": f"DT {n_sw} sweeps + MSDT {n_sw} sweeps + PP (Alg. 2, tolerance {PP_TOL}) "
                           f"{k_pp} outer steps to the DT run's final fitness - {TARGET_SLACK:g}",
                   "target_fitness": target, "dt_sweep_gflop": round(F_dt / 1e9, 3), "parallelism": "1 GPU"},
        "methods": methods,
        "long_run_comparison": long_cmp,
        "phase_ms_per_step": {k: round(v[0], 4) for k, v in phase.items()},
        "phase_note": "one extra step with every phase timed (its event pairs make it slower than a timed step)",
        "fitness_per_sweep": {"dt": fit["dt"], "msdt": fit["msdt"]},
        "roofline": {
            "kernel": ("first-level contraction, FP32 MFMA (k_ttm_kc32f / k_ttm_qg / k_ttm_qr with a "
                       "second-level contraction in the epilogue; k_ttm_kc32 / k_ttm_q alone)") if prec == "f32" else
                      "k_ttm (first-level contraction, FP64 MFMA)",
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
    for p in plans.values():
        p.close()
    del T
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        orc = oracle_timings(w, args.cpu_budget, pp_start, n_sw)
        nv = orc["naive"]
        out["cpu_baseline"] = {
            "value": F_dt / (nv["ms_per_sweep"] * 1e-3) / 1e12,
            "unit": "TFLOP/s (DT-equivalent)",
            "cores": orc["threads"],
            "kind": "oracle",
            "sample": f"{nv['sweeps']} exact FP64 ALS sweep(s) of the oracle (explicit-KRP MTTKRP) on the same "
                      f"tensor and init, {nv['ms_per_sweep']:.1f} ms/sweep; oracle-DT and oracle-MSDT sweeps "
                      f"and one PP initialization + approximated step timed on their own",
            "ms_per_sweep": nv["ms_per_sweep"],
            "variants_ms": {"naive": round(nv["ms_per_sweep"], 1), "dt": round(orc["dt"]["ms_per_sweep"], 1),
                            "msdt": round(orc["msdt"]["ms_per_sweep"], 1),
                            **({"pp_init_step": round(orc["pp"]["init_step_ms"], 1),
                                "pp_approx_step": round(orc["pp"]["approx_step_ms"], 1)} if "pp" in orc else {})},
        }
        d = [abs(a - b) for a, b in zip(fit["dt"], nv["fitness"])]
        out["fitness_vs_fp64_oracle"] = {"sweeps": len(d), "max_abs_diff_dt": max(d),
                                         "max_abs_diff_msdt": max(abs(a - b) for a, b in zip(fit["msdt"], nv["fitness"]))}
    print(json.dumps(out), flush=True)


PRECISION_WORKLOAD = "o3_s1024_r128_bf16"


def precision_bench(args):
    """The precision path: order-3 1024^3 tensor stored in BF16 (planted
    rank-128 N(0,1) factors with column norms spread log-uniformly over
    [1e-2, 1], noise 1e-3 of the norm; the FP32 copy is the FP32 plan's
    input), R = 128.  Times DT and MSDT sweeps for FP32, BF16 and BF16X2
    plans, and for the FP8 tensor with a BF16, split or E4M3 factor (FP8 x FP8
    products), reports the first-contraction kernel against the HBM roofline,
    and states the error of each low-precision path against the FP64 oracle
    run on the same stored values: the oracle's exact fitness of the GPU's own factors after each
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
    tensors = {"f32": T32, "bf16": Tb, "bf16x2": Tb, "fp8": T8, "fp8x2": T8, "fp8f8": T8}
    A0 = [torch.from_numpy(a).to(dev) for a in w.init]
    numel = int(np.prod(dims))
    stream = torch.cuda.current_stream(dev)
    res = {}
    for prec in ("f32", "bf16", "bf16x2", "fp8", "fp8x2", "fp8f8"):
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
    ttm88_ms = res["fp8f8"]["dt"]["ttm_avg_ms"]
    achieved88 = (numel + out_bytes) / (ttm88_ms * 1e-3) / 1e9
    # error against the FP64 oracle on the stored BF16 / FP8 values, resynced per sweep
    log("[bench] oracle checks")
    errs = {}
    for prec in ("bf16", "bf16x2", "fp8", "fp8x2", "fp8f8"):
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
        # the factor's rounding (the tensor is exact): BF16 2^-8, split 2^-16, E4M3 2^-4
        unit = {"bf16": 2.0 ** -8, "fp8": 2.0 ** -8, "fp8f8": 2.0 ** -4}.get(prec, 2.0 ** -16)
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
        "roofline_fp8f8": {"kernel": "k_ttm_bf16 (FP8 tensor, E4M3 factor, FP8 x FP8 products, first contraction)",
                           "bound": "hbm", "achieved": round(achieved88, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                           "frac": round(achieved88 / PEAK_HBM_GBS, 4), "traffic": None,
                           "bytes_per_launch": numel + out_bytes, "avg_launch_ms": ttm88_ms},
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
        "dtype": "f32 (contractions as three-part BF16 products with FP32 sums), f64 (solve, Gram, residual)",
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
    tree_bench(args)


if __name__ == "__main__":
    main()
