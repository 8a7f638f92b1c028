"""Launch-shape autotuner of the batched path (not from the paper).

The persistent batched kernel (cp_batch_sweeps) has two launch parameters:
waves per workgroup (4 or 8: how many waves share one tensor's contractions
and solves) and workgroups per compute unit in the grid (1 or 2; with the
kernel's 145 KB of LDS only one is resident at a time, so 2 means a second
round of workgroups that start as the first ones finish).
The tuner times every candidate on the actual batch (a few sweeps, after a
warm-up launch) and keeps the fastest; results are cached as JSON keyed by
the device and a signature of the batch (size, mode-size range, rank set).

    python -m paper_2010_12056_amd.autotune            # tunes the benchmark batch
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned", "batch_launch.json")
CANDIDATES = [(4, 1), (4, 2), (8, 1), (8, 2)]


def signature(dims, ranks):
    s = [x for d in dims for x in d]
    return f"order3|n{len(dims)}|s{min(s)}-{max(s)}|R{','.join(str(r) for r in sorted(set(ranks)))}"


def device_key(device="cuda"):
    import torch

    p = torch.cuda.get_device_properties(torch.device(device))
    return f"{getattr(p, 'gcnArchName', p.name)}|{p.multi_processor_count}cu"


def load_cache(path=CACHE):
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def lookup(dims, ranks, device="cuda", path=CACHE):
    return load_cache(path).get(device_key(device) + "|" + signature(dims, ranks))


def tune(workloads, sweeps=5, reps=3, device="cuda", path=CACHE, write=True, log=print):
    """Time every candidate launch shape on `workloads` (synth.Workload list)
    and return {"waves", "groups_per_cu", "ms": {...}}; cached in `path`."""
    import torch

    from . import cpals

    dims = [w.dims for w in workloads]
    ranks = [w.R for w in workloads]
    dev = torch.device(device)
    results = {}
    for waves, groups in CANDIDATES:
        b = cpals.Batch(dims, ranks, device=dev, waves=waves, groups_per_cu=groups)
        T = b.pack_tensors([w.T for w in workloads])
        A0 = b.pack_factors([w.init for w in workloads])
        A = A0.clone()
        fit = torch.empty((len(workloads), sweeps), dtype=torch.float64, device=dev)
        st = torch.empty(len(workloads), dtype=torch.int32, device=dev)
        b.sweeps(T, A, sweeps, fitness=fit, status=st)  # warm-up
        times = []
        for _ in range(reps):
            A.copy_(A0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.sweeps(T, A, sweeps, fitness=fit, status=st)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        results[f"{waves}x{groups}"] = min(times)
        log(f"[autotune] waves {waves}, groups/CU {groups}: {min(times):.3f} ms for {sweeps} sweeps")
        b.close()
    best = min(results, key=results.get)
    waves, groups = (int(x) for x in best.split("x"))
    entry = {"waves": waves, "groups_per_cu": groups, "ms": results, "sweeps": sweeps}
    if write:
        cache = load_cache(path)
        cache[device_key(device) + "|" + signature(dims, ranks)] = entry
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return entry


def main(argv=None):
    import argparse

    from . import synth

    ap = argparse.ArgumentParser(prog="python -m paper_2010_12056_amd.autotune")
    ap.add_argument("--out", default=CACHE, help="cache file to update")
    args = ap.parse_args(argv)
    ws = synth.batch_workload(512, seed=5001)
    entry = tune(ws, path=args.out)
    print(json.dumps(entry))
    return 0


if __name__ == "__main__":
    sys.exit(main())
