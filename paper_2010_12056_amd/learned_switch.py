"""Learned PP switch: traces, training and evaluation (not from the paper).

Alg. 2 runs PP sweeps while every factor changed by less than a tolerance
(||dA_i|| < eps ||A_i||).  Here a small network, D = N + 3 inputs -> 64 -> 64
-> 1, makes that call instead, from the per-mode change norms and the last
three fitness deltas (the features that cp_pp_set_switch in include/cpals.h
forms on the plan).

* Traces come from the method itself, on the GPU.  A behavior run of PP-ALS
  follows the hand test with a per-seed tolerance; at each outer step after the
  first, both choices are run from the same state: a regular sweep on a side
  plan, and a PP step (the PP initialization followed by its first approximated
  sweep when the run is outside the PP phase, the next approximated sweep
  inside it).  The exact fitness of every outcome comes from an FP64 audit
  plan.  Label 1 when the PP step's exact fitness gain is at least 0.9 of the
  regular sweep's gain.
* Training runs on the GPU through cp_mlp_grad / cp_mlp_adam, the library's
  own forward and backward kernels (full-batch Adam on the mean binary
  cross-entropy).  Parameters and the feature normalization are stored as JSON
  under paper_2010_12056_amd/models/.
* The regular sweep stays the fallback and the judge: the first sweep of a run
  is always regular; the plan undoes a PP phase that breaks down or that the
  regular sweep closing it shows to have lost fitness (cp_pp_set_switch); the
  evaluation checks every claimed target with the FP64 audit.

CLI (GPU):  python -m paper_2010_12056_amd.learned_switch collect|train|evaluate ...
"""

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from .cpals import CpalsError

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_DIR = os.path.join(HERE, "models")
DEFAULT_MODEL = os.path.join(MODEL_DIR, "pp_switch_o6_s24_r32.json")

# order-6 24^6 FP32 tensors, planted rank-32 factors with collinearity 0.9, noise 1e-2 of the norm
FAMILY = dict(dims=(24,) * 6, R=32, kind="collinear", noise_rel=1e-2, collinearity=0.9)
SMALL_FAMILY = dict(dims=(10,) * 6, R=8, kind="collinear", noise_rel=1e-2, collinearity=0.9)
TRAIN_SEEDS = list(range(4100, 4150))
HELDOUT_SEEDS = list(range(4200, 4210))
BEHAVIOR_EPS = (0.05, 0.1, 0.2, 0.3, 0.5)
HIDDEN = 64
GAIN_RATIO = 0.9


def features(dA_rel, fit_hist):
    """Unnormalized switch features, in the order the plan forms them:
    log10 of each factor's relative change, then log10 of the last three
    fitness deltas (fit_hist newest first; a delta not yet available counts
    as 1)."""
    x = [math.log10(max(float(r), 1e-12)) for r in dA_rel]
    for j in range(3):
        d = abs(fit_hist[j] - fit_hist[j + 1]) if len(fit_hist) >= j + 2 else 1.0
        x.append(math.log10(max(d, 1e-12)))
    return x


def make_workload(seed, small=False):
    from . import synth

    cfg = dict(SMALL_FAMILY if small else FAMILY)
    dims = cfg.pop("dims")
    R = cfg.pop("R")
    return synth.planted_tensor(dims, R, seed, dtype=np.float32, **cfg)


def _prefetch(seeds, small, workers=3):
    """Yield (seed, workload) in order, generating a few seeds ahead on host
    threads (the generator's numpy kernels release the GIL)."""
    with ThreadPoolExecutor(max_workers=workers) as ex:
        futs = [ex.submit(make_workload, s, small) for s in seeds[:workers]]
        for i, s in enumerate(seeds):
            w = futs[i].result()
            futs[i] = None
            if i + workers < len(seeds):
                futs.append(ex.submit(make_workload, seeds[i + workers], small))
            yield s, w


class Bench:
    """The plans one workload needs: the FP32 MSDT plan that runs the method,
    an FP32 side plan for counterfactual sweeps, and an FP64 plan that audits
    fitness exactly (cp_fitness on an FP64 copy of the tensor)."""

    def __init__(self, w, device="cuda"):
        import torch

        from . import cpals

        self.dev = torch.device(device)
        self.w = w
        self.T = torch.from_numpy(w.T).to(self.dev)
        self.T64 = self.T.double()
        self.main = cpals.Plan(w.dims, w.R, prec="f32", tree="msdt", device=self.dev)
        self.side = cpals.Plan(w.dims, w.R, prec="f32", tree="msdt", device=self.dev)
        self.audit_plan = cpals.Plan(w.dims, w.R, prec="f64", tree="dt", device=self.dev)
        self.main.set_tensor(self.T)
        self.side.set_tensor(self.T)
        self.audit_plan.set_tensor(self.T64)

    def init_factors(self):
        import torch

        return [torch.from_numpy(a).to(self.dev) for a in self.w.init]

    def audit(self, A):
        return self.audit_plan.fitness(A)

    def close(self):
        for p in (self.main, self.side, self.audit_plan):
            p.close()


def _copy(A):
    return [a.clone() for a in A]


def collect_seed(b, seed, steps, behavior_eps, log=print):
    """Features, labels and exact gains along one behavior run (see the module
    docstring).  Returns (X, y, gains[:, (regular, pp)], kind[0 init / 1 approx])."""
    A = b.init_factors()
    b.main.reset()
    X, Y, G, K = [], [], [], []
    hist = []  # reported fitness after each sweep of the run, newest first
    last = None
    f_cur = None  # audited fitness of the current factors
    stop = ""
    for _ in range(steps):
        if last is None:
            last = b.main.pp_sweep(A, mode="exact")
            hist.insert(0, last["fitness"])
            f_cur = b.audit(A)
            continue
        x = features(last["dA_rel"], hist)
        allowed = all(r < behavior_eps for r in last["dA_rel"])
        in_pp = last["kind"] in ("init", "approx")
        Ae = _copy(A)
        b.side.reset()
        try:
            b.side.als_sweep(Ae)
        except CpalsError as e:
            # a regular sweep from this state breaks down (non-finite Gamma after a
            # diverging approximated step): the trajectory ends here
            stop = f", stopped: regular sweep failed ({e.status})"
            break
        fe = b.audit(Ae)
        if not in_pp:
            Ap = _copy(A)
            b.side.reset()
            try:
                b.side.pp_sweep(Ap, mode="init")
                fp = b.audit(Ap)
            except CpalsError:
                fp = -math.inf  # the PP step broke down: certainly worse than the regular sweep
            X.append(x)
            Y.append(1.0 if fp - f_cur >= GAIN_RATIO * (fe - f_cur) else 0.0)
            G.append((fe - f_cur, fp - f_cur))
            K.append(0)
            use_pp = allowed and fp > -math.inf
            info = b.main.pp_sweep(A, mode="init" if use_pp else "exact")
            f_next = fp if use_pp else fe
        elif allowed:
            try:
                info = b.main.pp_sweep(A, mode="approx")
                fp = b.audit(A)
            except CpalsError as e:
                X.append(x)
                Y.append(0.0)
                G.append((fe - f_cur, -math.inf))
                K.append(1)
                stop = f", stopped: approximated sweep failed ({e.status})"
                break
            X.append(x)
            Y.append(1.0 if fp - f_cur >= GAIN_RATIO * (fe - f_cur) else 0.0)
            G.append((fe - f_cur, fp - f_cur))
            K.append(1)
            f_next = fp
        else:
            info = b.main.pp_sweep(A, mode="exact")
            f_next = fe
        hist.insert(0, info["fitness"])
        del hist[4:]
        last = info
        f_cur = f_next
    n = len(Y)
    log(f"[collect] seed {seed} eps {behavior_eps}: {n} samples ({sum(K)} approx), {int(sum(Y))} positive, "
        f"last audited fitness {f_cur:.6f}{stop}")
    return (np.array(X, dtype=np.float64).reshape(n, -1), np.array(Y), np.array(G).reshape(n, 2),
            np.array(K, dtype=np.int32))


def init_params(D, H, seed):
    """Glorot-uniform weights, zero biases, in the switch parameter layout."""
    rng = np.random.default_rng(seed)

    def glorot(a, b):
        lim = math.sqrt(6.0 / (a + b))
        return rng.uniform(-lim, lim, size=(a, b))

    return np.concatenate([glorot(D, H).ravel(), np.zeros(H), glorot(H, H).ravel(), np.zeros(H),
                           glorot(H, 1).ravel(), [0.0]]).astype(np.float32)


def _bce(p, y):
    p = np.clip(np.asarray(p, dtype=np.float64), 1e-7, 1.0 - 1e-7)
    return float(-np.mean(y * np.log(p) + (1.0 - y) * np.log(1.0 - p)))


def train(X, y, hidden=HIDDEN, steps=3000, lr=3e-3, seed=0, device="cuda", X_val=None, y_val=None, log=print):
    """Full-batch Adam on the GPU with the library's kernels.  With validation
    traces, the parameters of the step with the lowest validation loss are
    kept (early stopping).  Returns the model dict (theta, feature
    normalization, loss curves)."""
    import torch

    from . import cpals

    dev = torch.device(device)
    shift = X.mean(axis=0)
    scale = X.std(axis=0)
    scale[scale < 1e-6] = 1.0
    Xn = torch.tensor((X - shift) / scale, dtype=torch.float32, device=dev)
    yt = torch.tensor(y, dtype=torch.float32, device=dev)
    Xv = None
    if X_val is not None and len(X_val):
        Xv = torch.tensor((X_val - shift) / scale, dtype=torch.float32, device=dev)
    D = X.shape[1]
    theta = torch.tensor(init_params(D, hidden, seed), device=dev)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    n = theta.numel()
    scratch = torch.empty(int(cpals.lib().cp_mlp_scratch_floats(Xn.shape[0], hidden)), dtype=torch.float32,
                          device=dev)
    out = torch.empty(n + 1, dtype=torch.float32, device=dev)
    losses, best = [], (math.inf, 0, theta.clone())
    for t in range(1, steps + 1):
        cpals.mlp_grad(Xn, yt, theta, hidden, scratch=scratch, out=out)
        cpals.mlp_adam(theta, out[:n], m, v, t, lr=lr)
        if t == 1 or t % 25 == 0:
            rec = [t, float(out[n].item())]
            if Xv is not None:
                vl = _bce(cpals.mlp_forward(Xv, theta, hidden).cpu().numpy(), y_val)
                rec.append(vl)
                if vl < best[0]:
                    best = (vl, t, theta.clone())
            losses.append(rec)
    if Xv is not None:
        theta = best[2]
        log(f"[train] early stop at step {best[1]} (validation loss {best[0]:.4f})")
    p = cpals.mlp_forward(Xn, theta, hidden).cpu().numpy()
    acc = float(np.mean((p > 0.5) == (y > 0.5)))
    res = {"D": int(D), "H": int(hidden), "theta": [float(t) for t in theta.cpu().numpy()],
           "shift": shift.tolist(), "scale": scale.tolist(), "threshold": 0.5, "loss_curve": losses,
           "train_accuracy": acc, "n_samples": int(X.shape[0]), "n_positive": int(y.sum()),
           "steps_kept": best[1] if Xv is not None else steps}
    if Xv is not None:
        pv = cpals.mlp_forward(Xv, theta, hidden).cpu().numpy()
        res["val_accuracy"] = float(np.mean((pv > 0.5) == (y_val > 0.5)))
        res["val_loss"] = best[0]
    log(f"[train] {X.shape[0]} samples, loss {losses[0][1]:.4f} -> {losses[-1][1]:.4f}, training accuracy {acc:.3f}"
        + (f", validation accuracy {res['val_accuracy']:.3f}" if Xv is not None else ""))
    return res


def load_model(path=DEFAULT_MODEL):
    with open(path) as f:
        return json.load(f)


def attach(plan, model):
    """Attach a stored model to a plan; returns the device parameter tensor
    (the plan keeps a reference while the switch is set)."""
    import torch

    theta = torch.tensor(np.array(model["theta"], dtype=np.float32), device=plan.device)
    plan.set_switch(theta, model["H"], model["shift"], model["scale"], model.get("threshold", 0.5))
    return theta


def run_policy(b, policy, sweeps, eps=None, target=None):
    """One run of `policy` ("exact", "eps" or "learned") on the main plan, from
    the workload's initial factors.  Each sweep is timed alone (synchronized);
    the FP64 audit runs outside the timed region, on its own plan.  Stops once
    the audited fitness reaches `target` (checked whenever the reported fitness
    is within 1e-4 of it)."""
    import torch

    A = b.init_factors()
    plan = b.main
    plan.reset()
    kinds, times, fits = [], [], []
    reached = False
    f_audit = None
    failed = ""
    for _ in range(sweeps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            if policy == "exact":
                info = plan.pp_sweep(A, mode="exact")
            elif policy == "eps":
                info = plan.pp_sweep(A, tol=eps, mode="auto")
            else:
                info = plan.pp_sweep(A, mode="learned")
        except CpalsError as e:
            failed = f"sweep {len(kinds)}: status {e.status}"
            break
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        kinds.append(info["kind"])
        fits.append(info["fitness"])
        if target is not None and info["fitness"] >= target - 1e-4:
            f_audit = b.audit(A)
            if f_audit >= target:
                reached = True
                break
    if not reached:
        f_audit = b.audit(A) if not failed else float("nan")
    return {"kinds": kinds, "times": times, "fitness": fits, "audited": f_audit, "reached": reached,
            "failed": failed}


def summarize(run, t_regular):
    kinds = run["kinds"]
    return {"steps": len(kinds), "time_s": float(sum(run["times"])),
            "regular_equiv": float(sum(run["times"]) / t_regular), "reached": run["reached"],
            "n_exact": kinds.count("exact"), "n_init": kinds.count("init"), "n_approx": kinds.count("approx"),
            "audited_fitness": run["audited"], "failed": run["failed"]}


def evaluate_workload(b, model, sweeps=200, margin=1e-4, thresholds=None):
    """Time to reach the regular-only run's final (audited) fitness minus
    `margin`, for regular sweeps only, eps = 0.1, eps = 0.2 and the learned
    switch (at the model's threshold, or at each of `thresholds`)."""
    ref = run_policy(b, "exact", sweeps)
    target = ref["audited"] - margin
    t_regular = float(np.median(ref["times"][1:])) if len(ref["times"]) > 1 else ref["times"][0]
    out = {"target": target, "t_regular_sweep_s": t_regular,
           "regular": summarize(run_policy(b, "exact", sweeps, target=target), t_regular)}
    for name, eps in (("eps0.1", 0.1), ("eps0.2", 0.2)):
        out[name] = summarize(run_policy(b, "eps", sweeps, eps=eps, target=target), t_regular)
    ths = thresholds if thresholds else [model.get("threshold", 0.5)]
    for th in ths:
        theta = attach(b.main, dict(model, threshold=th))
        try:
            name = "learned" if not thresholds else f"learned@{th:g}"
            out[name] = summarize(run_policy(b, "learned", sweeps, target=target), t_regular)
        finally:
            b.main.set_switch(None, 0, None, None)
            del theta
    return out


def aggregate(res):
    """Per policy: runs that reached the target, and the geometric mean over
    seeds of (time to target) / (regular-only time to target) on those runs."""
    pols = [k for k, v in next(iter(res.values())).items() if isinstance(v, dict)]
    out = {}
    for pol in pols:
        ratios = [r[pol]["time_s"] / r["regular"]["time_s"] for r in res.values() if r[pol]["reached"]]
        out[pol] = {"reached": len(ratios), "runs": len(res),
                    "time_ratio_geomean": float(np.exp(np.mean(np.log(ratios)))) if ratios else None}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2010_12056_amd.learned_switch")
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--seeds", default=f"{TRAIN_SEEDS[0]}-{TRAIN_SEEDS[-1]}")
    c.add_argument("--steps", type=int, default=200)
    c.add_argument("--small", action="store_true")
    c.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--traces", required=True)
    t.add_argument("--steps", type=int, default=3000)
    t.add_argument("--lr", type=float, default=3e-3)
    t.add_argument("--exclude-seeds", default="",
                   help="seed range kept out of training (early stopping and threshold selection)")
    t.add_argument("--out", default=DEFAULT_MODEL)
    sel = sub.add_parser("select", help="set the model threshold from an evaluation with --thresholds")
    sel.add_argument("--eval", required=True)
    sel.add_argument("--model", default=DEFAULT_MODEL)
    e = sub.add_parser("evaluate")
    e.add_argument("--seeds", default=f"{HELDOUT_SEEDS[0]}-{HELDOUT_SEEDS[-1]}")
    e.add_argument("--sweeps", type=int, default=200)
    e.add_argument("--model", default=DEFAULT_MODEL)
    e.add_argument("--small", action="store_true")
    e.add_argument("--thresholds", default="", help="comma-separated switch thresholds to compare")
    e.add_argument("--out", required=True)
    args = ap.parse_args(argv)

    def seeds(spec):
        if not spec:
            return []
        a, b_ = spec.split("-")
        return list(range(int(a), int(b_) + 1))

    def log(msg):
        print(msg, flush=True)

    if args.cmd == "collect":
        Xs, Ys, Gs, Ks, S = [], [], [], [], []
        for sd, w in _prefetch(seeds(args.seeds), args.small):
            b = Bench(w)
            X, Y, G, K = collect_seed(b, sd, args.steps, BEHAVIOR_EPS[sd % len(BEHAVIOR_EPS)], log=log)
            b.close()
            del b, w
            Xs.append(X)
            Ys.append(Y)
            Gs.append(G)
            Ks.append(K)
            S += [sd] * len(Y)
            np.savez(args.out, X=np.concatenate(Xs), y=np.concatenate(Ys), gains=np.concatenate(Gs),
                     kind=np.concatenate(Ks), seed=np.array(S))
        log(f"[collect] wrote {args.out}")
    elif args.cmd == "train":
        d = np.load(args.traces)
        keep = ~np.isin(d["seed"], seeds(args.exclude_seeds))
        model = train(d["X"][keep], d["y"][keep], steps=args.steps, lr=args.lr, X_val=d["X"][~keep],
                      y_val=d["y"][~keep], log=log)
        fam = {k: (list(v) if isinstance(v, tuple) else v) for k, v in FAMILY.items()}
        model["traces"] = {"seeds": sorted(set(int(s) for s in d["seed"][keep])), "family": fam,
                           "behavior_eps": list(BEHAVIOR_EPS), "gain_ratio": GAIN_RATIO}
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        with open(args.out, "w") as f:
            json.dump(model, f)
        log(f"[train] wrote {args.out}")
    elif args.cmd == "select":
        with open(args.eval) as f:
            agg = json.load(f)["aggregate"]
        cands = [(v["reached"], -(v["time_ratio_geomean"] or math.inf), float(k.split("@")[1]))
                 for k, v in agg.items() if k.startswith("learned@")]
        best = max(cands)
        model = load_model(args.model)
        model["threshold"] = best[2]
        model["threshold_selection"] = {"eval": os.path.basename(args.eval), "aggregate": agg}
        with open(args.model, "w") as f:
            json.dump(model, f)
        log(f"[select] threshold {best[2]:g} (reached {best[0]}, time ratio {-best[1]:.3f})")
    else:
        model = load_model(args.model)
        ths = [float(t) for t in args.thresholds.split(",")] if args.thresholds else None
        res = {}
        for sd, w in _prefetch(seeds(args.seeds), args.small, workers=2):
            b = Bench(w)
            res[sd] = evaluate_workload(b, model, args.sweeps, thresholds=ths)
            b.close()
            del b, w
            log(f"[evaluate] seed {sd}: " + ", ".join(
                f"{k} {v['time_s'] * 1e3:.1f} ms/{v['steps']} sweeps{'' if v['reached'] else ' (not reached)'}"
                for k, v in res[sd].items() if isinstance(v, dict)))
            with open(args.out, "w") as f:
                json.dump({"seeds": res, "aggregate": aggregate(res)}, f, indent=1)
        for k, v in aggregate(res).items():
            log(f"[evaluate] {k}: reached {v['reached']}/{v['runs']}, time / regular-only time "
                f"{v['time_ratio_geomean']}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
