"""Sweeps captured in a HIP graph and replayed, against the same sweeps run
eagerly.  With info == NULL and a forced kind, cp_als_sweep and
cp_pp_sweep enqueue device work only (no host synchronization), so a
caller may capture one sweep and replay it: with the standard dimension
tree every exact sweep launches the same kernels with the same arguments,
and so does every approximated PP sweep (Alg. 2 inner loop).  Each replay
must equal the eager sweep it stands for bit for bit, with unrelated eager
work and synchronizations between the replays."""

import numpy as np
import pytest

from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _eager_and_graph(dev, w, prec, warm, kind, replays):
    """Factors after each of `replays` eager sweeps of `kind` (after the
    `warm` schedule) and after each replay of one captured sweep."""
    from paper_2010_12056_amd import cpals

    s = torch.cuda.Stream(dev)
    s.wait_stream(torch.cuda.current_stream(dev))
    out = {}
    with torch.cuda.stream(s):
        T = torch.from_numpy(w.T).to(dev)
        for mode in ("eager", "graph"):
            plan = cpals.Plan(w.dims, w.R, prec=prec, tree="dt", device=dev)
            plan.set_tensor(T)
            A = to_dev(w.init, dev)
            for k in warm:
                plan.pp_sweep(A, mode=k, info=False)
            res = []
            if mode == "eager":
                for _ in range(replays):
                    plan.pp_sweep(A, mode=kind, info=False)
                    s.synchronize()
                    res.append([a.cpu().numpy().copy() for a in A])
            else:
                s.synchronize()
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=s):
                    plan.pp_sweep(A, mode=kind, info=False)
                junk = torch.randn(512, 512, device=dev)
                for r in range(replays):
                    g.replay()
                    s.synchronize()
                    res.append([a.cpu().numpy().copy() for a in A])
                    junk = junk @ junk.T / 512.0  # unrelated eager work between replays
                    torch.cuda.synchronize()
                del g
            out[mode] = res
            plan.close()
    torch.cuda.current_stream(dev).wait_stream(s)
    return out


@pytest.mark.parametrize("name,prec", [("o4_small_f32", "f32"), ("o3_small_f64", "f64")])
def test_exact_sweep_graph_replay_equals_eager(dev, name, prec):
    from paper_2010_12056_amd import synth

    say(f"case graph exact {name}")
    w = synth.workload(name)
    out = _eager_and_graph(dev, w, prec, ["exact"], "exact", 4)
    for r, (ge, gg) in enumerate(zip(out["eager"], out["graph"])):
        for n in range(len(w.dims)):
            assert np.array_equal(ge[n], gg[n]), (r, n)


@pytest.mark.parametrize("name,prec", [("o4_small_f32", "f32"), ("o5_small_f64", "f64")])
def test_pp_approx_sweep_graph_replay_equals_eager(dev, name, prec):
    from paper_2010_12056_amd import synth

    say(f"case graph pp approx {name}")
    w = synth.workload(name)
    out = _eager_and_graph(dev, w, prec, ["exact"] * 5 + ["init"], "approx", 3)
    for r, (ge, gg) in enumerate(zip(out["eager"], out["graph"])):
        for n in range(len(w.dims)):
            assert np.array_equal(ge[n], gg[n]), (r, n)
