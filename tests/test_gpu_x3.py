"""GPU parity of the FP32 tensor path whose first contraction runs on the BF16
matrix cores with three-part splits (precision "f32x3") against the FP64
oracle, at the tolerances of the FP32 path: MTTKRPs of every mode and root
(both first-level layouts, ragged tiles, one to eight 16-column blocks, and
the shapes that fall back to the FP32 matrix cores), the full-size order-4
128^4 tensor on sampled rows, and free-running DT / MSDT sweeps."""

import numpy as np
import pytest

from gpu_util import relerr, say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


CASES = [
    # (dims, R): contraction lengths up to 128 take the split path
    ((40, 37, 33, 29), 20),   # KC with K = 29 (not a multiple of 8: FP32 fallback), q layouts
    ((40, 37, 33, 32), 20),   # KC with K = 32
    ((37, 45, 24), 12),       # one column block, ragged 512-row tiles
    ((64, 64, 64), 128),      # two workgroup column passes of 64
    ((21, 9, 128), 64),       # K = 128 in the KC layout, four column blocks
    ((128, 7, 3), 33),        # K = 128 in the q layout, R past two blocks
    ((3, 1, 5, 2, 8), 1),     # unit modes, R = 1
    ((16, 17, 15, 3, 5, 8), 33),
    ((200, 9, 16), 24),       # K = 200 > 128 for mode 0: FP32 fallback there
]


@pytest.mark.parametrize("dims,R", CASES)
def test_x3_mttkrp_every_mode_and_root(dev, dims, R):
    import oracle
    from paper_2010_12056_amd import cpals, synth

    say(f"case x3 mttkrp dims={dims} R={R}")
    w = synth.planted_tensor(dims, R, 300 + len(dims) + R, noise_rel=1e-2, dtype=np.float32)
    T = torch.from_numpy(w.T).to(dev)
    A = to_dev(w.init, dev)
    plan = cpals.Plan(dims, R, prec="f32x3", tree="dt", device=dev)
    plan.set_tensor(T)
    ref32 = cpals.Plan(dims, R, prec="f32", tree="dt", device=dev)
    ref32.set_tensor(T)
    T64 = w.T.astype(np.float64)
    worst = 0.0
    for n in range(len(dims)):
        ref = oracle.mttkrp_naive(T64, w.init, n)
        for root in [None] + [m for m in range(len(dims)) if m != n]:
            M = plan.mttkrp(A, n, root=root).cpu().numpy()
            e = relerr(M, ref)
            assert e <= 1e-5, (n, root, e)
            e32 = relerr(ref32.mttkrp(A, n, root=root).cpu().numpy(), ref)
            worst = max(worst, e / max(e32, 1e-12))
    say(f"  largest error relative to the FP32 path's: {worst:.2f}x")
    plan.close()
    ref32.close()


def test_x3_mttkrp_config_o4_s128_r64_sampled(dev):
    """Full-size order-4 128^4 FP32 tensor, R = 64, every mode and root (both
    layouts of the split kernel); rows sampled and computed one by one by the
    oracle's definition."""
    from oracle import core
    from paper_2010_12056_amd import cpals, synth

    say("case x3 mttkrp o4_s128_r64 full size")
    w = synth.workload("o4_s128_r64_f32")
    plan = cpals.Plan(w.dims, w.R, prec="f32x3", tree="dt", device=dev)
    T = torch.from_numpy(w.T).to(dev)
    plan.set_tensor(T)
    A = to_dev(w.init, dev)
    rng = np.random.default_rng(1)
    for n in range(4):
        rows = rng.choice(w.dims[n], size=6, replace=False)
        K = core.krp([w.init[m] for m in range(4) if m != n])
        X = np.moveaxis(w.T, n, 0)
        ref = np.stack([X[i].astype(np.float64).reshape(-1) @ K for i in rows])
        for root in [None] + [m for m in range(4) if m != n]:
            M = plan.mttkrp(A, n, root=root).cpu().numpy()[rows]
            e = relerr(M, ref)
            say(f"  mode {n} root {root} relerr {e:.2e}")
            assert e <= 1e-5
        del K
    plan.close()


@pytest.mark.parametrize("tree", ["dt", "msdt"])
def test_x3_als_free_running_trajectory(dev, tree):
    """Free-running sweeps against the oracle's, at the FP32 path's
    tolerances (fitness 1e-6, factors 1e-4)."""
    import oracle
    from paper_2010_12056_amd import cpals, synth

    say(f"case x3 als o4_small {tree}")
    w = synth.workload("o4_small_f32")
    plan = cpals.Plan(w.dims, w.R, prec="f32x3", tree=tree, device=dev)
    T = torch.from_numpy(w.T).to(dev)
    plan.set_tensor(T)
    A = to_dev(w.init, dev)
    st = oracle.AlsState.start(w.T.astype(np.float64), w.init)
    N = len(w.dims)
    for sweep in range(2 * (N - 1) + 1):
        info = plan.als_sweep(A)
        r_ref = oracle.als_sweep(st)
        assert abs(info["r"] - r_ref) <= 1e-6, (sweep, info["r"], r_ref)
        for n in range(N):
            assert relerr(A[n].cpu().numpy(), st.A[n]) <= 1e-4, (sweep, n)
    plan.close()
