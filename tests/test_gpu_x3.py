"""GPU parity of the FP32 tensor path whose first contraction runs on the BF16
matrix cores with three-part splits (precision "f32x3") against the FP64
oracle, at the tolerances of the FP32 path: MTTKRPs of every mode and root
(both first-level layouts, ragged tiles, one to eight 16-column blocks,
several factor chunks, and the KC shapes that fall back to the FP32 matrix
cores), the full-size order-4 128^4 tensor on sampled rows, free-running DT /
MSDT sweeps, and the combined-levels tree with its contractions split over K."""

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
    # (dims, R)
    ((40, 37, 33, 29), 20),   # KC with K = 29 (not a multiple of 8: FP32 fallback), q layouts
    ((40, 37, 33, 32), 20),   # KC with K = 32
    ((37, 45, 24), 12),       # one column block, ragged 512-row tiles
    ((64, 64, 64), 128),      # two workgroup column passes of 64
    ((21, 9, 128), 64),       # K = 128 in the KC layout, four column blocks
    ((128, 7, 3), 33),        # K = 128 in the q layout, R past two blocks
    ((3, 1, 5, 2, 8), 1),     # unit modes, R = 1
    ((16, 17, 15, 3, 5, 8), 33),
    ((200, 9, 16), 24),       # K = 200: four factor chunks, the last one ragged
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
    layouts of the split kernel) and the combined-levels tree (contractions
    over 16384 indices split over K); rows sampled and computed one by one by
    the oracle's definition.  Besides the norm-wise error, the signed mean
    error relative to the mean magnitude must stay below 1e-8: the factors
    and the tensor are positive here, so a rounding that favours one
    direction in the long sums would show as a bias (it did, -4.8e-8, while
    the small part products were added to the running sums directly)."""
    from oracle import core
    from paper_2010_12056_amd import cpals, synth

    say("case x3 mttkrp o4_s128_r64 full size")
    w = synth.workload("o4_s128_r64_f32")
    T = torch.from_numpy(w.T).to(dev)
    plan = cpals.Plan(w.dims, w.R, prec="f32x3", tree="dt", device=dev)
    plan.set_tensor(T)
    comb = cpals.Plan(w.dims, w.R, prec="f32x3", tree="dt_combined", device=dev)
    comb.set_tensor(T)
    A = to_dev(w.init, dev)
    rng = np.random.default_rng(1)
    for n in range(4):
        rows = rng.choice(w.dims[n], size=6, replace=False)
        K = core.krp([w.init[m] for m in range(4) if m != n])
        X = np.moveaxis(w.T, n, 0)
        ref = np.stack([X[i].astype(np.float64).reshape(-1) @ K for i in rows])
        runs = [(f"root {root}", plan.mttkrp(A, n, root=root)) for root in [None] + [m for m in range(4) if m != n]]
        runs.append(("combined", comb.mttkrp(A, n)))
        for name, Mt in runs:
            M = Mt.cpu().numpy()[rows]
            e = relerr(M, ref)
            bias = float(np.mean(M - ref) / np.mean(np.abs(ref)))
            say(f"  mode {n} {name} relerr {e:.2e} bias {bias:.1e}")
            assert e <= 1e-5
            assert abs(bias) <= 1e-8, (n, name, bias)
        del K
    plan.close()
    comb.close()


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


@pytest.mark.parametrize("dims,R", [((24, 20, 28, 32), 20), ((16, 18, 20, 14, 12), 33), ((12, 40, 36, 30), 64)])
def test_x3_combined_tree_mttkrp_and_sweeps(dev, dims, R):
    """The combined-levels tree with the three-part contractions (its two
    long contractions split over K on workgroup layers): MTTKRPs of every
    mode against the oracle at 1e-5, then free-running sweeps at the FP32
    tolerances."""
    import oracle
    from paper_2010_12056_amd import cpals, synth

    say(f"case x3 combined dims={dims} R={R}")
    w = synth.planted_tensor(dims, R, 500 + len(dims) + R, noise_rel=1e-2, dtype=np.float32)
    T = torch.from_numpy(w.T).to(dev)
    A = to_dev(w.init, dev)
    plan = cpals.Plan(dims, R, prec="f32x3", tree="dt_combined", device=dev)
    plan.set_tensor(T)
    T64 = w.T.astype(np.float64)
    for n in range(len(dims)):
        e = relerr(plan.mttkrp(A, n).cpu().numpy(), oracle.mttkrp_naive(T64, w.init, n))
        assert e <= 1e-5, (n, e)
    st = oracle.AlsState.start(T64, w.init)
    for sweep in range(4):
        info = plan.als_sweep(A)
        r_ref = oracle.als_sweep(st)
        assert abs(info["r"] - r_ref) <= 1e-6, (sweep, info["r"], r_ref)
    plan.close()
