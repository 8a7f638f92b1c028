"""GPU parity of the fused first and second levels (FP32 plans) against the
FP64 oracle: the standard tree's halves (each half's first two contractions
in one pass, the first-level node not stored) and MSDT's subtree roots (the
subtree's first child formed in the first level's epilogue, the first-level
node stored for the later child), and the PP initialization's first-level
node with a single pair child (the pair straight from the tensor, including
the contraction over the last mode after a mode with leading slices).  Leading half: the contraction over the last mode,
of size 128, and the one over the mode before it, a multiple of 32.
Trailing half: the contraction over mode 0 (a multiple of 32) and over mode
1, cut into ranges whose partial nodes are added in order.  MTTKRPs of every
mode (fused and two-pass halves side by side), one to four column blocks,
one to eight row tiles per output row, ranges of one index and a ragged last
range, orders 4 and 5, free-running DT sweeps, and the full-size order-4
128^4 tensor on sampled rows."""

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
    # (dims, R).  Leading half fused: the last mode 128, the one before it a
    # multiple of 32.  Trailing half fused: mode 0 a multiple of 32, the
    # product of modes 2.. a multiple of 64.
    ((7, 9, 32, 128), 24),     # leading: one column block, one tile per output row
    ((4, 5, 96, 128), 64),     # leading: two column blocks, three tiles per row
    ((3, 2, 256, 128), 40),    # leading: eight tiles per row, R past one block
    ((3, 4, 5, 64, 128), 33),  # leading, order 5
    ((6, 7, 64, 128), 17),     # leading: R just above that kernel's lower limit
    ((32, 5, 8, 16), 12),      # trailing: one 16-column block, ranges of one index
    ((64, 3, 16, 8), 24),      # trailing: two blocks
    ((96, 7, 4, 32), 64),      # trailing: four blocks, K = 96
    ((32, 13, 128, 128), 20),  # both halves; trailing: ranges of two, the last ragged
    ((64, 6, 4, 64, 128), 40), # both halves, order 5
]


@pytest.mark.parametrize("dims,R", CASES)
def test_fused_mttkrp_every_mode(dev, dims, R):
    import oracle
    from paper_2010_12056_amd import cpals, synth

    say(f"case fused mttkrp dims={dims} R={R}")
    w = synth.planted_tensor(dims, R, 700 + len(dims) + R, noise_rel=1e-2, dtype=np.float32)
    T = torch.from_numpy(w.T).to(dev)
    A = to_dev(w.init, dev)
    plan = cpals.Plan(dims, R, prec="f32", tree="dt", device=dev)
    plan.set_tensor(T)
    T64 = w.T.astype(np.float64)
    for n in range(len(dims)):
        e = relerr(plan.mttkrp(A, n).cpu().numpy(), oracle.mttkrp_naive(T64, w.init, n))
        say(f"  mode {n} relerr {e:.2e}")
        assert e <= 1e-5, (n, e)
    plan.close()


@pytest.mark.parametrize("dims,R", [((4, 5, 96, 128), 64), ((3, 4, 5, 64, 128), 33), ((64, 6, 4, 64, 128), 40)])
def test_fused_dt_free_running_trajectory(dev, dims, R):
    """Free-running DT sweeps against the oracle's, at the FP32 path's
    tolerances (fitness 1e-6, factors 1e-4)."""
    import oracle
    from paper_2010_12056_amd import cpals, synth

    say(f"case fused dt sweeps dims={dims} R={R}")
    w = synth.planted_tensor(dims, R, 800 + len(dims) + R, noise_rel=1e-2, dtype=np.float32)
    plan = cpals.Plan(dims, R, prec="f32", tree="dt", device=dev)
    plan.set_tensor(torch.from_numpy(w.T).to(dev))
    A = to_dev(w.init, dev)
    st = oracle.AlsState.start(w.T.astype(np.float64), w.init)
    for sweep in range(4):
        info = plan.als_sweep(A)
        r_ref = oracle.als_sweep(st)
        assert abs(info["r"] - r_ref) <= 1e-6, (sweep, info["r"], r_ref)
        for n in range(len(dims)):
            assert relerr(A[n].cpu().numpy(), st.A[n]) <= 1e-4, (sweep, n)
    plan.close()


@pytest.mark.parametrize("dims,R,sweeps", [((32, 32, 64, 128), 40, 4), ((3, 32, 32, 32, 128), 24, 5),
                                            ((64, 16, 8, 64), 16, 4)])
def test_fused_msdt_free_running_trajectory(dev, dims, R, sweeps):
    """MSDT sweeps through every subtree root against the oracle's ALS
    sweeps, at the FP32 path's tolerances.  The fused forms that also store
    the first-level node: the last-mode root (32 x 32 x 64 x 128 and order 5),
    the middle roots (both), the mode-0 root with the last mode in the
    epilogue (32 x 32 x 64 x 128, four column blocks past R; 64 x 16 x 8 x 64,
    one block); the other roots take the two-pass form."""
    import oracle
    from paper_2010_12056_amd import cpals, synth

    say(f"case fused msdt sweeps dims={dims} R={R}")
    w = synth.planted_tensor(dims, R, 900 + len(dims) + R, noise_rel=1e-2, dtype=np.float32)
    plan = cpals.Plan(dims, R, prec="f32", tree="msdt", device=dev)
    plan.set_tensor(torch.from_numpy(w.T).to(dev))
    A = to_dev(w.init, dev)
    st = oracle.AlsState.start(w.T.astype(np.float64), w.init)
    for sweep in range(sweeps):
        info = plan.als_sweep(A)
        r_ref = oracle.als_sweep(st)
        say(f"  sweep {sweep} r={info['r']:.10f} oracle={r_ref:.10f}")
        assert abs(info["r"] - r_ref) <= 1e-6, (sweep, info["r"], r_ref)
        for n in range(len(dims)):
            assert relerr(A[n].cpu().numpy(), st.A[n]) <= 1e-4, (sweep, n)
    plan.close()


@pytest.mark.parametrize("tree,exact", [("dt", 8), ("msdt", 8), ("msdt", 9), ("msdt", 10)])
def test_fused_pp_init_single_child_resynced(dev, tree, exact):
    """Forced PP schedule re-synced to the GPU's factors before each step
    (eight to ten regular sweeps, so that the approximated steps are valid at
    this point of the run; initialization with its approximated sweep, one
    more approximated sweep, a regular sweep, a second initialization) on a
    shape where the regular sweeps take the fused forms and the
    initialization's node with one pair child forms that pair in one pass
    where a fused kernel takes the mode pair.  Under MSDT the live node
    lacks mode 1 after eight sweeps (the single child: modes 2 then 0,
    k_ttm_qg), mode 0 after nine (modes 1 then 3: k_ttm_qr over 32 slices of
    mode 0) and mode 2 after ten (the pair of modes 3 and 1, taken as 1 then 3
by the same kernel, since a pair does not depend on the order); under the fused
    standard tree no node is live (modes 0 then 2).  Against the oracle's PP
    steps: fitness within 1e-6, factors within 1e-4."""
    from oracle import core, pp
    from paper_2010_12056_amd import cpals, synth

    dims, R = (32, 32, 64, 128), 40
    say(f"case fused pp init dims={dims} R={R} {tree} after {exact} sweeps")
    w = synth.planted_tensor(dims, R, 950 + R, noise_rel=1e-2, dtype=np.float32)
    plan = cpals.Plan(dims, R, prec="f32", tree=tree, device=dev)
    plan.set_tensor(torch.from_numpy(w.T).to(dev))
    A = to_dev(w.init, dev)
    st = pp.PPState.start(w.T.astype(np.float64), w.init)
    for step, kind in enumerate(["exact"] * exact + ["init", "approx", "exact", "init"]):
        st.A = [a.cpu().numpy().copy() for a in A]
        st.S = [core.gram(a) for a in st.A]
        if st.phase == "pp":
            st.dA = [st.A[i] - st.Ap[i] for i in range(len(st.A))]
        info = plan.pp_sweep(A, mode=kind)
        pp.pp_als_step(st, force=kind)
        say(f"  step {step} {kind} fit {info['fitness']:.10f} oracle {st.last_fit_est:.10f}")
        assert info["kind"] == kind
        assert not info["r_clamped"], (step, kind)
        assert abs(info["fitness"] - st.last_fit_est) <= 1e-6, (step, kind, info["fitness"], st.last_fit_est)
        for n in range(len(dims)):
            assert relerr(A[n].cpu().numpy(), st.A[n]) <= 1e-4, (step, n)
    plan.close()


def test_fused_config_o4_s128_r64_sampled(dev):
    """Full-size order-4 128^4 FP32 tensor, R = 64: the MTTKRPs of every mode
    on sampled rows computed one by one by the
    oracle's definition (modes 0 and 1 from the fused leading half, 2 and 3
    from the fused trailing half), with the signed bias bound of the other
    full-size checks."""
    from oracle import core
    from paper_2010_12056_amd import cpals, synth

    say("case fused mttkrp o4_s128_r64 full size")
    w = synth.workload("o4_s128_r64_f32")
    plan = cpals.Plan(w.dims, w.R, prec="f32", tree="dt", device=dev)
    plan.set_tensor(torch.from_numpy(w.T).to(dev))
    A = to_dev(w.init, dev)
    rng = np.random.default_rng(3)
    for n in range(4):
        rows = rng.choice(w.dims[n], size=6, replace=False)
        K = core.krp([w.init[m] for m in range(4) if m != n])
        X = np.moveaxis(w.T, n, 0)
        ref = np.stack([X[i].astype(np.float64).reshape(-1) @ K for i in rows])
        M = plan.mttkrp(A, n).cpu().numpy()[rows]
        e = relerr(M, ref)
        bias = float(np.mean(M - ref) / np.mean(np.abs(ref)))
        say(f"  mode {n} relerr {e:.2e} bias {bias:.1e}")
        assert e <= 1e-5
        assert abs(bias) <= 1e-8, (n, bias)
        del K
    plan.close()
