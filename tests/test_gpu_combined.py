"""GPU parity of the dimension tree with its upper two levels combined
(CP_TREE_DT_COMBINED: the half of the tree that keeps the leading modes
starts with one contraction of the tensor against the Khatri-Rao product of
the last two factors, the memory / computation trade-off of Sec. IV) against
the FP64 oracle.  The combination changes how the MTTKRP is computed, not
what it is: every MTTKRP equals the explicit-KRP definition, and the sweeps
follow the oracle's trajectory."""

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
    # (dims, R, prec): orders 4, 5 and 6; combined lengths s_{N-2} s_{N-1} from 20 to 957
    # (the long ones take the chunked last-mode kernels), ragged row tiles
    ((40, 37, 33, 29), 20, "f64"),
    ((40, 37, 33, 29), 20, "f32"),
    ((12, 10, 9, 8, 7), 20, "f64"),
    ((16, 17, 15, 3, 5, 4), 33, "f32"),
    ((50, 60, 33, 9), 50, "f32"),
    ((64, 84, 33, 9), 50, "f64"),
    # combined lengths long enough for the split-K form (the K range spread
    # over 2 to 8 workgroup layers, partials summed in layer order), with a
    # ragged last layer and every column-block width
    ((24, 20, 40, 30), 24, "f32"),
    ((10, 12, 64, 70), 40, "f32"),
    ((9, 11, 40, 35), 20, "f64"),
    ((8, 9, 36, 40), 80, "f32"),
    ((7, 5, 6, 48, 50), 12, "f32"),
]


@pytest.mark.parametrize("dims,R,prec", CASES)
def test_combined_mttkrp_every_mode(dev, dims, R, prec):
    import oracle
    from paper_2010_12056_amd import cpals, synth

    say(f"case combined mttkrp dims={dims} R={R} prec={prec}")
    dt = np.float64 if prec == "f64" else np.float32
    w = synth.planted_tensor(dims, R, 500 + len(dims) + R, noise_rel=1e-2, dtype=dt)
    plan = cpals.Plan(dims, R, prec=prec, tree="dt_combined", device=dev)
    T = torch.from_numpy(w.T).to(dev)
    plan.set_tensor(T)
    A = to_dev(w.init, dev)
    T64 = w.T.astype(np.float64)
    tol = 1e-12 if prec == "f64" else 1e-5
    for n in range(len(dims)):
        ref = oracle.mttkrp_naive(T64, w.init, n)
        M = plan.mttkrp(A, n).cpu().numpy()
        e = relerr(M, ref)
        say(f"  mode {n}: relerr {e:.2e}")
        assert e <= tol, (n, e)
    plan.close()


@pytest.mark.parametrize("name,prec,fit_tol,fac_tol", [
    ("o4_small_f32", "f32", 1e-6, 1e-4),
    ("timelapse_small", "f64", 1e-10, 1e-9),
    ("coil_small", "f64", 1e-10, 1e-9),
])
def test_combined_als_free_running_trajectory(dev, name, prec, fit_tol, fac_tol):
    import oracle
    from paper_2010_12056_amd import cpals, synth

    say(f"case combined als {name}")
    w = synth.workload(name)
    plan = cpals.Plan(w.dims, w.R, prec=prec, tree="dt_combined", device=dev)
    T = torch.from_numpy(w.T).to(dev)
    plan.set_tensor(T)
    A = to_dev(w.init, dev)
    st = oracle.AlsState.start(w.T.astype(np.float64), w.init)
    N = len(w.dims)
    sweeps = 2 * (N - 1) + 1
    ttm = 0
    for sweep in range(sweeps):
        info = plan.als_sweep(A)
        r_ref = oracle.als_sweep(st)
        ttm += info["ttm_count"]
        assert abs(info["r"] - r_ref) <= fit_tol, (sweep, info["r"], r_ref)
        for n in range(N):
            assert relerr(A[n].cpu().numpy(), st.A[n]) <= fac_tol, (sweep, n)
    assert ttm == 2 * sweeps  # the combined contraction is the first level of its half
    plan.close()


def test_combined_pp_forced_schedule_fp64(dev):
    """PP initialization keeps its own tree (Fig. 1b) and finds no first-level
    node of the leading half cached (the combined tree never forms it): the
    forced schedule must still follow the oracle."""
    from oracle import pp
    from paper_2010_12056_amd import cpals, synth

    say("case combined pp forced timelapse_small")
    w = synth.workload("timelapse_small")
    plan = cpals.Plan(w.dims, w.R, prec="f64", tree="dt_combined", device=dev)
    T = torch.from_numpy(w.T).to(dev)
    plan.set_tensor(T)
    A = to_dev(w.init, dev)
    st = pp.PPState.start(w.T.astype(np.float64), w.init)
    sched = ["exact"] * 3 + ["init", "approx", "exact", "init", "approx"]
    for step, kind in enumerate(sched):
        info = plan.pp_sweep(A, mode=kind)
        pp.pp_als_step(st, force=kind)
        assert info["kind"] == kind
        assert abs(info["fitness"] - st.last_fit_est) <= 1e-9, (step, kind, info["fitness"], st.last_fit_est)
    for n in range(len(w.dims)):
        assert relerr(A[n].cpu().numpy(), st.A[n]) <= 1e-8
    plan.close()


@pytest.mark.parametrize("prec,u", [("bf16", 2.0 ** -8), ("bf16x2", 2.0 ** -16)])
def test_combined_bf16_mttkrp_bound(dev, prec, u):
    """BF16 tensor, combined first level: each entry of the Khatri-Rao operand
    is rounded once (to BF16, or split into two BF16 parts), so every MTTKRP
    entry obeys |M_gpu - M| <= (u + 1e-5) (|T_(n)| |P^(n)|) as in the
    single-mode first contraction."""
    import oracle
    from paper_2010_12056_amd import cpals, synth

    dims, R = (50, 60, 33, 9), 50
    say(f"case combined bf16 {dims} R={R} {prec}")
    w = synth.planted_tensor(dims, R, 777, noise_rel=1e-2, dtype=np.float32)
    bits = synth.bf16_bits(w.T)
    T64 = synth.bf16_to_f32(bits).astype(np.float64)
    plan = cpals.Plan(dims, R, prec=prec, tree="dt_combined", device=dev)
    T = torch.from_numpy(bits.view(np.int16)).to(dev).view(torch.bfloat16)
    plan.set_tensor(T)
    A = to_dev(w.init, dev)
    absT = np.abs(T64)
    absA = [np.abs(a) for a in w.init]
    for n in range(len(dims)):
        ref = oracle.mttkrp_naive(T64, w.init, n)
        refabs = oracle.mttkrp_naive(absT, absA, n)
        M = plan.mttkrp(A, n).cpu().numpy()
        q = float((np.abs(M - ref) / ((u + 1e-5) * np.maximum(refabs, 1e-300))).max())
        say(f"  mode {n}: error / bound {q:.3f}")
        assert q <= 1.0, (n, q)
    plan.close()
