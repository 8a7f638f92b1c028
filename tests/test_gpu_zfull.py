"""Full-size order-4 128^4 FP32 workload (R = 64) against the FP64 oracle."""

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


def _plan(w, prec, tree, dev):
    from paper_2010_12056_amd import cpals

    plan = cpals.Plan(w.dims, w.R, prec=prec, tree=tree, device=dev)
    T = torch.from_numpy(w.T).to(dev)
    plan.set_tensor(T)
    return plan, T, to_dev(w.init, dev)


def test_o4_s128_r64_dt_msdt_against_oracle(dev):
    """Full-size order-4 128^4 FP32 workload, R = 64: three DT and three MSDT
    sweeps against the FP64 oracle (free running, same init)."""
    import oracle
    from paper_2010_12056_amd import synth

    say("case full-size o4_s128_r64_f32 sweeps")
    w = synth.workload("o4_s128_r64_f32")
    T64 = w.T.astype(np.float64)
    st = oracle.AlsState.start(T64, w.init)
    refs = [oracle.als_sweep(st) for _ in range(3)]
    for tree in ("dt", "msdt"):
        plan, T, A = _plan(w, "f32", tree, dev)
        for s in range(3):
            info = plan.als_sweep(A)
            say(f"  {tree} sweep {s} r={info['r']:.10f} oracle={refs[s]:.10f}")
            assert abs(info["r"] - refs[s]) <= 1e-6
        for n in range(4):
            assert relerr(A[n].cpu().numpy(), st.A[n]) <= 1e-4
        plan.close()
        del T
        torch.cuda.empty_cache()


def test_o4_s128_r64_pp_schedule_resynced_against_oracle(dev):
    """Full-size order-4 128^4 FP32 workload, R = 64, on the MSDT plan: the
    schedule Alg. 2 takes here with tolerance 0.1 (four regular sweeps, then
    PP initialization with its approximated sweep, then one more approximated
    sweep).  The oracle is restarted from the GPU's factors before every step
    (A_p taken from them at the initialization), so each comparison measures
    one step's rounding: the fitness the step reports (estimated from M~^(N)
    by Eq. (3) for PP steps, which must not have been clamped), the exact
    fitness of the factors it leaves (cp_fitness against the oracle's Eq. (2)
    audit), and the factors."""
    from oracle import core, pp
    from paper_2010_12056_amd import cpals, synth

    say("case full-size o4_s128_r64_f32 PP schedule")
    w = synth.workload("o4_s128_r64_f32")
    T64 = w.T.astype(np.float64)
    plan, T, A = _plan(w, "f32", "msdt", dev)
    audit = cpals.Plan(w.dims, w.R, prec="f32", tree="dt", device=dev)
    audit.set_tensor(T)
    st = pp.PPState.start(T64, w.init)
    for step, kind in enumerate(["exact"] * 4 + ["init", "approx"]):
        st.A = [a.cpu().numpy().copy() for a in A]
        st.S = [core.gram(a) for a in st.A]
        if st.phase == "pp":
            st.dA = [st.A[i] - st.Ap[i] for i in range(len(st.A))]
        info = plan.pp_sweep(A, mode=kind)
        pp.pp_als_step(st, force=kind)
        f_exact = audit.fitness(A)
        say(f"  step {step} {kind}: fitness {info['fitness']:.8f} oracle {st.last_fit_est:.8f}; "
            f"exact {f_exact:.8f} oracle {st.last_fit_exact:.8f}")
        assert info["kind"] == kind
        assert not info["r_clamped"], (step, kind)
        assert abs(info["fitness"] - st.last_fit_est) <= 1e-6, (step, kind)
        assert abs(f_exact - st.last_fit_exact) <= 1e-6, (step, kind)
        for n in range(4):
            e = relerr(A[n].cpu().numpy(), st.A[n])
            assert e <= 1e-4, (step, kind, n, e)
    plan.close()
    audit.close()
    del T
    torch.cuda.empty_cache()
