"""The configurations of the benchmark family at their own shapes, against
the FP64 oracle: the order-3 64^3 FP64 tensor (planted rank 16, noise 1e-3,
R = 16) over its 20 sweeps, and the order-6 24^6 FP32 collinear tensor
(R = 32) through regular sweeps and one PP phase, with the oracle restarted
from the GPU's factors before every step."""

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


@pytest.mark.parametrize("tree", ["dt", "msdt"])
def test_order3_s64_r16_f64_twenty_sweeps(dev, tree):
    """20 sweeps from the seeded init, free running: the residual after every
    sweep within 1e-10 of the oracle's and the factors within 1e-9."""
    import oracle
    from paper_2010_12056_amd import synth

    say(f"case o3_s64_r16_f64 {tree}")
    w = synth.workload("o3_s64_r16_f64")
    plan, T, A = _plan(w, "f64", tree, dev)
    st = oracle.AlsState.start(w.T.astype(np.float64), w.init)
    for sweep in range(20):
        info = plan.als_sweep(A)
        r_ref = oracle.als_sweep(st)
        assert abs(info["r"] - r_ref) <= 1e-10, (sweep, info["r"], r_ref)
    for n in range(3):
        assert relerr(A[n].cpu().numpy(), st.A[n]) <= 1e-9, n
    say(f"  fitness after 20 sweeps {1.0 - info['r']:.10f}")
    plan.close()


def test_order3_s64_r16_f64_pp_auto(dev):
    """Alg. 2 (tolerance 0.1) over 20 outer steps: the GPU takes the
    oracle's decision at every step whose test inputs are not within 1e-6
    (relative) of the tolerance, and reports the oracle's fitness; the
    comparison stops at a decision the two sides may take differently."""
    from oracle import pp
    from paper_2010_12056_amd import synth

    eps = 0.1
    say("case o3_s64_r16_f64 pp auto")
    w = synth.workload("o3_s64_r16_f64")
    plan, T, A = _plan(w, "f64", "msdt", dev)
    st = pp.PPState.start(w.T.astype(np.float64), w.init)
    kinds = []
    for step in range(20):
        ratios = [np.linalg.norm(st.dA[i]) / np.linalg.norm(st.A[i]) for i in range(3)]
        close = any(abs(q - eps) <= 1e-6 * eps for q in ratios)
        info = plan.pp_sweep(A, tol=eps, mode="auto")
        kind = pp.pp_als_step(st, eps=eps)
        if close:
            say(f"  step {step}: a test input within 1e-6 of the tolerance; comparison stops")
            break
        assert info["kind"] == kind, (step, info["kind"], kind)
        assert abs(info["fitness"] - st.last_fit_est) <= 1e-9, (step, kind)
        kinds.append(kind)
    say(f"  schedule {kinds}")
    plan.close()


def test_order6_s24_r32_f32_collinear_resynced(dev):
    """The order-6 24^6 FP32 collinear tensor (R = 32) on the MSDT plan:
    two regular sweeps, then a PP initialization with its approximated
    sweep, the oracle restarted from the GPU's factors (A_p taken from them
    at the initialization) before every step: the fitness the step reports
    within 1e-6 of the oracle's for the same step (exact, then estimated).
    Every PP-tree level and all fifteen pair operators run at this order.
    A second approximated sweep here breaks the approximation on both sides
    (Eq. (3)'s estimate turns negative at this collinearity), so the phase
    stops at one."""
    from oracle import core, pp
    from paper_2010_12056_amd import synth

    say("case o6_s24_r32_f32_col re-synced")
    w = synth.workload("o6_s24_r32_f32_col")
    T64 = w.T.astype(np.float64)
    plan, T, A = _plan(w, "f32", "msdt", dev)
    st = pp.PPState.start(T64, w.init)
    for step, kind in enumerate(["exact", "exact", "init"]):
        st.A = [a.cpu().numpy().copy() for a in A]
        st.S = [core.gram(a) for a in st.A]
        if st.phase == "pp":
            st.dA = [st.A[i] - st.Ap[i] for i in range(len(st.A))]
        info = plan.pp_sweep(A, mode=kind)
        pp.pp_als_step(st, force=kind)
        say(f"  step {step} {kind}: fitness {info['fitness']:.8f} oracle {st.last_fit_est:.8f}")
        assert info["kind"] == kind
        assert not info["r_clamped"], (step, kind)
        assert abs(info["fitness"] - st.last_fit_est) <= 1e-6, (step, kind)
    plan.close()
    del T
    torch.cuda.empty_cache()
