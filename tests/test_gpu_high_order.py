"""GPU parity at orders 5 and 6 against the FP64 oracle.

These orders reach what orders 3 and 4 do not: the PP dimension tree's
levels 3 and 4 (Sec. II-D, Fig. 1b: level l keeps N - l modes and has
C(l+2, 2) nodes), five or more first-order pair corrections per mode
(Eqs. (5)-(6)), the bracket of Eq. (7) over several pairs, and the DT / MSDT
node reuse of deeper trees (Sec. II-C, III).

Forced PP schedules are chosen so that the approximation stays valid (PP
steps taken far from convergence at these orders break down: the estimated
residual of Eq. (3) turns negative while the exact fitness collapses, on the
oracle as on the GPU); their trajectories move by less than 1e-13 when the
oracle's initial factors are perturbed by 1e-14 (relative)."""

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


HIGH = ["o5_small_f64", "o6_small_f64", "o6_col_small_f64"]


@pytest.mark.parametrize("tree", ["dt", "msdt"])
@pytest.mark.parametrize("name", HIGH)
def test_als_free_running_high_order(dev, tree, name):
    """Two whole MSDT trees plus one sweep (2(N-1)+1 sweeps), FP64, fitness
    after every sweep and every factor against the oracle's Alg. 1; first-level
    contraction counts 2 per sweep (DT) and N per N-1 sweeps (MSDT)."""
    import oracle
    from paper_2010_12056_amd import synth

    say(f"case high-order als {name} {tree}")
    w = synth.workload(name)
    plan, T, A = _plan(w, "f64", tree, dev)
    st = oracle.AlsState.start(w.T.astype(np.float64), w.init)
    N = len(w.dims)
    sweeps = 2 * (N - 1) + 1
    ttm = 0
    for sweep in range(sweeps):
        info = plan.als_sweep(A)
        r_ref = oracle.als_sweep(st)
        ttm += info["ttm_count"]
        assert abs(info["r"] - r_ref) <= 1e-10, (sweep, info["r"], r_ref)
        for n in range(N):
            assert relerr(A[n].cpu().numpy(), st.A[n]) <= 1e-9, (sweep, n)
    if tree == "dt":
        assert ttm == 2 * sweeps
    else:
        assert ttm == -(-sweeps * N // (N - 1))
    plan.close()


@pytest.mark.parametrize("tree", ["dt", "msdt"])
@pytest.mark.parametrize("name", HIGH)
def test_mttkrp_every_mode_high_order(dev, tree, name):
    """MTTKRP of every mode from every first-level layout (root mode), FP64,
    against the explicit Khatri-Rao definition."""
    import oracle
    from paper_2010_12056_amd import cpals, synth

    w = synth.workload(name)
    plan, T, A = _plan(w, "f64", tree, dev)
    T64 = w.T.astype(np.float64)
    N = len(w.dims)
    for n in range(N):
        ref = oracle.mttkrp_naive(T64, w.init, n)
        assert relerr(plan.mttkrp(A, n).cpu().numpy(), ref) <= 1e-12, n
        for root in range(N):
            if root != n:
                M = plan.mttkrp(A, n, root=root).cpu().numpy()
                assert relerr(M, ref) <= 1e-12, (n, root)
    plan.close()


PP_SCHED = {
    "o5_small_f64": ["exact"] * 5 + ["init", "approx", "approx", "exact", "init", "approx", "approx"],
    "o6_small_f64": ["exact"] * 3 + ["init", "approx", "approx", "exact", "init", "approx"],
    "o6_col_small_f64": ["exact"] * 5 + ["init", "approx", "exact", "init", "approx"],
}


@pytest.mark.parametrize("tree", ["dt", "msdt"])
@pytest.mark.parametrize("name", HIGH)
def test_pp_forced_schedule_high_order(dev, tree, name):
    """FP64 forced schedule on both sides from the same init: the fitness the
    step reports (estimated for PP steps, Eq. (3) with M~^(N)), the exact
    fitness of the factors it leaves (audited on a second plan), and the
    factors, after every step.  The PP initialization at these orders builds
    the operators through every level of the PP tree."""
    from oracle import pp
    from paper_2010_12056_amd import cpals, synth

    say(f"case high-order pp forced {name} {tree}")
    w = synth.workload(name)
    plan, T, A = _plan(w, "f64", tree, dev)
    audit = cpals.Plan(w.dims, w.R, prec="f64", tree="dt", device=dev)
    audit.set_tensor(T)
    st = pp.PPState.start(w.T.astype(np.float64), w.init)
    N = len(w.dims)
    for step, kind in enumerate(PP_SCHED[name]):
        info = plan.pp_sweep(A, mode=kind)
        pp.pp_als_step(st, force=kind)
        assert info["kind"] == kind
        assert info["fitness_is_exact"] == (kind == "exact")
        assert not info["r_clamped"], (step, kind)
        assert abs(info["fitness"] - st.last_fit_est) <= 1e-9, (step, kind, info["fitness"], st.last_fit_est)
        f_exact = audit.fitness(A)
        assert abs(f_exact - st.last_fit_exact) <= 1e-9, (step, kind, f_exact, st.last_fit_exact)
        for n in range(N):
            assert relerr(A[n].cpu().numpy(), st.A[n]) <= 1e-8, (step, n)
    plan.close()
    audit.close()


AUTO_CASES = [("o5_small_f64", 0.05), ("o6_small_f64", 0.1), ("o6_col_small_f64", 0.05)]


@pytest.mark.parametrize("name,eps", AUTO_CASES)
def test_pp_auto_high_order(dev, name, eps):
    """Alg. 2's own schedule (the test ||dA_i|| < eps ||A_i|| for every i)
    over 20 outer steps: the GPU takes the oracle's decision at every step
    (every test input is at least 0.8 % away from eps here) and reports its
    fitness."""
    from oracle import pp
    from paper_2010_12056_amd import synth

    say(f"case high-order pp auto {name} {eps}")
    w = synth.workload(name)
    plan, T, A = _plan(w, "f64", "msdt", dev)
    st = pp.PPState.start(w.T.astype(np.float64), w.init)
    kinds = []
    for step in range(20):
        info = plan.pp_sweep(A, tol=eps, mode="auto")
        kind = pp.pp_als_step(st, eps=eps)
        assert info["kind"] == kind, (step, info["kind"], kind)
        assert abs(info["fitness"] - st.last_fit_est) <= 1e-9, (step, kind)
        kinds.append(kind)
    assert "init" in kinds and "approx" in kinds
    for n in range(len(w.dims)):
        assert relerr(A[n].cpu().numpy(), st.A[n]) <= 1e-8
    plan.close()
