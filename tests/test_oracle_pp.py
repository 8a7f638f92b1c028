"""Pins of the oracle's pairwise perturbation (CPU only)."""

import itertools

import numpy as np
import pytest

from oracle import core, pp
from paper_2010_12056_amd import synth


def _setup(dims=(6, 5, 7, 4), R=3, seed=40):
    w = synth.planted_tensor(dims, R, seed, noise_rel=1e-2, dtype=np.float64)
    rng = np.random.default_rng(seed + 1)
    Ap = [rng.random((d, R)) for d in dims]
    return w.T, Ap, rng


def test_operators_equal_eq4_bruteforce():
    T, Ap, _ = _setup(dims=(3, 4, 2, 3), R=2)
    pairs, mp = pp.pp_operators(T, Ap)
    dims = T.shape
    for (i, j), P in pairs.items():
        ref = np.zeros((dims[i], dims[j], 2))
        for idx in itertools.product(*[range(d) for d in dims]):
            for k in range(2):
                v = T[idx]
                for m in range(4):
                    if m not in (i, j):
                        v *= Ap[m][idx[m], k]
                ref[idx[i], idx[j], k] += v
        np.testing.assert_allclose(P, ref, rtol=1e-13, atol=1e-13)
    for n in range(4):
        np.testing.assert_allclose(mp[n], core.mttkrp_bruteforce(T, Ap, n), rtol=1e-13, atol=1e-13)


def test_zero_perturbation_is_exact():
    T, Ap, _ = _setup()
    pairs, mp = pp.pp_operators(T, Ap)
    dA = [np.zeros_like(a) for a in Ap]
    S = [core.gram(a) for a in Ap]
    for n in range(4):
        Mt = pp.pp_approx_mttkrp(pairs, mp, Ap, dA, S, n)
        np.testing.assert_allclose(Mt, core.mttkrp_naive(T, Ap, n), rtol=1e-12, atol=1e-12)


def test_single_perturbed_mode_is_exact():
    T, Ap, rng = _setup()
    pairs, mp = pp.pp_operators(T, Ap)
    for pert in range(4):
        A = [a.copy() for a in Ap]
        A[pert] = A[pert] + 0.3 * rng.standard_normal(A[pert].shape)
        dA = [A[i] - Ap[i] for i in range(4)]
        S = [core.gram(a) for a in A]
        for n in range(4):
            Mt = pp.pp_approx_mttkrp(pairs, mp, A, dA, S, n)
            ref = core.mttkrp_naive(T, A, n)
            np.testing.assert_allclose(Mt, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


def test_v_recurrence_equals_literal():
    rng = np.random.default_rng(9)
    N, R = 6, 5
    S = [rng.standard_normal((R, R)) for _ in range(N)]
    dS = [rng.standard_normal((R, R)) for _ in range(N)]
    A_n = rng.standard_normal((7, R))
    for n in range(N):
        V, W = pp.pp_v_literal(A_n, S, dS, n)
        np.testing.assert_allclose(pp.pp_v_recurrence(S, dS, n), W, rtol=1e-12, atol=1e-12)


def test_pp_error_is_second_order():
    """Halving a perturbation of every mode cuts the error of M~ by about 4x:
    the first-order terms are exact and V carries part of the second order."""
    T, Ap, rng = _setup(dims=(8, 7, 6, 9), R=3)
    pairs, mp = pp.pp_operators(T, Ap)
    D = [rng.standard_normal(a.shape) for a in Ap]
    errs = []
    for t in (0.1, 0.05, 0.025, 0.0125):
        A = [Ap[i] + t * D[i] for i in range(4)]
        dA = [t * D[i] for i in range(4)]
        S = [core.gram(a) for a in A]
        Mt = pp.pp_approx_mttkrp(pairs, mp, A, dA, S, 3)
        ref = core.mttkrp_naive(T, A, 3)
        errs.append(np.linalg.norm(Mt - ref) / np.linalg.norm(ref))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.5 < q < 4.6 for q in ratios), ratios


def test_pp_state_machine_first_step_exact_then_init():
    w = synth.planted_tensor((10, 9, 8), 3, 55, noise_rel=1e-3, dtype=np.float64)
    st = pp.PPState.start(w.T, w.init)
    kinds = [pp.pp_als_step(st, eps=0.2) for _ in range(25)]
    assert kinds[0] == "exact"  # dA = A at the start fails the test
    assert "init" in kinds
    i = kinds.index("init")
    assert all(k == "exact" for k in kinds[:i])
    # after an init only approximated sweeps follow until one regular sweep
    for a, b in zip(kinds, kinds[1:]):
        if b == "approx":
            assert a in ("init", "approx")


def test_first_two_updates_after_init_are_exact():
    w = synth.planted_tensor((8, 7, 9, 6), 3, 56, noise_rel=1e-3, dtype=np.float64)
    st = pp.PPState.start(w.T, w.init)
    for _ in range(3):
        pp.pp_als_step(st, force="exact")
    # replay one approximated sweep by hand next to an exact sweep from the same point
    st_exact = pp.PPState.start(w.T, st.A)
    pp._init(st)
    N = 4
    for n in range(N):
        G = core.gamma(st.S, n)
        Mt = pp.pp_approx_mttkrp(st.pairs, st.mp, st.A, st.dA, st.S, n)
        Me = core.mttkrp_naive(st.T, st.A, n)
        if n < 2:
            np.testing.assert_allclose(Mt, Me, rtol=1e-11, atol=1e-11 * np.abs(Me).max())
        else:
            assert np.abs(Mt - Me).max() > 0
        st.A[n], _ = core.spd_solve(G, Mt)
        st.dA[n] = st.A[n] - st.Ap[n]
        st.S[n] = core.gram(st.A[n])
    del st_exact


def test_forced_approx_outside_pp_phase_is_an_error():
    w = synth.planted_tensor((5, 6, 7), 2, 57, noise_rel=1e-3, dtype=np.float64)
    st = pp.PPState.start(w.T, w.init)
    with pytest.raises(RuntimeError):
        pp.pp_als_step(st, force="approx")


def test_pp_fitness_tracks_exact_near_convergence():
    """After many exact sweeps the factors barely move and an approximated
    sweep's exact fitness agrees with the estimate from M~^(N)."""
    w = synth.planted_tensor((12, 11, 10), 4, 58, noise_rel=1e-2, dtype=np.float64)
    st = pp.PPState.start(w.T, w.init)
    for _ in range(30):
        pp.pp_als_step(st, force="exact")
    f_exact_before = st.last_fit_exact
    pp.pp_als_step(st, force="init")
    assert abs(st.last_fit_est - st.last_fit_exact) < 1e-6
    assert st.last_fit_exact >= f_exact_before - 1e-9


def test_pp_error_is_third_order_at_exact_factors():
    """On a noiseless rank-R tensor expanded at its own factors, V^(n) matches
    the second-order term of the MTTKRP, so the error of M~ is third order:
    about 8x smaller per halving of the perturbation.  This pins the sign and
    operands of Eq. (7)."""
    rng = np.random.default_rng(5)
    dims, R = (8, 7, 6, 9), 3
    B = [rng.random((d, R)) for d in dims]
    T = core.reconstruct(B)
    pairs, mp = pp.pp_operators(T, B)
    D = [rng.standard_normal(b.shape) for b in B]
    for n in range(4):
        errs = []
        for t in (0.05, 0.025, 0.0125):
            A = [B[i] + t * D[i] for i in range(4)]
            dA = [t * D[i] for i in range(4)]
            S = [core.gram(a) for a in A]
            Mt = pp.pp_approx_mttkrp(pairs, mp, A, dA, S, n)
            ref = core.mttkrp_naive(T, A, n)
            errs.append(np.linalg.norm(Mt - ref) / np.linalg.norm(ref))
        ratios = [errs[i] / errs[i + 1] for i in range(2)]
        assert all(7.0 < q < 9.0 for q in ratios), (n, ratios)
