"""Pins of the oracle's ALS sweep, dimension trees and flop counters (CPU only)."""

import numpy as np
import pytest

import oracle
from oracle import core, trees
from oracle.als import AlsState, als_sweep
from paper_2010_12056_amd import synth


def _small_planted(dims, R, seed, noise=1e-2, kind="uniform"):
    w = synth.planted_tensor(dims, R, seed, kind=kind, noise_rel=noise, dtype=np.float64)
    return w.T, w.init, w


def test_als_residual_monotone_and_fast_equals_explicit():
    T, A0, _ = _small_planted((9, 11, 7, 8), 5, 21)
    st = AlsState.start(T, A0)
    prev = 1.0
    for _ in range(15):
        r, Ms = als_sweep(st, record_M=True)
        # Eq. (3) with the squared norm reproduces Eq. (2)
        assert abs(r - core.residual_explicit(T, st.A)) < 1e-10
        # normal equations of the last solve: <M^(N), A^(N)> = <Gamma^(N), S^(N)>
        G = core.gamma(st.S, 3)
        assert abs(np.sum(Ms[-1] * st.A[3]) - np.sum(G * st.S[3])) < 1e-9 * np.sum(G * st.S[3])
        # ALS never increases the residual
        assert r <= prev + 1e-12
        prev = r


def test_unsquared_norm_reading_is_wrong():
    """The printed Eq. (3) has ||T|| (not squared) under the root; only the
    squared reading reproduces Eq. (2), which fixes the reading."""
    T, A0, _ = _small_planted((6, 5, 4), 3, 22)
    st = AlsState.start(T, A0)
    r, Ms = als_sweep(st, record_M=True)
    G = core.gamma(st.S, 2)
    nT = np.sqrt(st.normT2)
    literal = np.sqrt(max(nT + np.sum(G * st.S[2]) - 2 * np.sum(Ms[-1] * st.A[2]), 0)) / nT
    assert abs(literal - core.residual_explicit(T, st.A)) > 1e-3
    assert abs(r - core.residual_explicit(T, st.A)) < 1e-12


def test_planted_noiseless_recovery():
    rng = np.random.default_rng(123)
    dims, R = (12, 14, 16), 4
    P = [rng.standard_normal((d, R)) for d in dims]
    T = core.reconstruct(P)
    A0 = [p + 1e-2 * rng.standard_normal(p.shape) for p in P]
    st = AlsState.start(T, A0)
    for _ in range(40):
        r = als_sweep(st)
    assert core.residual_explicit(T, st.A) < 1e-12
    # Eq. (3) subtracts terms of size ||T||^2, so in FP64 it cannot resolve a
    # residual below about sqrt(eps) ~ 1.5e-8
    assert r < 1e-7


def _run_tree(T, A0, path_fn, sweeps):
    """ALS where every MTTKRP comes from the versioned tree cache; each tree
    MTTKRP is compared with the naive definition on the same factors."""
    N = T.ndim
    A = [a.copy() for a in A0]
    S = [core.gram(a) for a in A]
    cache = trees.DTCache(T, A)
    worst = 0.0
    Ms = []
    for u in range(sweeps * N):
        n = u % N
        M = cache.mttkrp(path_fn(N, u))
        ref = core.mttkrp_naive(T, A, n)
        worst = max(worst, float(np.abs(M - ref).max() / np.abs(ref).max()))
        Ms.append(M)
        A[n], _ = core.spd_solve(core.gamma(S, n), M)
        S[n] = core.gram(A[n])
        cache.bump(n)
    return A, Ms, worst, cache


@pytest.mark.parametrize("N", [3, 4, 5])
def test_dt_and_msdt_equal_naive_and_each_other(N):
    dims = {3: (7, 6, 5), 4: (6, 5, 4, 7), 5: (4, 3, 5, 4, 3)}[N]
    T, A0, _ = _small_planted(dims, 3, 30 + N)
    sweeps = 2 * (N - 1)  # two whole MSDT trees
    A_dt, M_dt, w_dt, c_dt = _run_tree(T, A0, lambda N_, u: trees.dt_path(N_, u % N_), sweeps)
    A_ms, M_ms, w_ms, c_ms = _run_tree(T, A0, trees.msdt_path, sweeps)
    assert w_dt < 1e-12 and w_ms < 1e-12
    for a, b in zip(M_dt, M_ms):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(a).max())
    # TTM counts: 2 per DT sweep, N per N-1 MSDT sweeps
    assert c_dt.ttm_count == 2 * sweeps
    assert c_ms.ttm_count == N * sweeps // (N - 1)
    # MSDT root order N, N-1, ..., 1, N, ... (0-based N-1, ..., 0)
    assert c_ms.ttm_modes == [(N - 1 - j) % N for j in range(c_ms.ttm_count)]


def test_dt_tree_shape_matches_fig_1a():
    # Fig. 1a: M^(1,2,3) -> M^(1,2) -> M^(1), M^(2); M^(2,3,4) -> M^(3,4) -> M^(3), M^(4)
    assert trees.dt_path(4, 0) == [3, 2, 1]
    assert trees.dt_path(4, 1) == [3, 2, 0]
    assert trees.dt_path(4, 2) == [0, 1, 3]
    assert trees.dt_path(4, 3) == [0, 1, 2]


def test_msdt_subtrees_match_fig_2():
    # Fig. 2 (N = 4): subtree roots T x_4, T x_3, T x_2, T x_1 in that order,
    # each serving the next three updates in cyclic order.
    N = 4
    roots = [trees.msdt_path(N, u)[0] for u in range(12)]
    assert roots == [3] * 3 + [2] * 3 + [1] * 3 + [0] * 3
    served = [u % N for u in range(12)]
    assert served == [0, 1, 2, 3, 0, 1, 2, 3, 0, 1, 2, 3]
    # second subtree (root mode 3 in the paper's numbering) serves M^(4), M^(1)
    # from M^(1,4) and M^(2) from M^(1,2,4) directly
    assert trees.msdt_path(N, 3) == [2, 1, 0]
    assert trees.msdt_path(N, 4) == [2, 1, 3]
    assert trees.msdt_path(N, 5)[:1] == [2]


@pytest.mark.parametrize("N,s,R", [(3, 6, 3), (4, 5, 2), (4, 6, 3)])
def test_flop_counters_match_closed_forms(N, s, R):
    rng = np.random.default_rng(1)
    T = rng.standard_normal((s,) * N)
    A0 = [rng.random((s, R)) for _ in range(N)]
    _, _, _, c_dt = _run_tree(T, A0, lambda N_, u: trees.dt_path(N_, u % N_), N - 1)
    _, _, _, c_ms = _run_tree(T, A0, trees.msdt_path, N - 1)
    assert c_dt.flops == (N - 1) * trees.dt_flops_closed(N, s, R)
    assert c_ms.flops == trees.msdt_flops_closed(N, s, R)


@pytest.mark.parametrize("N", [3, 4])
def test_closed_forms_leading_terms_match_table_1(N):
    R = 64
    s = 4096
    dt = trees.dt_flops_closed(N, s, R)
    ms = trees.msdt_flops_closed(N, s, R) / (N - 1)
    assert abs(dt / (4 * s**N * R) - 1) < 2e-3
    assert abs(ms / (2 * N / (N - 1) * s**N * R) - 1) < 3e-3


def test_config2_flop_counts():
    # order 4, s = 128, R = 64: DT 69.265 GFLOP and MSDT 46.537 GFLOP per sweep
    # (hand arithmetic: 4*128^4*64 + 4*128^3*64 + 8*128^2*64, and
    #  4*(2*128^4*64 + 4*128^3*64 + 6*128^2*64) for three sweeps)
    assert trees.dt_flops_closed(4, 128, 64) == 69_264_736_256
    assert trees.msdt_flops_closed(4, 128, 64) == 139_611_602_944


@pytest.mark.parametrize("N", [3, 4, 5, 6])
def test_pp_tree_family(N):
    from math import comb
    levels = trees.pp_tree_levels(N)
    assert len(levels) == N - 2
    for l, nodes in enumerate(levels, start=1):
        assert len(nodes) == comb(l + 2, 2)
        assert len(set(nodes)) == len(nodes)
        assert all(len(x) == N - l for x in nodes)
        if l > 1:
            for x in nodes:
                assert any(x < p for p in levels[l - 2])
    pairs = {frozenset(p) for p in [(i, j) for i in range(N) for j in range(i + 1, N)]}
    assert set(levels[-1]) == pairs
    if N == 4:
        # Fig. 1b: M_p^(1,2,3), M_p^(1,3,4), M_p^(2,3,4)
        assert set(levels[0]) == {frozenset({0, 1, 2}), frozenset({0, 2, 3}), frozenset({1, 2, 3})}


@pytest.mark.parametrize("N", [3, 4])
def test_tree_sweeps_follow_the_naive_sweep(N):
    """The oracle's DT and MSDT sweeps (MTTKRPs walked down the trees, used
    for the host timings) follow the naive-MTTKRP sweep's trajectory: the same
    residual after every sweep and the same factors, over two whole MSDT
    trees (Sec. III: no accuracy loss)."""
    from oracle import als

    dims = {3: (7, 6, 5), 4: (6, 5, 4, 7)}[N]
    T, A0, _ = _small_planted(dims, 3, 50 + N)
    sweeps = 2 * (N - 1)
    ref = als.AlsState.start(T, A0)
    st_dt = als.AlsState.start(T, A0)
    st_ms = als.AlsState.start(T, A0)
    c_dt = trees.DTCache(T, st_dt.A)
    c_ms = trees.DTCache(T, st_ms.A)
    u = 0
    for _ in range(sweeps):
        r = als.als_sweep(ref)
        r_dt = trees.als_sweep_tree(st_dt, c_dt, [trees.dt_path(N, n) for n in range(N)])
        r_ms = trees.als_sweep_tree(st_ms, c_ms, [trees.msdt_path(N, u + n) for n in range(N)])
        u += N
        assert abs(r_dt - r) <= 1e-12 and abs(r_ms - r) <= 1e-12
        for n in range(N):
            np.testing.assert_allclose(st_dt.A[n], ref.A[n], rtol=1e-10, atol=1e-12)
            np.testing.assert_allclose(st_ms.A[n], ref.A[n], rtol=1e-10, atol=1e-12)
    assert c_dt.ttm_count == 2 * sweeps and c_ms.ttm_count == N * sweeps // (N - 1)
