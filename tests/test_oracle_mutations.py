"""Planted mistakes in the oracle must trip its pins (CPU only).

Each case patches one plausible slip into a copy of an oracle routine and
checks that the corresponding pin statistic leaves its tolerance."""

import numpy as np

from oracle import core, pp
from paper_2010_12056_amd import synth


def _rng_case(dims, R, seed):
    rng = np.random.default_rng(seed)
    T = rng.standard_normal(dims)
    A = [rng.standard_normal((d, R)) for d in dims]
    return T, A


def test_reversed_krp_order_is_caught_by_bruteforce():
    T, A = _rng_case((3, 4, 5), 2, 1)

    def wrong(T, A, n):
        X = np.moveaxis(T, n, 0).reshape(T.shape[n], -1)
        K = core.krp([A[m] for m in range(T.ndim) if m != n][::-1])
        return X @ K

    errs = [np.abs(wrong(T, A, n) - core.mttkrp_bruteforce(T, A, n)).max() for n in range(3)]
    assert max(errs) > 1e-3


def test_gamma_including_own_gram_is_caught_by_normal_equations():
    w = synth.planted_tensor((8, 7, 6), 3, 2, noise_rel=1e-2, dtype=np.float64)
    A = [a.copy() for a in w.init]
    S = [core.gram(a) for a in A]
    for n in range(3):
        G = np.ones((3, 3))
        for m in range(3):
            G = G * S[m]  # slip: includes S^(n)
        M = core.mttkrp_naive(w.T, A, n)
        A[n], _ = core.spd_solve(G, M)
        S[n] = core.gram(A[n])
    G_right = core.gamma(S, 2)
    gap = abs(np.sum(M * A[2]) - np.sum(G_right * S[2])) / np.sum(G_right * S[2])
    assert gap > 1e-6


def test_unswapped_pair_axes_is_caught_by_single_mode_exactness():
    dims, R = (5, 6, 7, 4), 2
    w = synth.planted_tensor(dims, R, 3, noise_rel=1e-2, dtype=np.float64)
    rng = np.random.default_rng(4)
    Ap = [rng.random((d, R)) for d in dims]
    pairs, mp = pp.pp_operators(w.T, Ap)
    A = [a.copy() for a in Ap]
    A[0] = A[0] + 0.2 * rng.standard_normal(A[0].shape)
    dA = [A[i] - Ap[i] for i in range(4)]
    n = 2

    def wrong_pair(pairs, n, i):  # slip: never swaps, shapes only fit by accident or fail
        key = (min(n, i), max(n, i))
        P = pairs[key]
        return P if P.shape[0] == dims[n] else None

    M = np.array(mp[n])
    for i in range(4):
        if i == n:
            continue
        P = wrong_pair(pairs, n, i)
        if P is None:
            P = pairs[(min(n, i), max(n, i))].reshape(dims[n], -1, R)[:, : dims[i], :]
        M = M + np.einsum("xyk,yk->xk", P, dA[i])
    ref = core.mttkrp_naive(w.T, A, n)
    assert np.abs(M - ref).max() / np.abs(ref).max() > 1e-3


def test_flipped_v_sign_is_caught_by_error_order():
    dims, R = (8, 7, 6, 9), 3
    rng = np.random.default_rng(5)
    B = [rng.random((d, R)) for d in dims]
    T = core.reconstruct(B)
    pairs, mp = pp.pp_operators(T, B)
    D = [rng.standard_normal(b.shape) for b in B]
    errs = []
    for t in (0.05, 0.025):
        A = [B[i] + t * D[i] for i in range(4)]
        dA = [t * D[i] for i in range(4)]
        S = [core.gram(a) for a in A]
        dS = [A[i].T @ dA[i] for i in range(4)]
        V, _ = pp.pp_v_literal(A[3], S, dS, 3)
        Mt = pp.pp_mode_mttkrp(pairs, mp, dA, 3) - V  # slip: sign of V
        ref = core.mttkrp_naive(T, A, 3)
        errs.append(np.linalg.norm(Mt - ref) / np.linalg.norm(ref))
    # the correct method is third order here (ratio about 8); the slip is not
    assert errs[0] / errs[1] < 5.0
