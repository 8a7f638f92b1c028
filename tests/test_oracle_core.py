"""Pins of the FP64 oracle's core definitions (CPU only).

Each test checks an oracle function against something other than itself:
a hand-worked fixture, brute-force index sums, a library routine, or an
identity that the mathematics fixes."""

import itertools
import os

import numpy as np
import pytest

import oracle
from oracle import core

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_2x2x2():
    T = np.array([[[1 + 4 * i + 2 * j + k for k in range(2)] for j in range(2)] for i in range(2)], dtype=float)
    A = [np.array([[1.0, 1.0], [2.0, 1.0]]), np.array([[3.0, 1.0], [-1.0, 1.0]]), np.array([[2.0, 1.0], [5.0, 1.0]])]
    want = {}
    scalars = {}
    with open(os.path.join(GOLDEN, "mttkrp_2x2x2.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            p = line.split()
            if p[0] == "M":
                want[(int(p[1]), int(p[2]), int(p[3]))] = float(p[4])
            else:
                scalars[p[0]] = float(p[1])
    return T, A, want, scalars


@pytest.mark.parametrize("fn", [core.mttkrp_naive, core.mttkrp_bruteforce])
def test_mttkrp_hand_worked_fixture(fn):
    T, A, want, _ = _golden_2x2x2()
    for n in range(3):
        M = fn(T, A, n)
        for (mode, row, col), v in want.items():
            if mode == n:
                assert M[row, col] == v


def test_residual_hand_worked_fixture():
    T, A, want, sc = _golden_2x2x2()
    ones = [np.ones((2, 1)) for _ in range(3)]
    assert float(np.sum(T * T)) == sc["NORMT2"]
    S = [core.gram(a) for a in ones]
    G = core.gamma(S, 2)
    M = core.mttkrp_naive(T, ones, 2)
    r = core.residual_fast(sc["NORMT2"], G, S[2], M, ones[2])
    assert abs(r - np.sqrt(sc["RESID2_ONES"] / sc["NORMT2"])) < 1e-15
    assert abs(core.residual_explicit(T, ones) - np.sqrt(sc["RESID2_ONES"] / sc["NORMT2"])) < 1e-15


def test_krp_column_identity():
    rng = np.random.default_rng(0)
    B, C, D = rng.random((3, 4)), rng.random((5, 4)), rng.random((2, 4))
    K = core.krp([B, C, D])
    assert K.shape == (30, 4)
    for k in range(4):
        np.testing.assert_array_equal(K[:, k], np.kron(np.kron(B[:, k], C[:, k]), D[:, k]))


@pytest.mark.parametrize("N", [3, 4, 5, 6])
def test_mttkrp_naive_equals_bruteforce(N):
    rng = np.random.default_rng(N)
    for trial in range(3):
        dims = tuple(int(x) for x in rng.integers(1, 4 if N >= 5 else 6, size=N))
        R = int(rng.integers(1, 5))
        T = rng.standard_normal(dims)
        A = [rng.standard_normal((d, R)) for d in dims]
        for n in range(N):
            a = core.mttkrp_naive(T, A, n)
            b = core.mttkrp_bruteforce(T, A, n)
            np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-13 * np.abs(b).max())


def test_partial_mttkrp_consistency():
    rng = np.random.default_rng(7)
    dims = (3, 4, 2, 5)
    R = 3
    T = rng.standard_normal(dims)
    A = [rng.standard_normal((d, R)) for d in dims]
    # keeping one mode is the MTTKRP
    for n in range(4):
        np.testing.assert_allclose(core.partial_mttkrp(T, A, [n]), core.mttkrp_naive(T, A, n), rtol=1e-13, atol=1e-13)
    # keeping every mode returns T (times an all-ones rank axis)
    X = core.partial_mttkrp(T, A, [0, 1, 2, 3])
    for k in range(R):
        np.testing.assert_allclose(X[..., k], T, rtol=0, atol=0)
    # keeping a pair, brute-force index sums of Eq. (4)
    P = core.partial_mttkrp(T, A, [1, 3])
    ref = np.zeros((4, 5, R))
    for idx in itertools.product(*[range(d) for d in dims]):
        for k in range(R):
            ref[idx[1], idx[3], k] += T[idx] * A[0][idx[0], k] * A[2][idx[2], k]
    np.testing.assert_allclose(P, ref, rtol=1e-13, atol=1e-13)


def test_reconstruct_bruteforce():
    rng = np.random.default_rng(3)
    dims = (3, 2, 4)
    R = 2
    A = [rng.standard_normal((d, R)) for d in dims]
    ref = np.zeros(dims)
    for i, j, k in itertools.product(*[range(d) for d in dims]):
        ref[i, j, k] = sum(A[0][i, r] * A[1][j, r] * A[2][k, r] for r in range(R))
    np.testing.assert_allclose(core.reconstruct(A), ref, rtol=1e-14, atol=1e-14)


def test_spd_solve_matches_numpy():
    rng = np.random.default_rng(11)
    B = rng.standard_normal((20, 8))
    G = B.T @ B + 0.1 * np.eye(8)
    M = rng.standard_normal((13, 8))
    A, used = core.spd_solve(G, M)
    assert not used
    np.testing.assert_allclose(A, np.linalg.solve(G, M.T).T, rtol=1e-12, atol=1e-12)


def test_spd_solve_pinv_fallback():
    rng = np.random.default_rng(12)
    B = rng.standard_normal((20, 5))
    B[:, 4] = 0.0  # a zero factor column makes Gamma singular
    G = B.T @ B
    M = rng.standard_normal((6, 5))
    A, used = core.spd_solve(G, M)
    assert used
    np.testing.assert_allclose(A, M @ np.linalg.pinv(G, rcond=5 * np.finfo(float).eps, hermitian=True), rtol=1e-10, atol=1e-12)


def test_spd_solve_drops_numerically_singular_directions():
    """Alg. 1 writes the pseudo-inverse: a direction whose eigenvalue is below
    the numerical-rank cutoff is dropped even where a Cholesky factorization
    would still succeed (and return entries of order 1e19)."""
    rng = np.random.default_rng(13)
    B = rng.standard_normal((20, 5))
    B[:, 4] = 1e-10 * rng.standard_normal(20)
    G = B.T @ B
    M = rng.standard_normal((6, 5))
    A, used = core.spd_solve(G, M)
    assert used
    ref = np.zeros((6, 5))
    ref[:, :4] = M[:, :4] @ np.linalg.inv(G[:4, :4])
    np.testing.assert_allclose(A, ref, rtol=1e-7, atol=1e-8)


def test_gamma_is_hadamard_of_others():
    rng = np.random.default_rng(5)
    S = [rng.random((4, 4)) for _ in range(4)]
    G = core.gamma(S, 2)
    for a in range(4):
        for b in range(4):
            assert G[a, b] == S[0][a, b] * S[1][a, b] * S[3][a, b]
