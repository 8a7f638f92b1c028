"""Pairwise perturbation for CP-ALS (paper Sec. II-D, Alg. 2, Eqs. (4)-(8)),
FP64, followed step by step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings of the paper taken here (each is listed in the design notes):
  * PP operators M_p^(i,j) are stored once per unordered pair i < j with axes
    (s_i, s_j, R); U^(n,i) for i < n contracts the FIRST axis of the stored
    M_p^(i,n) (Eq. (6) with the pair's axes read in either order).
  * dS^(i) = A^(i)T dA^(i) uses the current A^(i) (Eq. (8)); V^(n) uses the
    current, not yet updated, A^(n) and sums unordered pairs i < j, both != n;
    an empty Hadamard product is the all-ones matrix (Eq. (7)).
  * dA means the per-sweep change after a regular sweep and the cumulative
    A - A_p inside the PP phase; at the start dA = A, so the first outer
    iteration always runs a regular sweep (Alg. 2).
  * The activation test is strict: for every mode, ||dA^(i)||_F <
    eps ||A^(i)||_F with the current A^(i) (Alg. 2).
  * Alg. 2 updates r only after regular sweeps; approximated sweeps report an
    estimated residual from M~^(N) through Eq. (3).

Pins: zero perturbation gives the exact MTTKRP; one perturbed mode gives it
exactly (the MTTKRP is multilinear and V^(n) needs two perturbed modes); the
error of M~ falls by about 4x when the perturbation is halved (second-order
method); the V recurrence equals the literal double sum; the operators equal
Eq. (4) by brute force on tiny shapes.
Parity unpinned: whole PP trajectories beyond these properties (the paper
prints no worked example) and AUTO-mode switching decisions.
"""

from dataclasses import dataclass, field

import numpy as np

from .core import gamma, gram, mttkrp_naive, partial_mttkrp, residual_fast, spd_solve


def pp_operators(T, Ap):
    """PP initialization (Alg. 2, the operator step; Eq. (4) with A_p):
    M_p^(i,j) for every pair i < j (axes s_i, s_j, R) and M_p^(n) for every n."""
    N = np.asarray(T).ndim
    pairs = {}
    for i in range(N):
        for j in range(i + 1, N):
            pairs[(i, j)] = partial_mttkrp(T, Ap, [i, j])
    mp = [mttkrp_naive(T, Ap, n) for n in range(N)]
    return pairs, mp


def pair_operator(pairs, n, i):
    """M_p^(n,i) with axes (s_n, s_i, R), read from the stored unordered pair."""
    if n < i:
        return pairs[(n, i)]
    return np.swapaxes(pairs[(i, n)], 0, 1)


def pp_v_literal(A_n, S, dS, n):
    """Eq. (7): V^(n) = A^(n) (sum_{i<j; i,j != n} dS^(i) * dS^(j) * prod_{k != i,j,n} S^(k))."""
    N = len(S)
    R = S[0].shape[0]
    W = np.zeros((R, R))
    for i in range(N):
        for j in range(i + 1, N):
            if i == n or j == n:
                continue
            H = dS[i] * dS[j]
            for k in range(N):
                if k not in (i, j, n):
                    H = H * S[k]
            W = W + H
    return A_n @ W, W


def pp_v_recurrence(S, dS, n):
    """The bracket of Eq. (7) as the coefficient of t^2 in the Hadamard
    product over k != n of (S^(k) + t dS^(k)), built by the recurrence
    e2 <- e2*S + e1*dS, e1 <- e1*S + e0*dS, e0 <- e0*S.  Algebraically the same
    matrix as the literal double sum; pinned against it."""
    R = S[0].shape[0]
    e0 = np.ones((R, R))
    e1 = np.zeros((R, R))
    e2 = np.zeros((R, R))
    for k in range(len(S)):
        if k == n:
            continue
        e2 = e2 * S[k] + e1 * dS[k]
        e1 = e1 * S[k] + e0 * dS[k]
        e0 = e0 * S[k]
    return e2


def pp_mode_mttkrp(pairs, mp, dA, n):
    """First-order part of Eq. (5): M_p^(n) + sum_{i != n} U^(n,i), with U by Eq. (6)."""
    N = len(dA)
    M = np.array(mp[n], copy=True)
    for i in range(N):
        if i == n:
            continue
        P = pair_operator(pairs, n, i)
        M = M + np.einsum("xyk,yk->xk", P, dA[i])
    return M


def pp_approx_mttkrp(pairs, mp, A, dA, S, n):
    """Eq. (5): M~^(n) = M_p^(n) + sum_{i != n} U^(n,i) + V^(n), with
    dS^(i) = A^(i)T dA^(i) from the current factors (Eq. (8))."""
    dS = [np.asarray(A[i]).T @ dA[i] for i in range(len(A))]
    V, _ = pp_v_literal(A[n], S, dS, n)
    return pp_mode_mttkrp(pairs, mp, dA, n) + V


@dataclass
class PPState:
    """State of Alg. 2 between outer iterations."""
    T: np.ndarray
    A: list
    S: list = field(default_factory=list)
    dA: list = field(default_factory=list)
    Ap: list = None
    pairs: dict = None
    mp: list = None
    normT2: float = 0.0
    phase: str = "exact"  # "exact" or "pp"
    r: float = 1.0
    r_old: float = 0.0
    last_fit_exact: float = None
    last_fit_est: float = None

    @classmethod
    def start(cls, T, A0):
        T = np.asarray(T, dtype=np.float64)
        A = [np.array(a, dtype=np.float64, copy=True) for a in A0]
        return cls(T=T, A=A, S=[gram(a) for a in A], dA=[a.copy() for a in A],
                   normT2=float(np.sum(T * T)))


def pp_test(st: PPState, eps):
    """Alg. 2 activation test: for all i, ||dA^(i)||_F < eps ||A^(i)||_F."""
    return all(np.linalg.norm(st.dA[i]) < eps * np.linalg.norm(st.A[i]) for i in range(len(st.A)))


def _regular_sweep(st: PPState):
    N = st.T.ndim
    before = [a.copy() for a in st.A]
    G = M = None
    for n in range(N):
        G = gamma(st.S, n)
        M = mttkrp_naive(st.T, st.A, n)
        st.A[n], _ = spd_solve(G, M)
        st.S[n] = gram(st.A[n])
    st.dA = [st.A[i] - before[i] for i in range(N)]
    st.phase = "exact"
    st.r_old = st.r
    st.r = residual_fast(st.normT2, G, st.S[N - 1], M, st.A[N - 1])
    st.last_fit_exact = 1.0 - st.r
    st.last_fit_est = st.last_fit_exact


def _approx_sweep(st: PPState):
    """Inner loop body of Alg. 2: for each mode n, Gamma^(n), M~^(n) by
    Eq. (5), A^(n) <- M~ Gamma^dagger, dA^(n) = A^(n) - A_p^(n), S^(n)."""
    N = st.T.ndim
    G = Mt = None
    for n in range(N):
        G = gamma(st.S, n)
        Mt = pp_approx_mttkrp(st.pairs, st.mp, st.A, st.dA, st.S, n)
        st.A[n], _ = spd_solve(G, Mt)
        st.dA[n] = st.A[n] - st.Ap[n]
        st.S[n] = gram(st.A[n])
    st.last_fit_est = 1.0 - residual_fast(st.normT2, G, st.S[N - 1], Mt, st.A[N - 1])
    # audit only: the exact residual of the same factors.  Eq. (3) is the
    # expansion of ||T - T~||^2 and holds for any factors once M^(N) is exact.
    M_exact = mttkrp_naive(st.T, st.A, N - 1)
    st.last_fit_exact = 1.0 - residual_fast(st.normT2, gamma(st.S, N - 1), st.S[N - 1], M_exact, st.A[N - 1])


def _init(st: PPState):
    """Alg. 2: A_p <- A, dA <- 0, then the PP operators at A_p."""
    st.Ap = [a.copy() for a in st.A]
    st.dA = [np.zeros_like(a) for a in st.A]
    st.pairs, st.mp = pp_operators(st.T, st.Ap)
    st.phase = "pp"


def pp_als_step(st: PPState, eps=None, force=None):
    """One outer step of Alg. 2 (one sweep of N updates).

    force=None runs the AUTO state machine with tolerance eps:
      phase exact and the test holds -> init, then an approximated sweep;
      phase pp and the test holds    -> an approximated sweep;
      otherwise                      -> a regular sweep.
    force in {"exact", "init", "approx"} replays a given schedule.
    Returns the kind actually run: "exact", "init" or "approx"."""
    if force is None:
        ok = pp_test(st, eps)
        if ok and st.phase == "exact":
            kind = "init"
        elif ok and st.phase == "pp":
            kind = "approx"
        else:
            kind = "exact"
    else:
        kind = force
    if kind == "exact":
        _regular_sweep(st)
    elif kind == "init":
        _init(st)
        _approx_sweep(st)
    elif kind == "approx":
        if st.phase != "pp":
            raise RuntimeError("approximated sweep requested outside the PP phase")
        _approx_sweep(st)
    else:
        raise ValueError(kind)
    return kind
