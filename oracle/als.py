"""Plain CP-ALS sweeps (paper Alg. 1, Sec. II-B), FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The MTTKRP inside a sweep is always the naive explicit-KRP definition: DT and
MSDT reach the same matrices exactly (Sec. III), so the oracle does not need a
tree to be right; `oracle.trees` re-derives the trees independently to check
that claim and to count flops.

Pins: monotone residual over exact sweeps (ALS decreases the residual, Sec. I);
Eq. (3) equals Eq. (2) after a sweep; normal equations <M,A> = <Gamma,S> after
an exact solve; planted noiseless recovery to r < 1e-10.
"""

from dataclasses import dataclass, field

import numpy as np

from .core import gamma, gram, mttkrp_naive, residual_fast, spd_solve


@dataclass
class AlsState:
    T: np.ndarray
    A: list
    S: list = field(default_factory=list)
    normT2: float = 0.0
    r: float = 1.0
    r_old: float = 0.0
    used_pinv: bool = False

    @classmethod
    def start(cls, T, A0):
        T = np.asarray(T, dtype=np.float64)
        A = [np.array(a, dtype=np.float64, copy=True) for a in A0]
        return cls(T=T, A=A, S=[gram(a) for a in A], normT2=float(np.sum(T * T)))


def als_sweep(st: AlsState, record_M=False):
    """One sweep of Alg. 1: for each mode n in order, Gamma^(n) by Eq. (1),
    M^(n) by definition, A^(n) <- M^(n) Gamma^(n)^dagger, S^(n) <- A^T A; then
    r_old <- r and r from Eq. (3).  Returns the new residual (and the list of
    MTTKRP matrices if record_M)."""
    N = st.T.ndim
    Ms = []
    G = M = None
    st.used_pinv = False
    for n in range(N):
        G = gamma(st.S, n)
        M = mttkrp_naive(st.T, st.A, n)
        st.A[n], pinv = spd_solve(G, M)
        st.used_pinv |= pinv
        st.S[n] = gram(st.A[n])
        if record_M:
            Ms.append(M)
    st.r_old = st.r
    st.r = residual_fast(st.normT2, G, st.S[N - 1], M, st.A[N - 1])
    return (st.r, Ms) if record_M else st.r


def als_run(T, A0, sweeps, tol=None):
    """Alg. 1 outer loop: at most `sweeps` sweeps, stopping early when
    |r - r_old| <= tol (if tol is given).  Returns (state, residuals)."""
    st = AlsState.start(T, A0)
    rs = []
    for _ in range(sweeps):
        rs.append(als_sweep(st))
        if tol is not None and abs(st.r - st.r_old) <= tol:
            break
    return st, rs
