"""Core definitions of CP-ALS (paper Sec. II-A and II-B), in FP64 NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Pins (tests marked "not gpu"):
  krp                -> column identity with np.kron (Sec. II-A definition)
  mttkrp_naive       -> brute-force index sums on tiny shapes; hand-worked
                        2x2x2 fixture under tests/golden/
  mttkrp_bruteforce  -> hand-worked fixture (independent of the KRP route)
  partial_mttkrp     -> equals mttkrp_naive when one mode is kept, equals T
                        when all are kept, and brute force on tiny shapes
  reconstruct        -> brute-force outer-product sums
  spd_solve          -> numpy.linalg.solve / numpy.linalg.pinv
  residual_fast      -> residual_explicit after an exact solve (Eq. (3) vs
                        Eq. (2)); the normal-equation identity <M,A> = <G,S>
"""

import itertools

import numpy as np


def krp(mats):
    """Khatri-Rao (column-wise Kronecker) product of a list of (s_i, R)
    matrices, left factor's row index slowest (Sec. II-A: column k of B (.) C
    is kron(b_k, c_k)).  An empty list gives a 1 x R row of ones."""
    if len(mats) == 0:
        raise ValueError("krp of an empty list needs R; use krp_or_ones")
    out = np.asarray(mats[0], dtype=np.float64)
    for m in mats[1:]:
        m = np.asarray(m, dtype=np.float64)
        out = (out[:, None, :] * m[None, :, :]).reshape(out.shape[0] * m.shape[0], out.shape[1])
    return out


def krp_or_ones(mats, R):
    if len(mats) == 0:
        return np.ones((1, R))
    return krp(mats)


def mttkrp_naive(T, A, n):
    """MTTKRP by definition with an explicit Khatri-Rao product (Sec. II-B):
    M^(n) = T_(n) P^(n), P^(n) the KRP of every factor except A^(n)."""
    T = np.asarray(T, dtype=np.float64)
    X = np.moveaxis(T, n, 0).reshape(T.shape[n], -1)
    K = krp([A[m] for m in range(T.ndim) if m != n])
    return X @ K


def mttkrp_bruteforce(T, A, n):
    """M^(n)[i_n, k] = sum over all other indices of T[i] * prod_{m != n} A^(m)[i_m, k].
    Pure-Python loops; tiny inputs only."""
    T = np.asarray(T, dtype=np.float64)
    N = T.ndim
    R = A[0].shape[1]
    M = np.zeros((T.shape[n], R))
    for idx in itertools.product(*[range(d) for d in T.shape]):
        t = T[idx]
        for k in range(R):
            p = t
            for m in range(N):
                if m != n:
                    p *= A[m][idx[m], k]
            M[idx[n], k] += p
    return M


def partial_mttkrp(T, A, keep):
    """Partially contracted intermediate of Eq. (4): the tensor keeps the modes
    in `keep` (in increasing order) and contracts every other mode with its
    factor, sharing the rank index k.  Returned shape: (s_keep..., R), k last."""
    T = np.asarray(T, dtype=np.float64)
    N = T.ndim
    keep = sorted(keep)
    other = [m for m in range(N) if m not in keep]
    R = A[0].shape[1]
    Xt = np.transpose(T, keep + other)
    kshape = [T.shape[m] for m in keep]
    X = Xt.reshape(int(np.prod(kshape, dtype=np.int64)), -1)
    K = krp_or_ones([A[m] for m in other], R)
    return (X @ K).reshape(kshape + [R])


def reconstruct(A):
    """[[A^(1), ..., A^(N)]] = sum_r a^(1)_r o ... o a^(N)_r (Sec. II-B)."""
    dims = [a.shape[0] for a in A]
    K = krp([np.asarray(a, dtype=np.float64) for a in A[1:]])
    return (np.asarray(A[0], dtype=np.float64) @ K.T).reshape(dims)


def gram(Amat):
    """S = A^T A (Sec. II-B)."""
    Amat = np.asarray(Amat, dtype=np.float64)
    return Amat.T @ Amat


def gamma(S, n):
    """Eq. (1): Hadamard product of every Gram matrix except S^(n)."""
    R = S[0].shape[0]
    G = np.ones((R, R))
    for m in range(len(S)):
        if m != n:
            G = G * S[m]
    return G


def spd_solve(G, M):
    """A = M G^dagger, the update of A^(i) in Alg. 1 (and Alg. 2), with the
    Moore-Penrose pseudo-inverse of the symmetric positive semidefinite
    G = Gamma^(i) taken by its definition: G = V diag(w) V^T (symmetric
    eigendecomposition), eigenvalues at or below R * eps * lambda_max treated
    as zero.  For a well-conditioned G this is G^-1.  Returns
    (A, rank_deficient) where rank_deficient says an eigenvalue was dropped."""
    G = np.asarray(G, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    if not np.all(np.isfinite(G)):
        raise np.linalg.LinAlgError("non-finite Gamma")
    w, V = np.linalg.eigh(G)
    cut = G.shape[0] * np.finfo(np.float64).eps * max(w.max(), 0.0)
    keep = w > cut
    winv = np.where(keep, 1.0 / np.where(keep, w, 1.0), 0.0)
    return M @ ((V * winv) @ V.T), bool(not keep.all())


def residual_fast(normT2, G_last, S_last, M_last, A_last):
    """Eq. (3) with the squared tensor norm under the root (the printed form
    has ||T||_F unsquared, which is dimensionally inconsistent):
    r = sqrt(||T||^2 + <Gamma^(N), S^(N)> - 2 <M^(N), A^(N)>) / ||T||,
    the squared numerator clamped at zero."""
    num = normT2 + float(np.sum(G_last * S_last)) - 2.0 * float(np.sum(M_last * A_last))
    return float(np.sqrt(max(num, 0.0) / normT2))


def residual_explicit(T, A):
    """Eq. (2): r = ||T - [[A]]||_F / ||T||_F."""
    T = np.asarray(T, dtype=np.float64)
    return float(np.linalg.norm(T - reconstruct(A)) / np.linalg.norm(T))
