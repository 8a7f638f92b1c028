"""Dimension trees (Sec. II-C, Fig. 1a), the multi-sweep dimension tree
(Sec. III, Fig. 2) and the PP dimension tree (Sec. II-D, Fig. 1b), written
independently of the GPU runtime, in FP64 NumPy, with flop counters.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The oracle's truth for an MTTKRP is `core.mttkrp_naive`; this module exists to
check the claims that DT and MSDT reach the same matrices ("no accuracy loss",
Sec. I and III) and to count work against the closed forms of Sec. II-C,
Sec. III and Table I.

Representation: an intermediate is the tensor of Eq. (4) keeping a set of
modes (in increasing order) with the rank index k as its last axis.  A node is
valid while every factor contracted into it still has the version it had when
the node was built; `DTCache.mttkrp` walks a root-to-leaf path, reuses the
deepest valid node and contracts one mode at a time below it.

Pins: DT == naive and MSDT == DT == naive to 1e-12 over two whole MSDT trees;
TTM counts (2 per DT sweep, N per N-1 MSDT sweeps), MSDT root order N, N-1,
..., 1, N, ... (Sec. III); flop counters == hand-derived closed forms whose
leading terms are Table I's; PP-tree node counts C(l+2, 2) and pair coverage.
"""

import itertools
from math import comb

import numpy as np

from .core import gamma, gram, residual_fast, spd_solve


def _split(lo, hi):
    """Balanced binary split of positions [lo, hi]: the left part takes the
    first ceil(len/2) positions."""
    n = hi - lo + 1
    mid = lo + (n + 1) // 2 - 1
    return mid


def _tree_path(order, leaf_pos):
    """Root-to-leaf list of contracted positions for a binary dimension tree
    over an ordered list of modes (positions 0..len-1).  Moving from a range to
    its left child contracts the right part's positions from the far end
    inward; moving to the right child contracts the left part's positions from
    the far end inward (the first contraction out of a range is the mode
    farthest from the leaf's half)."""
    lo, hi = 0, len(order) - 1
    contracted = []
    while lo < hi:
        mid = _split(lo, hi)
        if leaf_pos <= mid:
            contracted += list(range(hi, mid, -1))
            hi = mid
        else:
            contracted += list(range(lo, mid + 1))
            lo = mid + 1
    return contracted


def dt_path(N, n):
    """Contraction sequence (list of modes) of the standard DT for leaf n
    (Fig. 1a for N = 4: leaf 0 contracts 3, 2, 1; leaf 2 contracts 0, 1, 3)."""
    order = list(range(N))
    return [order[p] for p in _tree_path(order, n)]


def msdt_root_mode(N, u):
    """Root mode of the MSDT subtree that serves global update u (0-based).
    Subtree j = u // (N-1) has root T x_m A^(m) with m = N-1 - (j mod N): the
    paper's mode N - i + 1 for its i-th subtree (Sec. III)."""
    j = u // (N - 1)
    return (N - 1) - (j % N)


def msdt_path(N, u):
    """Contraction sequence for global update u under MSDT (Sec. III): the
    subtree's root contracts its root mode m, then a binary DT runs over the
    N-1 remaining modes in the cyclic order m+1, ..., m+N-1 (mod N)."""
    m = msdt_root_mode(N, u)
    order = [(m + t) % N for t in range(1, N)]
    t = u % (N - 1)
    assert order[t] == u % N
    return [m] + [order[p] for p in _tree_path(order, t)]


class DTCache:
    """Versioned cache of Eq. (4) intermediates with flop/TTM counters."""

    def __init__(self, T, A):
        self.T = np.asarray(T, dtype=np.float64)
        self.A = A  # list shared with the caller; factors are replaced, not mutated
        self.N = self.T.ndim
        self.R = A[0].shape[1]
        self.version = [0] * self.N
        self.cache = {}
        self.flops = 0
        self.ttm_count = 0
        self.ttm_modes = []

    def bump(self, n):
        """Record that factor n was replaced."""
        self.version[n] += 1

    def _contract(self, X, modes, m):
        """Contract mode m of node X (axes = sorted(modes) + [k]) with A^(m)."""
        ax = sorted(modes).index(m)
        Y = np.einsum(X, list(range(X.ndim)), self.A[m], [ax, X.ndim - 1],
                      [d for d in range(X.ndim) if d != ax])
        self.flops += 2 * X.size
        return Y

    def _root(self, m):
        """First-level TTM: T contracted with A^(m), k appended last."""
        Tm = np.moveaxis(self.T, m, -1)
        X = Tm @ self.A[m]
        self.flops += 2 * self.T.size * self.R
        self.ttm_count += 1
        self.ttm_modes.append(m)
        return X

    def mttkrp(self, contraction_seq):
        """Walk a root-to-leaf contraction sequence, reusing valid nodes."""
        N = self.N
        remaining = set(range(N))
        sets = []
        for m in contraction_seq:
            remaining = remaining - {m}
            sets.append(frozenset(remaining))
        start, X = -1, None
        for d in range(len(sets) - 1, -1, -1):
            key = sets[d]
            hit = self.cache.get(key)
            if hit is not None:
                Xc, vers = hit
                if all(self.version[m] == v for m, v in vers.items()):
                    start, X = d, Xc
                    break
        modes = set(range(N)) if start < 0 else set(sets[start])
        for d in range(start + 1, len(sets)):
            m = contraction_seq[d]
            X = self._root(m) if d == 0 else self._contract(X, modes, m)
            modes = set(sets[d])
            contracted = [c for c in range(N) if c not in modes]
            self.cache[sets[d]] = (X, {c: self.version[c] for c in contracted})
        assert X.ndim == 2
        return X


def dt_flops_closed(N, s, R):
    """Exact flops of one DT sweep for an equidimensional tensor, derived by
    hand from the tree of `dt_path` (leading term 4 s^N R, Sec. II-C, Table I)."""
    if N == 3:
        return 4 * s**3 * R + 6 * s**2 * R
    if N == 4:
        return 4 * s**4 * R + 4 * s**3 * R + 8 * s**2 * R
    raise NotImplementedError


def msdt_flops_closed(N, s, R):
    """Exact flops of N-1 MSDT sweeps (= N subtrees), derived by hand from
    `msdt_path` (leading term 2N/(N-1) s^N R per sweep, Sec. III, Table I)."""
    if N == 3:
        per_subtree = 2 * s**3 * R + 4 * s**2 * R
    elif N == 4:
        per_subtree = 2 * s**4 * R + 4 * s**3 * R + 6 * s**2 * R
    else:
        raise NotImplementedError
    return N * per_subtree


def pp_tree_levels(N, order=None):
    """Node sets of the PP dimension tree (Sec. II-D, Fig. 1b), level by level.

    Level l (1-based, nodes keep N - l modes) holds C(l+2, 2) nodes: mode i
    together with the run of N-l-1 consecutive modes starting at j, for
    positions 1 <= i < j <= l + 2.  (The printed index range C(l+1, 2) does
    not reproduce Fig. 1b; this one does, and at the last level it is every
    pair.)  `order` relabels positions to modes so that a different root set
    can be used; by default positions are the modes themselves.
    Returns a list (levels 1..N-2) of lists of frozensets of 0-based modes."""
    order = list(range(N)) if order is None else list(order)
    levels = []
    for l in range(1, N - 1):
        w = N - l - 1
        nodes = []
        for i, j in itertools.combinations(range(1, l + 3), 2):
            pos = {i} | set(range(j, j + w))
            assert max(pos) <= N
            nodes.append(frozenset(order[p - 1] for p in pos))
        assert len(nodes) == comb(l + 2, 2)
        levels.append(nodes)
    return levels


def als_sweep_tree(st, cache, paths):
    """One sweep of Alg. 1, as `oracle.als.als_sweep`, with each MTTKRP walked
    down a tree by `cache` (a DTCache built on st.T sharing the list st.A):
    paths[n] is the contraction sequence of the n-th update, e.g.
    dt_path(N, n) for the standard tree (Sec. II-C) or msdt_path(N, u) with
    the global update count u for MSDT (Sec. III).  Returns the new residual
    of Eq. (3)."""
    N = st.T.ndim
    G = M = None
    for n in range(N):
        G = gamma(st.S, n)
        M = cache.mttkrp(paths[n])
        st.A[n], pinv = spd_solve(G, M)
        st.used_pinv |= pinv
        cache.bump(n)
        st.S[n] = gram(st.A[n])
    st.r_old = st.r
    st.r = residual_fast(st.normT2, G, st.S[N - 1], M, st.A[N - 1])
    return st.r
