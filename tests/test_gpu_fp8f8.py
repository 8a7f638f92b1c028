"""GPU parity of the FP8 x FP8 first contraction (CP_FP8F8: E4M3 tensor, the
contracted factor quantized per column to E4M3 after a power-of-two scale,
products on the FP8 matrix cores, FP32 accumulation, FP32 levels below).

MTTKRP parity: the oracle quantizes the same FP32 copy of the root's factor
(oracle.quantize_columns, written from the format's definition) and takes
the MTTKRP of the FP8 tensor values with it and the FP32 copies of the other
factors in FP64.  Both operands of every product are then the same E4M3
values on both sides and each product is exact.  What is left is the matrix
instruction's own summation and FP32 accumulation.  Measured on gfx950
(v_mfma_f32_16x16x32_fp8_fp8, one output element fed with powers of two):
each lane's group of eight products is summed in a fixed-point window under
the group's largest product (a product 2^-12 below it kept exactly, one 2^-14
below dropped), groups and the accumulator at FP32 precision.  The kernel's
groups are eight consecutive contraction indices (k = 8 j .. 8 j + 7), so a
first-level entry is off by less than 8 * 2^-12 max_{k in group} |x_k b_k|
summed over its groups, carried down the FP32 levels by the absolute values
of the other factors, plus f = 1e-5 of |T_(n)| |P^(n)| for FP32:
    |M_gpu - M| <= 2^-9 W + f |T_(n)| |P^(n)|      elementwise.
Sweeps: the DT sweep's Eq. (3) residual against the oracle's Eq. (3) with the
last MTTKRP formed from the same quantized factor, to the same bound; and
the error of each sweep against the exact (Eq. (2)) residual of the same
factors, which the factor's quantization brings (stated, and bounded by the
E4M3 rounding of every entry of the contracted factor)."""

import numpy as np
import pytest

from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FP32_ALLOWANCE = 1e-5


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _case(dims, R, seed, kind="uniform", noise_rel=1e-2):
    from paper_2010_12056_amd import synth

    w = synth.planted_tensor(dims, R, seed, kind=kind, noise_rel=noise_rel, dtype=np.float32)
    bits = synth.fp8_bits(w.T, scale=synth.fp8_scale(w.T))
    T64 = synth.fp8_to_f32(bits).astype(np.float64)
    return w, bits, T64


def _dev_fp8(bits, dev):
    return torch.from_numpy(np.ascontiguousarray(bits)).to(dev).view(torch.float8_e4m3fn)


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _used_factors(A, root):
    """The factors as the contraction uses them: FP32 copies, the root's
    quantized by the oracle."""
    import oracle

    used = [_f32(a) for a in A]
    used[root] = oracle.quantize_columns(used[root])[0]
    return used


GROUP = 8          # contraction indices summed together by one lane of the FP8 instruction
WINDOW = 2.0 ** -9  # 8 products, each off by less than 2^-12 of the group's largest


def _group_bound(absT, absB, root):
    """sum over the groups of eight consecutive indices of mode `root` of
    max_{k in group} |T| |B[k, r]|: shape of T with mode `root` replaced by
    a trailing rank index."""
    X = np.moveaxis(absT, root, -1)
    K = X.shape[-1]
    pad = (-K) % GROUP
    out = np.empty(X.shape[:-1] + (absB.shape[1],))
    for r in range(absB.shape[1]):
        Y = X * absB[:, r]
        if pad:
            Y = np.concatenate([Y, np.zeros(Y.shape[:-1] + (pad,))], axis=-1)
        out[..., r] = Y.reshape(Y.shape[:-1] + (-1, GROUP)).max(axis=-1).sum(axis=-1)
    return out


def _carry(node, absA, n, root):
    """The first-level bound `node` (modes other than root, rank last)
    contracted with |A| of every mode other than n and root."""
    modes = [m for m in range(len(absA)) if m != root]
    Y = node
    for m in reversed(modes):
        if m == n:
            continue
        ax = modes.index(m)
        Y = np.moveaxis(Y, ax, -2)
        Y = np.einsum("...ir,ir->...r", Y, absA[m])
        modes.remove(m)
    return Y


def _bound(absT, used, n, root):
    import oracle

    absA = [np.abs(a) for a in used]
    w = _carry(_group_bound(absT, absA[root], root), absA, n, root)
    return WINDOW * w + FP32_ALLOWANCE * oracle.mttkrp_naive(absT, absA, n)


def _every_mode_and_root(dev, dims, R, w, bits, T64, tree="dt"):
    import oracle
    from paper_2010_12056_amd import cpals

    plan = cpals.Plan(dims, R, prec="fp8f8", tree=tree, device=dev)
    plan.set_tensor(_dev_fp8(bits, dev))
    A = to_dev(w.init, dev)
    N = len(dims)
    absT = np.abs(T64)
    worst = 0.0
    for n in range(N):
        for root in [m for m in range(N) if m != n]:
            used = _used_factors(w.init, root)
            ref = oracle.mttkrp_naive(T64, used, n)
            M = plan.mttkrp(A, n, root=root).cpu().numpy()
            q = float((np.abs(M - ref) / np.maximum(_bound(absT, used, n, root), 1e-300)).max())
            worst = max(worst, q)
            assert q <= 1.0, (n, root, q)
    plan.close()
    return worst


CASES = [
    # (dims, R).  Last-mode contraction: three register sets with 16-byte rows (K = 512, 80, 96;
    # with R > 64 one set, since three would not fit beside 128 columns), one set (K = 48 with a
    # clamped tail, K = 16 below one chunk), 4-byte loads (K = 12, 8, 40), byte loads (K = 29).
    # Other modes: the LDS-staged chunk read with the transposing 8-bit LDS read (Q % 16 == 0),
    # groups of four q (Q % 4 == 0), guarded (odd Q); ragged K (17, 37, 520); R = 1 ... 128.
    ((40, 37, 33, 29), 20),
    ((24, 17, 512), 128),
    ((8, 520, 12), 33),
    ((300, 12, 8), 64),
    ((3, 1, 5, 2, 4), 1),
    ((48, 72, 40), 24),
    ((36, 20, 48), 50),
    ((64, 9, 6, 16), 17),
    ((40, 30, 80), 24),
    ((600, 250, 96), 20),
    ((32, 48, 96), 100),
]


@pytest.mark.parametrize("dims,R", CASES)
def test_fp8f8_mttkrp_every_mode_and_root(dev, dims, R):
    say(f"case fp8f8 mttkrp dims={dims} R={R}")
    w, bits, T64 = _case(dims, R, 1900 + len(dims) + R)
    worst = _every_mode_and_root(dev, dims, R, w, bits, T64)
    say(f"  worst error / bound {worst:.3f}")


def test_fp8f8_every_finite_code_and_wide_columns(dev):
    """Tensor entries drawn from all 254 finite codes, factor columns spread
    over 2^-30 .. 2^30 (each column's scale moves it into range) with a zero
    column and entries down in the subnormal range of their column."""
    from paper_2010_12056_amd import synth

    dims, R = (40, 36, 48), 24
    say(f"case fp8f8 all codes {dims} R={R}")
    rng = np.random.default_rng(171)
    finite = np.array([c for c in range(256) if c not in (0x7F, 0xFF)], dtype=np.uint8)
    bits = rng.choice(finite, size=dims)
    T64 = synth.fp8_to_f32(bits).astype(np.float64)
    w = synth.planted_tensor(dims, R, 172, noise_rel=0.0, dtype=np.float32)
    col = 2.0 ** rng.integers(-30, 31, size=R)
    for m in range(3):
        a = w.init[m] * col[None, :]
        a[:, 3] = 0.0
        a[: dims[m] // 4, 5] *= 2.0 ** -14  # subnormal after the column's scale
        w.init[m] = a
    worst = _every_mode_and_root(dev, dims, R, w, bits, T64)
    say(f"  worst error / bound {worst:.3f}")


def test_fp8f8_combined_first_level(dev):
    """The combined first level: the Khatri-Rao product of the last two FP32
    factor copies (formed in FP32) quantized per column, every mode."""
    import oracle
    from paper_2010_12056_amd import cpals

    dims, R = (50, 60, 33, 9), 50
    say(f"case fp8f8 combined {dims} R={R}")
    w, bits, T64 = _case(dims, R, 1777)
    plan = cpals.Plan(dims, R, prec="fp8f8", tree="dt_combined", device=dev)
    plan.set_tensor(_dev_fp8(bits, dev))
    A = to_dev(w.init, dev)
    f = [np.asarray(a, dtype=np.float32) for a in w.init]
    krp32 = (f[2][:, None, :] * f[3][None, :, :]).reshape(dims[2] * dims[3], R).astype(np.float64)
    kq = oracle.quantize_columns(krp32)[0]
    # leading half: node (modes 0, 1) = T (s0 s1) x (s2 s3) times the quantized product
    X = T64.reshape(dims[0] * dims[1], -1)
    node = (X @ kq).reshape(dims[0], dims[1], R)
    nodeabs = (np.abs(X) @ np.abs(kq)).reshape(dims[0], dims[1], R)
    nodewin = _group_bound(np.abs(X), np.abs(kq), 1).reshape(dims[0], dims[1], R)
    for n, other in ((0, 1), (1, 0)):
        spec = "ijr,jr->ir" if n == 0 else "ijr,ir->jr"
        a = _f32(w.init[other])
        ref = np.einsum(spec, node, a)
        bound = WINDOW * np.einsum(spec, nodewin, np.abs(a)) + FP32_ALLOWANCE * np.einsum(spec, nodeabs, np.abs(a))
        M = plan.mttkrp(A, n).cpu().numpy()
        q = float((np.abs(M - ref) / np.maximum(bound, 1e-300)).max())
        say(f"  mode {n}: error / bound {q:.3f}")
        assert q <= 1.0, (n, q)
    plan.close()


@pytest.mark.parametrize("tree", ["dt", "msdt"])
def test_fp8f8_als_sweeps(dev, tree):
    """Free-running sweeps.  After each, with the GPU's own factors A:
    * DT: the last mode's MTTKRP comes from the trailing half, whose root is
      mode 0 after its update, so the oracle forms M^(N-1) with the quantized
      FP32 copy of the final A^(0) and evaluates Eq. (3); the GPU's residual
      agrees within the MTTKRP bound above, carried by |A^(N-1)|:
      |r_gpu^2 - r_q^2| <= 2 <bound, |A^(N-1)|> / ||T||^2 (+1e-12).
    * both trees: the error against the exact residual (Eq. (2)) of the same
      factors is stated; it comes from M^(N-1) being formed with a quantized
      factor (which one depends on the MSDT subtree), each entry of which is
      within 2^-4 of its value plus 2^-10 of the column's step below 2^-6
      (at most 2^-18 of the column's largest magnitude), so
      |r_gpu^2 - r_exact^2| <= 2 <(2^-4 + 2^-9 + f)|T||P| + 2^-18 cmax |T||P'|, |A^(N-1)|> / ||T||^2,
      the larger over the possible roots (P' with the root's factor replaced
      by its column maxima)."""
    import oracle
    from oracle import core
    from paper_2010_12056_amd import cpals

    say(f"case fp8f8 sweeps {tree}")
    dims, R = (40, 37, 33, 29), 20
    N = len(dims)
    w, bits, T64 = _case(dims, R, 15)
    absT = np.abs(T64)
    normT2 = float(np.sum(T64 * T64))
    plan = cpals.Plan(dims, R, prec="fp8f8", tree=tree, device=dev)
    plan.set_tensor(_dev_fp8(bits, dev))
    A = to_dev(w.init, dev)
    for sweep in range(6):
        info = plan.als_sweep(A)
        Ah = [a.cpu().numpy() for a in A]
        S = [core.gram(a) for a in Ah]
        G = core.gamma(S, N - 1)
        r_gpu = info["r"]
        r_exact = core.residual_explicit(T64, Ah)
        absAl = np.abs(Ah[N - 1])
        msg = f"  sweep {sweep}: r {r_gpu:.6f}, exact {r_exact:.6f}, |dr| {abs(r_gpu - r_exact):.2e}"
        if tree == "dt":
            used = _used_factors(Ah, 0)
            Mq = oracle.mttkrp_naive(T64, used, N - 1)
            r_q = core.residual_fast(normT2, G, S[N - 1], Mq, Ah[N - 1])
            lim = 2.0 * float(np.sum(_bound(absT, used, N - 1, 0) * absAl)) / normT2 + 1e-12
            d2 = abs(r_gpu ** 2 - r_q ** 2)
            msg += f"; vs oracle with the same quantized factor |dr^2| {d2:.2e} (bound {lim:.2e})"
            assert d2 <= lim, (sweep, d2, lim)
        lim_q = 0.0
        f32A = [np.abs(_f32(a)) for a in Ah]
        for root in range(N - 1):
            P = f32A.copy()
            rel = oracle.mttkrp_naive(absT, P, N - 1)
            P[root] = np.broadcast_to(P[root].max(axis=0), P[root].shape)
            flo = oracle.mttkrp_naive(absT, P, N - 1)
            e = (2.0 ** -4 + WINDOW + FP32_ALLOWANCE) * rel + 2.0 ** -18 * flo
            lim_q = max(lim_q, 2.0 * float(np.sum(e * absAl)) / normT2 + 1e-12)
        d2e = abs(r_gpu ** 2 - r_exact ** 2)
        say(msg + f"; vs exact |dr^2| {d2e:.2e} (bound {lim_q:.2e})")
        assert d2e <= lim_q, (sweep, d2e, lim_q)
    plan.close()
