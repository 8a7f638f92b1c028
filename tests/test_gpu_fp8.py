"""GPU parity of the FP8 tensor path (E4M3 tensor widened exactly to BF16 in
registers, first contraction on the BF16 matrix cores with FP32
accumulation, FP32 levels below) against the FP64 oracle run on the same
FP8 tensor values.

Every E4M3 value is a BF16 value, so the tensor enters the products exactly
and the bound is that of the BF16 path: only the factor of the first
contraction is rounded (u = 2^-8 for one BF16 part, 2^-16 for the split),
    |M_gpu - M| <= (u + f) * (|T_(n)| |P^(n)|)      elementwise,
with f = 1e-5 an allowance for the FP32 accumulation and FP32 levels."""

import numpy as np
import pytest

from gpu_util import relerr, say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FP32_ALLOWANCE = 1e-5
UNIT = {"fp8": 2.0 ** -8, "fp8x2": 2.0 ** -16}


def _ratio(M, ref, refabs, prec):
    """max over entries of |M - ref| / ((u + f) |T||P|); must be <= 1."""
    return float((np.abs(M - ref) / ((UNIT[prec] + FP32_ALLOWANCE) * np.maximum(refabs, 1e-300))).max())


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _fp8_case(dims, R, seed, kind="uniform", noise_rel=1e-2):
    from paper_2010_12056_amd import synth

    w = synth.planted_tensor(dims, R, seed, kind=kind, noise_rel=noise_rel, dtype=np.float32)
    # stored as E4M3 times the power of two that puts the largest entry near 448 (the
    # precision workload's entries are ~1e-5 and would otherwise mostly round to zero)
    bits = synth.fp8_bits(w.T, scale=synth.fp8_scale(w.T))
    T64 = synth.fp8_to_f32(bits).astype(np.float64)
    assert np.count_nonzero(T64) > 0.9 * T64.size
    return w, bits, T64


def _dev_fp8(bits, dev):
    return torch.from_numpy(np.ascontiguousarray(bits)).to(dev).view(torch.float8_e4m3fn)


def _every_mode_and_root(dev, dims, R, prec, w, bits, T64, tree="dt"):
    import oracle
    from paper_2010_12056_amd import cpals

    plan = cpals.Plan(dims, R, prec=prec, tree=tree, device=dev)
    plan.set_tensor(_dev_fp8(bits, dev))
    A = to_dev(w.init, dev)
    N = len(dims)
    absT = np.abs(T64)
    absA = [np.abs(a) for a in w.init]
    worst = 0.0
    for n in range(N):
        ref = oracle.mttkrp_naive(T64, w.init, n)
        refabs = oracle.mttkrp_naive(absT, absA, n)
        roots = [None] if tree != "dt" else [None] + [m for m in range(N) if m != n]
        for root in roots:
            M = plan.mttkrp(A, n, root=root).cpu().numpy()
            q = _ratio(M, ref, refabs, prec)
            worst = max(worst, q)
            assert q <= 1.0, (n, root, q)
    plan.close()
    return worst


CASES = [
    # (dims, R).  Last-mode contraction (K = last size): unguarded 16-byte rows when K % 16 == 0
    # (K = 512 over eight chunks, K = 48 with a clamped tail, K = 16 below one chunk, K = 32 with
    # more than 256 row tiles), 4-byte loads when K % 4 == 0 (K = 12, 8, 40), byte loads
    # otherwise (K = 29).  Other modes: unguarded groups of four q when Q % 4 == 0 (Q from 8 to
    # 8704, Q below one wave's 64 rows, more than 256 tiles at (300, 12, 8)), guarded otherwise
    # (odd Q); ragged K against the 64-index chunk (17, 37, 520); R = 1 ... 128.
    ((40, 37, 33, 29), 20),
    ((24, 17, 512), 128),
    ((8, 520, 12), 33),
    ((300, 12, 8), 64),
    ((3, 1, 5, 2, 4), 1),
    ((48, 72, 40), 24),
    ((36, 20, 48), 50),
    ((64, 9, 6, 16), 17),
    ((400, 340, 32), 16),
    # three register sets (unguarded contiguous rows, two or more chunks): K = 80 is exactly two
    # chunks, so every step's look-ahead crosses into the next tile; 293 row tiles at K = 96
    ((40, 30, 80), 24),
    ((600, 250, 96), 20),
]


@pytest.mark.parametrize("prec", ["fp8", "fp8x2"])
@pytest.mark.parametrize("dims,R", CASES)
def test_fp8_mttkrp_every_mode_and_root(dev, dims, R, prec):
    say(f"case fp8 mttkrp dims={dims} R={R} prec={prec}")
    w, bits, T64 = _fp8_case(dims, R, 900 + len(dims) + R)
    worst = _every_mode_and_root(dev, dims, R, prec, w, bits, T64)
    say(f"  worst error / bound {worst:.3f}")


@pytest.mark.parametrize("prec", ["fp8", "fp8x2"])
def test_fp8_every_finite_code(dev, prec):
    """Tensor entries drawn uniformly from all 254 finite codes (both signs,
    both zeros, the subnormals down to 2^-9, up to 448): the widening must be
    exact across the whole format, in both layouts."""
    from paper_2010_12056_amd import synth

    dims, R = (40, 36, 48), 24
    say(f"case fp8 all codes {dims} R={R} {prec}")
    rng = np.random.default_rng(71)
    finite = np.array([c for c in range(256) if c not in (0x7F, 0xFF)], dtype=np.uint8)
    bits = rng.choice(finite, size=dims)
    T64 = synth.fp8_to_f32(bits).astype(np.float64)
    w = synth.planted_tensor(dims, R, 72, noise_rel=0.0, dtype=np.float32)
    worst = _every_mode_and_root(dev, dims, R, prec, w, bits, T64)
    say(f"  worst error / bound {worst:.3f}")


def test_fp8_norm_and_fitness_match_oracle(dev):
    """The tensor norm (read from FP8 by its own kernel) enters the residual:
    one sweep's residual against the oracle's on the same FP8 values."""
    import oracle
    from paper_2010_12056_amd import cpals

    dims, R = (44, 38, 36), 12
    say(f"case fp8 norm {dims}")
    w, bits, T64 = _fp8_case(dims, R, 81)
    plan = cpals.Plan(dims, R, prec="fp8x2", tree="dt", device=dev)
    plan.set_tensor(_dev_fp8(bits, dev))
    A = to_dev(w.init, dev)
    st = oracle.AlsState.start(T64, w.init)
    info = plan.als_sweep(A)
    r_ref = oracle.als_sweep(st)
    say(f"  r {info['r']:.9f} vs {r_ref:.9f}")
    assert abs(info["r"] - r_ref) <= 1e-5
    plan.close()


@pytest.mark.parametrize("tree", ["dt", "msdt"])
def test_fp8x2_als_sweeps_resynced(dev, tree):
    """Each sweep from the same factors on both sides: fitness and factors of
    one FP8X2 sweep against the FP64 oracle on the FP8 tensor."""
    import oracle
    from paper_2010_12056_amd import cpals

    say(f"case fp8x2 sweeps {tree}")
    dims, R = (40, 37, 33, 29), 20
    w, bits, T64 = _fp8_case(dims, R, 5)
    plan = cpals.Plan(dims, R, prec="fp8x2", tree=tree, device=dev)
    plan.set_tensor(_dev_fp8(bits, dev))
    A = to_dev(w.init, dev)
    for sweep in range(6):
        st = oracle.AlsState.start(T64, [a.cpu().numpy() for a in A])
        info = plan.als_sweep(A)
        r_ref = oracle.als_sweep(st)
        fe = abs(info["r"] - r_ref)
        ae = max(relerr(A[n].cpu().numpy(), st.A[n]) for n in range(4))
        say(f"  sweep {sweep}: |dr| {fe:.2e}, factor relerr {ae:.2e}")
        assert fe <= 1e-5, (sweep, fe)
        assert ae <= 2e-3, (sweep, ae)
    plan.close()


@pytest.mark.parametrize("prec", ["fp8", "fp8x2"])
def test_fp8_combined_first_level(dev, prec):
    """The combined first level (contraction with the Khatri-Rao product of
    the last two factors) on an FP8 tensor, every mode."""
    dims, R = (50, 60, 33, 9), 50
    say(f"case fp8 combined {dims} R={R} {prec}")
    w, bits, T64 = _fp8_case(dims, R, 777)
    worst = _every_mode_and_root(dev, dims, R, prec, w, bits, T64, tree="dt_combined")
    say(f"  worst error / bound {worst:.3f}")


@pytest.mark.parametrize("prec", ["fp8", "fp8x2"])
def test_fp8_config_distribution_sampled(dev, prec):
    """The precision workload's distribution (N(0,1) factor columns with norms
    spread log-uniformly over [1e-2, 1], noise 1e-3 of the norm, R = 128) at
    384 x 320 x 288: many tiles and chunks in every mode; rows sampled and
    computed one by one by the oracle's definition."""
    from oracle import core
    from paper_2010_12056_amd import cpals

    dims, R = (384, 320, 288), 128
    say(f"case fp8 sampled {dims} R={R} {prec}")
    w, bits, T64 = _fp8_case(dims, R, 3003, kind="lognorm", noise_rel=1e-3)
    plan = cpals.Plan(dims, R, prec=prec, tree="dt", device=dev)
    plan.set_tensor(_dev_fp8(bits, dev))
    A = to_dev(w.init, dev)
    rng = np.random.default_rng(1)
    for n in range(3):
        rows = rng.choice(dims[n], size=5, replace=False)
        others = [m for m in range(3) if m != n]
        K = core.krp([w.init[m] for m in others])
        Kabs = core.krp([np.abs(w.init[m]) for m in others])
        X = np.moveaxis(T64, n, 0)
        ref = np.stack([X[i].reshape(-1) @ K for i in rows])
        refabs = np.stack([np.abs(X[i]).reshape(-1) @ Kabs for i in rows])
        for root in [None] + others:
            M = plan.mttkrp(A, n, root=root).cpu().numpy()[rows]
            q = _ratio(M, ref, refabs, prec)
            say(f"  mode {n} root {root}: error / bound {q:.3f}, norm-wise {relerr(M, ref):.2e}")
            assert q <= 1.0
    plan.close()
