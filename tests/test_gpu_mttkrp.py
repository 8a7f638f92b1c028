"""GPU parity of the MTTKRP path (first-level TTM + batched TTVs) against the
FP64 oracle's explicit-KRP definition."""

import numpy as np
import pytest

from gpu_util import relerr, say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _case(dims, R, seed, dtype):
    from paper_2010_12056_amd import synth

    return synth.planted_tensor(dims, R, seed, noise_rel=1e-2, dtype=dtype)


CASES = [
    # (dims, R, prec) : several tiles with ragged tails, odd sizes, R beyond one column tile
    ((37, 45, 29), 12, "f64"),
    ((40, 37, 33, 29), 20, "f32"),
    ((40, 37, 33, 29), 20, "f64"),
    ((131, 7, 130), 70, "f32"),
    ((3, 1, 5, 2, 4), 1, "f32"),
    ((1, 9, 1), 3, "f64"),
    ((16, 17, 15, 3, 5, 4), 33, "f32"),
    ((64, 64, 64), 128, "f32"),
    # long contracted last modes: the factor in chunks (ragged last chunk; K not a
    # multiple of 4 takes the element-wise loads)
    ((20, 9, 700), 40, "f32"),
    ((20, 9, 701), 20, "f32"),
    ((17, 5, 1000), 16, "f32"),
    ((30, 11, 300), 70, "f64"),
    # long contracted modes that are not the last (FP32): chunked factor, one and two
    # 64-column passes, q rows not a multiple of 4
    ((700, 9, 8), 40, "f32"),
    ((300, 10, 8), 70, "f32"),
    ((520, 65, 3), 20, "f32"),
    ((260, 7, 10), 128, "f32"),  # 128 columns in one pass, a last factor chunk of one 32-index piece
    # FP32 last mode of exactly 128 (the 32x32x2 kernel): one and two 32-column blocks, ragged
    # 32-row tiles, R not a multiple of 32
    ((37, 5, 128), 24, "f32"),
    ((21, 9, 128), 64, "f32"),
    ((7, 3, 2, 128), 50, "f32"),
    # a short run of q after the contracted mode (1 < Q < 64: rows (p, q) tiled as one index),
    # ragged row tiles, one to four column blocks
    ((30, 41, 33, 9), 50, "f32"),
    ((30, 41, 33, 9), 50, "f64"),
    ((50, 100, 3, 2), 17, "f32"),
]


@pytest.mark.parametrize("dims,R,prec", CASES)
def test_mttkrp_every_mode_and_root(dev, dims, R, prec):
    import oracle
    from paper_2010_12056_amd import cpals

    say(f"case mttkrp dims={dims} R={R} prec={prec}")
    dt = np.float64 if prec == "f64" else np.float32
    w = _case(dims, R, 100 + len(dims) + R, dt)
    plan = cpals.Plan(dims, R, prec=prec, tree="dt", device=dev)
    T = torch.from_numpy(w.T).to(dev)
    plan.set_tensor(T)
    A = to_dev(w.init, dev)
    T64 = w.T.astype(np.float64)
    tol = 1e-12 if prec == "f64" else 1e-5
    N = len(dims)
    for n in range(N):
        ref = oracle.mttkrp_naive(T64, w.init, n)
        M = plan.mttkrp(A, n).cpu().numpy()
        e = relerr(M, ref)
        assert e <= tol, (n, "dt", e)
        for root in range(N):
            if root == n:
                continue
            M = plan.mttkrp(A, n, root=root).cpu().numpy()
            e = relerr(M, ref)
            assert e <= tol, (n, root, e)
    plan.close()


def test_mttkrp_config_o4_s128_r64_sampled(dev):
    """Full-size order-4 128^4 FP32 tensor, R = 64, every mode, both
    first-level layouts; rows sampled and computed one by one by the oracle's
    definition."""
    import oracle
    from oracle import core
    from paper_2010_12056_amd import cpals, synth

    say("case mttkrp o4_s128_r64_f32 full size")
    w = synth.workload("o4_s128_r64_f32")
    plan = cpals.Plan(w.dims, w.R, prec="f32", tree="dt", device=dev)
    T = torch.from_numpy(w.T).to(dev)
    plan.set_tensor(T)
    A = to_dev(w.init, dev)
    rng = np.random.default_rng(0)
    for n in range(4):
        rows = rng.choice(w.dims[n], size=6, replace=False)
        K = core.krp([w.init[m] for m in range(4) if m != n])
        X = np.moveaxis(w.T, n, 0)
        ref = np.stack([X[i].astype(np.float64).reshape(-1) @ K for i in rows])
        for root in [None] + [m for m in range(4) if m != n]:
            M = plan.mttkrp(A, n, root=root).cpu().numpy()[rows]
            e = relerr(M, ref)
            say(f"  mode {n} root {root} relerr {e:.2e}")
            assert e <= 1e-5
        del K
    plan.close()
    del oracle


@pytest.mark.parametrize("dims,R", [((1024, 129, 133), 40), ((1024, 128, 260), 24)])
def test_mttkrp_long_last_mode_many_rows(dev, dims, R):
    """FP32 first-level contraction over a long last mode with many rows (the
    32x32x2 chunked kernel takes over from 131072 rows): a ragged last chunk
    with K % 4 != 0, and an aligned one; modes 0 and 1 rooted at the last."""
    import oracle
    from paper_2010_12056_amd import cpals

    say(f"case long last mode dims={dims} R={R}")
    w = _case(dims, R, 900 + R, np.float32)
    plan = cpals.Plan(dims, R, prec="f32", tree="dt", device=dev)
    T = torch.from_numpy(w.T).to(dev)
    plan.set_tensor(T)
    A = to_dev(w.init, dev)
    T64 = w.T.astype(np.float64)
    for n in (0, 1):
        ref = oracle.mttkrp_naive(T64, w.init, n)
        M = plan.mttkrp(A, n, root=2).cpu().numpy()
        e = relerr(M, ref)
        say(f"  mode {n}: relerr {e:.2e}")
        assert e <= 1e-5, (n, e)
    plan.close()
