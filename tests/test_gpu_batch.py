"""GPU parity of the batched path (many small order-3 tensors, one
persistent launch) against the FP64 oracle's ALS sweeps, tensor by tensor,
plus determinism, launch-shape independence and HIP-graph replay."""

import numpy as np
import pytest

from gpu_util import relerr, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _edge_workloads():
    """Shapes at the limits: unit and tiny modes, sizes not a multiple of 4
    or 16, the largest mode (96), R = 1, R = 17 (padded to 32), R = 32."""
    from paper_2010_12056_amd import synth

    shapes = [((1, 5, 7), 1), ((3, 2, 9), 2), ((17, 33, 5), 17), ((96, 96, 96), 32), ((96, 16, 40), 4),
              ((20, 21, 22), 8), ((50, 3, 61), 16), ((16, 96, 17), 32)]
    return [synth.planted_tensor(d, R, 7000 + i, kind="uniform", noise_rel=1e-3, dtype=np.float32)
            for i, (d, R) in enumerate(shapes)]


def _run(dev, ws, sweeps, waves=4, groups=2, A_init=None):
    from paper_2010_12056_amd import cpals

    b = cpals.Batch([w.dims for w in ws], [w.R for w in ws], device=dev, waves=waves, groups_per_cu=groups)
    T = b.pack_tensors([w.T for w in ws])
    A = b.pack_factors([w.init for w in ws]) if A_init is None else A_init.clone()
    fit, status = b.sweeps(T, A, sweeps)
    torch.cuda.synchronize()
    return b, T, A, fit.cpu().numpy(), status.cpu().numpy()


def _fit_tol(r):
    # The contractions with the tensor carry a relative error e of about one
    # FP32 rounding per product (three-part BF16 products, FP32 sums), so
    # <M, A> in Eq. (3) is off by a few 1e-8 of ||T||^2; Eq. (3) subtracts
    # terms of size ||T||^2, so r moves by about e / r.  Measured on these
    # cases: |df| r <= 6.7e-8.
    return 1e-7 + 1e-7 / max(r, 1e-12)


def _oracle_check(ws, b, A, fit, sweeps, fac_tol):
    import oracle

    worst, worst_r, worst_fac = 0.0, 0.0, 0.0
    for i, w in enumerate(ws):
        st = oracle.AlsState.start(w.T.astype(np.float64), w.init)
        for s in range(sweeps):
            r = oracle.als_sweep(st)
            d = abs(fit[i, s] - (1.0 - r))
            assert d <= _fit_tol(r), (i, w.dims, w.R, s, fit[i, s], 1.0 - r)
            worst = max(worst, d / _fit_tol(r))
            worst_r = max(worst_r, d * r)
        got = [a.cpu().numpy() for a in b.unpack_factors(A, i)]
        for m in range(3):
            e = relerr(got[m], st.A[m])
            assert e <= fac_tol, (i, w.dims, w.R, m)
            worst_fac = max(worst_fac, e)
    say(f"  fitness error / tolerance <= {worst:.3g}, |df| r <= {worst_r:.3g}, factor relerr <= {worst_fac:.3g}")


def test_batch_edge_shapes_match_oracle(dev):
    say("case batch edge shapes")
    ws = _edge_workloads()
    b, T, A, fit, status = _run(dev, ws, 5)
    assert np.all(status == 0)
    _oracle_check(ws, b, A, fit, 5, 2e-4)
    b.close()


def test_batch_mixed_workload_matches_oracle(dev):
    """64 tensors of the benchmark's distribution (modes in [16, 96], R in
    {4, 8, 16, 32}), 5 sweeps, every tensor checked."""
    from paper_2010_12056_amd import synth

    say("case batch mixed 64")
    ws = synth.batch_workload(64, seed=5101)
    b, T, A, fit, status = _run(dev, ws, 5)
    assert np.all(status == 0)
    _oracle_check(ws, b, A, fit, 5, 2e-4)
    b.close()


def test_batch_deterministic_and_independent_of_residency(dev):
    """Same launch twice: bitwise equal.  One or two resident workgroups per
    compute unit (a different assignment of tensors to workgroups): bitwise
    equal, since each tensor is computed by one workgroup in a fixed order."""
    from paper_2010_12056_amd import synth

    say("case batch determinism")
    ws = synth.batch_workload(40, seed=5202)
    b1, _, A1, f1, _ = _run(dev, ws, 4, groups=2)
    b2, _, A2, f2, _ = _run(dev, ws, 4, groups=2)
    b3, _, A3, f3, _ = _run(dev, ws, 4, groups=1)
    assert np.array_equal(f1, f2) and torch.equal(A1, A2)
    assert np.array_equal(f1, f3) and torch.equal(A1, A3)
    b4, _, A4, f4, _ = _run(dev, ws, 4, waves=8, groups=1)
    assert np.max(np.abs(f4 - f1)) <= 1e-10  # eight waves: another reduction tree
    for b in (b1, b2, b3, b4):
        b.close()


def test_batch_graph_replay(dev):
    """The sweeps call enqueues kernels only (no allocation, no memset): it is
    captured in a HIP graph and replayed; every replay, after the factors are
    reset eagerly, reproduces the eager result bit for bit."""
    from paper_2010_12056_amd import synth

    say("case batch graph replay")
    ws = synth.batch_workload(32, seed=5303)
    b, T, A_eager, f_eager, _ = _run(dev, ws, 3)
    A0 = b.pack_factors([w.init for w in ws])
    A = A0.clone()
    fit = torch.empty((len(ws), 3), dtype=torch.float64, device=dev)
    status = torch.empty(len(ws), dtype=torch.int32, device=dev)
    s = torch.cuda.Stream(dev)
    s.wait_stream(torch.cuda.current_stream(dev))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        from paper_2010_12056_amd import cpals

        bg = cpals.Batch([w.dims for w in ws], [w.R for w in ws], device=dev)
        with torch.cuda.graph(g, stream=s):
            bg.sweeps(T, A, 3, fitness=fit, status=status)
    torch.cuda.current_stream(dev).wait_stream(s)
    for rep in range(3):
        A.copy_(A0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(fit.cpu().numpy(), f_eager), rep
        assert torch.equal(A, A_eager), rep
        _ = torch.ones(8, device=dev).sum().item()  # eager work between replays
    b.close()
    bg.close()


def test_batch_singular_gamma_flags_only_its_tensor(dev):
    """A tensor whose two factor columns are equal in modes 1 and 2 makes
    Gamma0 = S1 * S2 singular at the first update: its status is 1 (its
    sweeps stop), and the other tensors in the same launch still match the
    oracle sweep by sweep."""
    from paper_2010_12056_amd import synth

    say("case batch singular gamma")
    ws = [synth.planted_tensor(d, R, 7200 + i, kind="uniform", noise_rel=1e-3, dtype=np.float32)
          for i, (d, R) in enumerate([((30, 20, 25), 2), ((40, 33, 21), 8), ((17, 64, 48), 16)])]
    bad = ws[0]
    for m in (1, 2):
        bad.init[m][:, 1] = bad.init[m][:, 0]
    b, T, A, fit, status = _run(dev, ws, 4)
    assert status[0] == 1
    assert np.all(status[1:] == 0)
    import oracle

    for i in (1, 2):
        st = oracle.AlsState.start(ws[i].T.astype(np.float64), ws[i].init)
        for s in range(4):
            r = oracle.als_sweep(st)
            assert abs(fit[i, s] - (1.0 - r)) <= _fit_tol(r), (i, s)
    b.close()


QUEUE_SKIP = ("the work-queue form of the batched kernel (a tensor's contraction stages split into items over "
              "several workgroups, with dependency waits between workgroups) hung on the GPU twice, its cause "
              "not found; that kernel is not in the library and these tests of it stay skipped")


@pytest.mark.skip(reason=QUEUE_SKIP)
@pytest.mark.parametrize("parts", [1, 16])
def test_batch_queue_split_edge_shapes_match_oracle(dev, parts):
    """Work-queue kernel: the edge shapes with every bucket's contraction
    stages in `parts` items, against the oracle."""
    from paper_2010_12056_amd import cpals

    ws = _edge_workloads()
    b = cpals.Batch([w.dims for w in ws], [w.R for w in ws], device=dev, split={k: parts for k in range(12)})
    T = b.pack_tensors([w.T for w in ws])
    A = b.pack_factors([w.init for w in ws])
    fit, status = b.sweeps(T, A, 5)
    torch.cuda.synchronize()
    assert np.all(status.cpu().numpy() == 0)
    _oracle_check(ws, b, A, fit.cpu().numpy(), 5, 2e-4)
    b.close()


@pytest.mark.skip(reason=QUEUE_SKIP)
def test_batch_queue_split_changes_rounding_only(dev):
    """Work-queue kernel: large tensors with one item per stage and with
    sixteen agree to FP64 rounding of the partial sums after five sweeps."""
    from paper_2010_12056_amd import cpals, synth

    shapes = [((96, 96, 96), 32), ((90, 71, 83), 16), ((64, 96, 50), 8), ((77, 80, 96), 4)]
    ws = [synth.planted_tensor(d, R, 7100 + i, kind="uniform", noise_rel=1e-3, dtype=np.float32)
          for i, (d, R) in enumerate(shapes)]
    out = []
    for parts in (1, 16):
        b = cpals.Batch([w.dims for w in ws], [w.R for w in ws], device=dev, split={k: parts for k in range(12)})
        T = b.pack_tensors([w.T for w in ws])
        A = b.pack_factors([w.init for w in ws])
        fit, _ = b.sweeps(T, A, 5)
        torch.cuda.synchronize()
        out.append(fit.cpu().numpy())
        b.close()
    assert np.max(np.abs(out[0] - out[1])) <= 1e-10
