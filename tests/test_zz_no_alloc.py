"""The allocation-free MTTKRP (cp_mttkrp_static: intermediates in the
library's static device scratch, no plan and no workspace) against the
planned MTTKRP (cp_mttkrp, caller workspace) on the same inputs.  Both run
the same kernels along the same tree path, so the results must agree bit
for bit.  Two calls in a row, the second on a smaller tensor, check that
nothing left in the shared scratch by the first call leaks into the second;
the oracle pins both to the Khatri-Rao definition."""

import ctypes

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


# (dims, R, prec): the second case of each pair is the smaller one
CASES = [
    (((29, 23, 17, 19), 12, "f32"), ((11, 9, 13, 7), 5, "f32")),
    (((24, 20, 18), 16, "f64"), ((7, 5, 6), 3, "f64")),
    (((9, 8, 7, 6, 5), 6, "f64"), ((5, 4, 3, 4, 3), 2, "f64")),
]


@pytest.mark.parametrize("pair", CASES, ids=["o4_f32", "o3_f64", "o5_f64"])
def test_static_mttkrp_matches_planned(dev, pair):
    import oracle
    from paper_2010_12056_amd import cpals, synth

    for dims, R, prec in pair:
        say(f"case static mttkrp dims={dims} R={R} {prec}")
        dt = np.float32 if prec == "f32" else np.float64
        w = synth.planted_tensor(dims, R, 9100 + len(dims) + R, noise_rel=1e-2, dtype=dt)
        T = torch.from_numpy(w.T).to(dev)
        A = to_dev(w.init, dev)
        plan = cpals.Plan(w.dims, R, prec=prec, tree="dt", device=dev)
        plan.set_tensor(T)
        T64 = w.T.astype(np.float64)
        for n in range(len(dims)):
            ref = plan.mttkrp(A, n).cpu().numpy()
            got = cpals.mttkrp_static(T, [None if m == n else A[m] for m in range(len(dims))], n, R,
                                      prec=prec).cpu().numpy()
            assert np.array_equal(got, ref), (dims, n, float(np.max(np.abs(got - ref))))
            tol = 1e-5 if prec == "f32" else 1e-12
            assert relerr(got, oracle.mttkrp_naive(T64, w.init, n)) <= tol
        plan.close()
        torch.cuda.synchronize()


def test_static_mttkrp_rejects_oversize(dev):
    """A tensor whose intermediates exceed the static scratch is refused
    before anything is enqueued, with a message naming the limit."""
    from paper_2010_12056_amd import cpals

    T = torch.zeros(1, dtype=torch.float32, device=dev)
    A = [torch.zeros(1, dtype=torch.float64, device=dev) for _ in range(4)]
    L = cpals.lib()
    dims = (ctypes.c_int64 * 4)(128, 128, 128, 128)
    M = torch.zeros(1, dtype=torch.float64, device=dev)
    s = L.cp_mttkrp_static(4, dims, 64, cpals.CP_F32, ctypes.c_void_p(T.data_ptr()), cpals._ptrs(A), 0,
                           ctypes.c_void_p(M.data_ptr()), None)
    assert s == cpals.CP_ERR_UNSUPPORTED
    assert b"static scratch" in L.cp_last_error(None)
