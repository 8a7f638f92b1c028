"""What the trained switch gains over the method without it (Alg. 2 with
its hand tolerance) on a held-out workload of the family it was trained on:
order-6 24^6 FP32, planted rank-32 factors with collinearity 0.9, noise 1e-2,
R = 32, MSDT plan, at most 200 outer steps.  Target: the regular-only run's
final exact fitness minus 1e-4, checked with the FP64 audit.  The full
ten-seed evaluation (profiles/pp_switch_o6_s24_r32_eval.md) is a separate
run; this test replays one held-out seed with the committed model."""

import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_learned_switch_reaches_target_where_hand_threshold_fails(dev):
    from paper_2010_12056_amd import learned_switch as ls

    seed = 4209
    say(f"case learned switch gain, held-out seed {seed}")
    model = ls.load_model()
    b = ls.Bench(ls.make_workload(seed))
    try:
        res = ls.evaluate_workload(b, model, sweeps=200)
    finally:
        b.close()
    for k in ("regular", "eps0.1", "eps0.2", "learned"):
        v = res[k]
        say(f"  {k}: {v['steps']} steps, {v['time_s'] * 1e3:.1f} ms, reached {v['reached']}, "
            f"regular/init/approx {v['n_exact']}/{v['n_init']}/{v['n_approx']} {v['failed']}")
    assert res["regular"]["reached"]
    assert res["learned"]["reached"]
    assert res["learned"]["n_approx"] > 0  # it did use PP steps
    assert not res["eps0.1"]["reached"] and not res["eps0.2"]["reached"]
