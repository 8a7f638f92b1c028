"""Host-side logic that needs no GPU: the learned switch's feature formula,
the autotuner's cache keys, the BF16 storage rounding and the batch
workload generator."""

import json
import math

import numpy as np

from paper_2010_12056_amd import autotune, learned_switch, synth


def test_switch_features_formula():
    # log10 of the relative changes (clamped at 1e-12), then the three newest fitness deltas;
    # a delta that does not exist yet counts as 1 (log10 = 0)
    x = learned_switch.features([0.1, 1e-15, 2.0], [0.9, 0.89])
    assert x[0] == math.log10(0.1) and x[1] == -12.0 and x[2] == math.log10(2.0)
    assert abs(x[3] - math.log10(0.01)) < 1e-12
    assert x[4] == 0.0 and x[5] == 0.0
    x = learned_switch.features([0.5] * 3, [0.5, 0.5, 0.4, 0.1])
    assert x[3] == -12.0  # equal fitness: the clamp
    assert abs(x[4] - math.log10(0.1)) < 1e-12 and abs(x[5] - math.log10(0.3)) < 1e-12


def test_autotune_signature_and_cache(tmp_path):
    dims = [(16, 20, 96), (50, 50, 50)]
    ranks = [8, 32]
    assert autotune.signature(dims, ranks) == "order3|n2|s16-96|R8,32"
    path = tmp_path / "cache.json"
    path.write_text(json.dumps({"devA|order3|n2|s16-96|R8,32": {"waves": 8, "groups_per_cu": 1}}))
    cache = autotune.load_cache(str(path))
    assert cache["devA|order3|n2|s16-96|R8,32"]["waves"] == 8
    assert autotune.load_cache(str(tmp_path / "missing.json")) == {}


def test_bf16_rounding_is_nearest_even():
    one = np.float32(1.0)
    half_ulp = np.float32(2.0 ** -8)  # bf16 has 8 significant bits: spacing 2^-7 above 1
    vals = np.array([one + half_ulp, one + 3 * half_ulp, -(one + half_ulp), 3.0, 0.0], dtype=np.float32)
    back = synth.bf16_to_f32(synth.bf16_bits(vals))
    assert back[0] == 1.0  # tie -> even
    assert back[1] == np.float32(1.0 + 2.0 ** -6)  # tie -> even (upwards)
    assert back[2] == -1.0
    assert back[3] == 3.0 and back[4] == 0.0
    x = np.random.default_rng(0).standard_normal(1000).astype(np.float32)
    assert np.all(np.abs(synth.bf16_to_f32(synth.bf16_bits(x)) - x) <= 2.0 ** -8 * np.abs(x))


def test_batch_workload_distribution():
    ws = synth.batch_workload(40, seed=9)
    assert len(ws) == 40
    for w in ws:
        assert all(16 <= s <= 96 for s in w.dims) and w.R in (4, 8, 16, 32)
        assert w.T.dtype == np.float32 and w.T.shape == w.dims
    again = synth.batch_workload(40, seed=9)
    assert all(np.array_equal(a.T, b.T) for a, b in zip(ws, again))
