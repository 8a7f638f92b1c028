"""Pins of the oracle's E4M3 factor quantization (CPU only): the format's
fixed facts, midpoint rounding worked out by hand, and torch's own
float8_e4m3fn conversion as an independent library routine."""

import numpy as np
import pytest

from oracle import quant


def test_e4m3_values_fixed_by_the_format():
    v = quant.e4m3_values()
    assert v.shape == (127,)
    assert v[0] == 0.0 and v[1] == 2.0 ** -9 and v[7] == 7 * 2.0 ** -9
    assert v[8] == 2.0 ** -6  # smallest normal, continuing the subnormal steps
    assert v[0x38] == 1.0 and v[0x3C] == 1.5 and v[-1] == 448.0
    assert np.all(np.diff(v) > 0)
    # spacing: 2^-9 below 2^-5 (subnormals and binade e = 1), then 2^(e-10) in
    # binade [2^(e-7), 2^(e-6)); the step up from code - 1 is that of its binade
    for code in range(1, 127):
        e = (code - 1) >> 3
        step = 2.0 ** -9 if e <= 1 else 2.0 ** (e - 10)
        assert v[code] - v[code - 1] == step, code


def test_every_finite_value_is_fixed():
    v = quant.e4m3_values()
    both = np.concatenate([v, -v])
    assert np.array_equal(quant.e4m3_round(both), both)


def test_midpoints_go_to_the_even_code():
    v = quant.e4m3_values()
    mids = (v[:-1] + v[1:]) / 2
    got = quant.e4m3_round(mids)
    even = np.where(np.arange(126) % 2 == 0, v[:-1], v[1:])
    assert np.array_equal(got, even)
    # worked by hand: 1.0625 lies between 1.0 (code 0x38) and 1.125 (0x39) -> 1.0;
    # 1.1875 between 1.125 (0x39) and 1.25 (0x3A) -> 1.25; 2^-10 between 0 and 2^-9 -> 0
    assert quant.e4m3_round(np.array([1.0625, 1.1875, 2.0 ** -10, -1.1875])).tolist() == [1.0, 1.25, 0.0, -1.25]


def test_nearest_rounding_against_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(11)
    x = np.concatenate([
        rng.uniform(-448, 448, 20000),
        rng.uniform(-1, 1, 20000) * 2.0 ** rng.integers(-12, 9, 20000),
        (quant.e4m3_values()[:-1] + quant.e4m3_values()[1:]) / 2,
    ]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(quant.e4m3_round(x.astype(np.float64)), want)


def test_quantize_columns_scale_and_error():
    rng = np.random.default_rng(12)
    A = rng.standard_normal((300, 9)) * np.array([1e-30, 1e-3, 0.5, 1.0, 3.0, 1e3, 7e20, 1.0, 1.0])
    A[:, 7] = 0.0
    A[5, 8] = 448.0 * 2.0 ** -3  # the maximum exactly at a power-of-two multiple of 448
    Aq, e = quant.quantize_columns(A)
    for c in range(A.shape[1]):
        col = A[:, c]
        mx = np.max(np.abs(col))
        if mx == 0.0:
            assert e[c] == 0 and np.all(Aq[:, c] == 0.0)
            continue
        s = 2.0 ** e[c]
        assert 224.0 < mx * s <= 448.0, c
        # each entry within half an E4M3 step of its scaled value
        y = col * s
        a = np.abs(y)
        half = np.where(a < 2.0 ** -6, 2.0 ** -10, 2.0 ** (np.floor(np.log2(np.maximum(a, 2.0 ** -6))) - 4))
        assert np.all(np.abs(Aq[:, c] * s - y) <= half), c
    assert e[8] == 3


def test_quantize_columns_rejects_nothing_in_range_and_keeps_signs():
    A = np.array([[-448.0, 1.0], [1e-9, -2.0], [0.0, 0.0]])
    Aq, e = quant.quantize_columns(A)
    assert e.tolist() == [0, 7]
    assert Aq[0, 0] == -448.0 and Aq[1, 0] == 0.0
    assert Aq[0, 1] == 1.0 and Aq[1, 1] == -2.0
