"""Checks of the seeded input generators (CPU only)."""

import numpy as np
import pytest

from paper_2010_12056_amd import synth
from oracle import core


def test_deterministic_and_seed_sensitive():
    a = synth.planted_tensor((6, 5, 4), 3, 7, noise_rel=1e-2, dtype=np.float32)
    b = synth.planted_tensor((6, 5, 4), 3, 7, noise_rel=1e-2, dtype=np.float32)
    c = synth.planted_tensor((6, 5, 4), 3, 8, noise_rel=1e-2, dtype=np.float32)
    assert np.array_equal(a.T, b.T)
    assert all(np.array_equal(x, y) for x, y in zip(a.init, b.init))
    assert not np.array_equal(a.T, c.T)


def test_planted_structure_and_noise_level():
    w = synth.planted_tensor((30, 20, 25), 5, 3, noise_rel=1e-2, dtype=np.float64)
    T0 = core.reconstruct(w.planted)
    assert abs(np.linalg.norm(T0) - w.norm_T0) < 1e-9 * w.norm_T0
    E = w.T - T0
    rel = np.linalg.norm(E) / np.linalg.norm(T0)
    assert 0.0095 < rel < 0.0105
    assert all(0.0 <= a.min() and a.max() < 1.0 for a in w.init)


def test_block_size_does_not_change_values_without_noise():
    a = synth.planted_tensor((9, 8, 7), 2, 5, noise_rel=0.0, dtype=np.float64, block_elems=56)
    b = synth.planted_tensor((9, 8, 7), 2, 5, noise_rel=0.0, dtype=np.float64, block_elems=1 << 20)
    np.testing.assert_allclose(a.T, b.T, rtol=1e-15, atol=0)


def test_collinear_factors():
    w = synth.planted_tensor((400, 400, 3), 16, 11, kind="collinear", noise_rel=0.0, dtype=np.float64)
    A = w.planted[0]
    np.testing.assert_allclose(np.linalg.norm(A, axis=0), 1.0, rtol=1e-12)
    C = A.T @ A
    off = C[~np.eye(16, dtype=bool)]
    assert 0.8 < off.mean() < 0.97


def test_lognorm_column_norms():
    w = synth.planted_tensor((50, 40, 30), 8, 12, kind="lognorm", noise_rel=0.0, dtype=np.float64)
    for A in w.planted:
        nrm = np.linalg.norm(A, axis=0)
        assert np.all(nrm >= 1e-2 - 1e-12) and np.all(nrm <= 1.0 + 1e-12)


def test_fp8_decode_matches_the_format_and_torch():
    """E4M3 decoding pinned to fixed points of the format (1.0 = 0x38, the
    largest finite value 448 = 0x7e, the smallest subnormal 2^-9 = 0x01, the
    largest subnormal 7 2^-9 = 0x07, NaN at 0x7f / 0xff, -0 = 0x80) and to
    torch's float8_e4m3fn on all 256 codes."""
    torch = pytest.importorskip("torch")
    codes = np.arange(256, dtype=np.uint8)
    v = synth.fp8_to_f32(codes)
    assert v[0x38] == 1.0 and v[0x7E] == 448.0 and v[0xFE] == -448.0
    assert v[0x01] == 2.0 ** -9 and v[0x07] == 7 * 2.0 ** -9 and v[0x08] == 2.0 ** -6
    assert np.isnan(v[0x7F]) and np.isnan(v[0xFF]) and np.isnan(v).sum() == 2
    assert v[0x80] == 0.0 and np.signbit(v[0x80])
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).float().numpy()
    fin = ~np.isnan(v)
    assert np.array_equal(v[fin], ref[fin]) and np.array_equal(np.isnan(ref), ~fin)
    # strictly increasing over the non-negative finite codes: 127 distinct values
    assert np.all(np.diff(v[:0x7F].astype(np.float64)) > 0)


def test_fp8_encode_rounds_to_nearest_even():
    torch = pytest.importorskip("torch")
    codes = np.arange(256, dtype=np.uint8)
    fin = codes[~np.isnan(synth.fp8_to_f32(codes))]
    vals = synth.fp8_to_f32(fin).astype(np.float64)
    assert np.array_equal(synth.fp8_bits(vals), fin)  # every code round-trips (-0 included)
    pos = np.sort(synth.fp8_to_f32(np.arange(0, 0x7F, dtype=np.uint8)).astype(np.float64))
    mids = (pos[:-1] + pos[1:]) / 2  # exact ties: the even code wins
    got = synth.fp8_bits(mids)
    lo = synth.fp8_bits(pos[:-1])
    assert np.array_equal(got, np.where(lo % 2 == 0, lo, lo + 1))
    rng = np.random.default_rng(4)
    x = rng.standard_normal(50000) * np.exp(rng.uniform(-14, 5, 50000))
    x = x[np.abs(x) <= 440].astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(synth.fp8_bits(x), ref)
    with pytest.raises(ValueError):
        synth.fp8_bits(np.array([465.0]))  # rounds past 448
    with pytest.raises(ValueError):
        synth.fp8_bits(np.array([np.inf]))


def test_fp8_scale_uses_the_top_of_the_range():
    rng = np.random.default_rng(9)
    for mag in (1e-6, 3e-3, 0.7, 1.0, 448.0, 5e4):
        x = (rng.standard_normal(1000) * mag).astype(np.float32)
        s = synth.fp8_scale(x)
        m = float(np.max(np.abs(x)))
        assert np.log2(s) == np.round(np.log2(s))  # a power of two: exact scaling
        assert m * s <= synth.FP8_MAX < 2 * m * s
        bits = synth.fp8_bits(x, scale=s)
        y = synth.fp8_to_f32(bits).astype(np.float64) / s
        # relative error of E4M3 rounding (3 mantissa bits) above the subnormal range
        big = np.abs(x) * s >= 2.0 ** -6
        assert np.all(np.abs(y[big] - x[big]) <= 2.0 ** -4 * np.abs(x[big]))
    assert synth.fp8_scale(np.zeros(4, dtype=np.float32)) == 1.0
