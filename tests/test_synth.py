"""Checks of the seeded input generators (CPU only)."""

import numpy as np

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
