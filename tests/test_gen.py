"""Seeded synthetic inputs: determinism, normalisation and parameter ranges."""
import numpy as np

from dosegen import make_config_pair, make_pair_2d, make_pair_3d


def test_seed_determinism():
    a = make_pair_2d(3)
    b = make_pair_2d(3)
    assert np.array_equal(a.ref, b.ref) and np.array_equal(a.eval, b.eval)
    c = make_pair_2d(4)
    assert not np.array_equal(a.ref, c.ref)


def test_2d_ranges():
    p = make_config_pair("2d_64x64_1mm", 0)
    assert p.ref.shape == (64, 64) and p.ref.dtype == np.float32
    assert p.ref.max() == np.float32(1.0)
    assert all(-1.5 <= s <= 1.5 for s in p.meta["shift_mm"])
    assert 0.97 <= p.meta["scale"] <= 1.03
    frac = (p.ref >= 0.1).mean()
    assert 0.05 < frac < 0.9


def test_3d_small_ranges():
    p = make_pair_3d(100, shape=(24, 32, 32), spacing=(10.0, 10.0, 10.0))
    assert p.ref.shape == (24, 32, 32)
    assert p.ref.max() == np.float32(1.0)
    assert p.meta["spot_sign"] in (-1.0, 1.0)
    iz, iy, ix = p.meta["spot_index"]
    assert p.ref[iz, iy, ix] > 0.5
    d = p.eval.astype(np.float64) - p.ref
    assert np.abs(d).max() < 0.5
