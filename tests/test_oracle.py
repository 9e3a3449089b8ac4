"""The FP64 oracle against its pins (CPU only)."""
import numpy as np
import pytest

import oracle
import oracle_pins


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)


def test_levels_beyond_depth_are_noops(orc):
    """Once every length is 1, a further level carries everything unchanged."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal(37)
    assert np.array_equal(orc.fwd_1d(x, 6), orc.fwd_1d(x, 9))
    X = rng.standard_normal((5, 12))
    assert np.array_equal(orc.fwd_2d(X, 4), orc.fwd_2d(X, 7))


def test_band_slices_cover_layout():
    sl = oracle.band_slices_2d(13, 22, 3)
    cover = np.zeros((13, 22), int)
    for key, (r, c) in sl.items():
        cover[r, c] += 1
    assert np.all(cover == 1)
    sl1 = oracle.band_slices_1d(37, 5)
    cover1 = np.zeros(37, int)
    for s in sl1.values():
        cover1[s] += 1
    assert np.all(cover1 == 1)


def test_rejects_bad_levels(orc):
    with pytest.raises(ValueError):
        orc.fwd_1d(np.zeros(4), -1)
    with pytest.raises(ValueError):
        orc.fwd_2d(np.zeros((4, 4)), 63)
