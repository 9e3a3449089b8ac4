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


def test_band_slices_3d_cover_and_locate_bands():
    """Every element of the 3D packed layout lies in exactly one band, and
    each band's slice starts where the 3D transform puts that band: the
    volume b_z (x) b_y (x) b_x built from 1D basis functions (the 1D
    synthesis, j levels, of a unit at a_j[0] for an L axis or d_j[0] for an H
    axis) transforms to a single 1 at the slice's first element."""
    d, h, w, L = 9, 14, 23, 3
    sl = oracle.band_slices_3d(d, h, w, L)
    cover = np.zeros((d, h, w), int)
    for zs, ys, xs in sl.values():
        cover[zs, ys, xs] += 1
    assert np.all(cover == 1)
    assert len(sl) == 1 + 7 * L

    def basis(n, j, high):
        c = np.zeros(n)
        c[oracle.band_slices_1d(n, j)[("d", j)].start if high else 0] = 1.0
        return oracle.inv_1d(c, j)

    for key, (zs, ys, xs) in sl.items():
        code, j = ("LLL", L) if key == "LLL" else key
        bx, by, bz = (basis(n, j, ch == "H") for n, ch in zip((w, h, d), code))
        vol = bz[:, None, None] * by[None, :, None] * bx[None, None, :]
        got = oracle.fwd_3d(vol, L)
        want = np.zeros_like(got)
        want[zs.start, ys.start, xs.start] = 1.0
        assert np.max(np.abs(got - want)) < 1e-12, key


def test_rejects_bad_levels(orc):
    with pytest.raises(ValueError):
        orc.fwd_1d(np.zeros(4), -1)
    with pytest.raises(ValueError):
        orc.fwd_2d(np.zeros((4, 4)), 63)
