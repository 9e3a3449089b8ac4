"""Seeded workload generators: determinism, shapes, distributions, storage rounding."""
import numpy as np
import pytest

from workloads import generators as G


def test_determinism_per_seed():
    a = G.white_signal(G.rng_for(1), 1000)
    b = G.white_signal(G.rng_for(1), 1000)
    c = G.white_signal(G.rng_for(2), 1000)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_config1_shape_and_moments():
    x = G.config1()
    assert x.dtype == np.float32 and x.shape == (65536,)
    assert abs(float(x.mean())) < 0.02 and abs(float(x.std()) - 1.0) < 0.02


def test_smooth_image_amplitude_and_noise():
    img = G.smooth_image(G.rng_for(2), 256, 256)
    assert img.shape == (256, 256)
    rms = float(np.sqrt(np.mean(img ** 2)))
    assert 100.0 < rms < 400.0          # 8 sinusoids of amplitude 100
    assert img.max() - img.min() > 400.0
    # the 0.1*U[0,255] noise has mean 12.75 and adds high-frequency content
    d = np.diff(img, axis=1)
    assert float(np.std(d)) > 5.0


def test_sine_mix_signal():
    x = G.sine_mix_signal(G.rng_for(3), 1 << 14)
    assert x.shape == (1 << 14,)
    assert 0.3 < float(np.std(x)) < 5.0


def test_uneven_sizes_config5_statistics():
    sizes = G.uneven_even_sizes(G.rng_for(5), 512)
    hs = np.array([h for h, _ in sizes]); ws = np.array([w for _, w in sizes])
    assert np.all(hs % 2 == 0) and np.all(ws % 2 == 0)
    assert hs.min() >= 256 and hs.max() <= 2048 and ws.min() >= 256 and ws.max() <= 2048
    frac16 = float(np.mean(np.concatenate([hs, ws]) % 16 == 0))
    assert 0.05 < frac16 < 0.25      # expected 1/8 of even sizes are divisible by 16


def test_dyadic_lengths():
    ls = G.dyadic_lengths(G.rng_for(3), 1024)
    ks = np.log2(ls)
    assert np.all(ks == np.round(ks)) and ks.min() >= 10 and ks.max() <= 20
    assert len(set(ks.astype(int))) == 11


def test_bf16_round_to_nearest_even_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000).astype(np.float32),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.4e38, 1e-40,
                                  np.inf, -np.inf], np.float32)])
    mine = G.f32_to_bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(mine, ref)
    # ties go to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert G.bf16_bits_to_f32(G.f32_to_bf16_bits(np.float32([1.00390625])))[0] == 1.0
    nan = G.f32_to_bf16_bits(np.float32([np.nan]))
    assert np.isnan(G.bf16_bits_to_f32(nan))[0]


def test_widen_roundtrip():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(100)
    for dt in (G.F32, G.BF16, G.F16):
        s = G.to_storage(x, dt)
        w = G.widen(s, dt)
        assert w.dtype == np.float64
        assert np.array_equal(G.to_storage(w, dt), s)
        rel = 2.0 ** -7 if dt == G.BF16 else (2.0 ** -10 if dt == G.F16 else 2.0 ** -23)
        assert np.max(np.abs(w - x) / np.maximum(np.abs(x), 1e-3)) <= rel
