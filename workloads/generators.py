"""Seeded synthetic workloads shaped like the paper's data.

The paper decomposes one subject's laser-Doppler recording (a 1D biosignal,
Sec. V, Figs. 9-11) and a natural image (Sec. V, Fig. 12).  Neither is
available here, so every workload is synthetic:

* ``white_signal``     -- i.i.d. N(0, 1) samples (plain 1D case);
* ``sine_mix_signal``  -- a sum of 3..10 sinusoids at 0.5..50 Hz sampled at
  1 kHz plus N(0, 0.1^2) noise (biosignal stand-in);
* ``smooth_image``     -- a sum of 8 random 2D sinusoids of amplitude 100 plus
  0.1 * U[0, 255] noise (natural-image stand-in);
* ``uniform_images``   -- U[0, 1] images of uneven even sizes;
* ``phantom_volume``   -- CT-like volumes (ellipsoids of tissue intensity in
  air, plus noise) for the 3D transform.

All draws use ``numpy.random.default_rng(SEED + config)`` (PCG64) in float64
and are rounded to the storage type with round-to-nearest-even.  Reduced
precision data is carried as raw bit patterns (``uint16``) so that numpy
needs no bfloat16 type.
"""
from __future__ import annotations

import numpy as np

SEED = 10022184

F32, BF16, F16 = 0, 1, 2
DTYPE_NAMES = {F32: "f32", BF16: "bf16", F16: "f16"}


def rng_for(config: int, salt: int = 0) -> np.random.Generator:
    """The generator of one workload: PCG64 seeded with SEED + config (+ salt)."""
    return np.random.default_rng(SEED + int(config) + 1000 * int(salt))


# --------------------------------------------------------------------------
# storage conversions (round to nearest even)
# --------------------------------------------------------------------------
def f32_to_bf16_bits(a) -> np.ndarray:
    """float32 -> bfloat16 bit patterns (uint16), round-to-nearest-even, NaN kept quiet."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    bias = ((u >> 16) & 1) + 0x7FFF
    r = ((u + bias) >> 16).astype(np.uint16)
    nan = np.isnan(a)
    if nan.any():
        r[nan] = (((u[nan] >> 16) | 0x40) & 0xFFFF).astype(np.uint16)
    return r


def bf16_bits_to_f32(b) -> np.ndarray:
    """bfloat16 bit patterns (uint16) -> float32 (exact)."""
    b = np.ascontiguousarray(b, dtype=np.uint16)
    return (b.astype(np.uint32) << 16).view(np.float32)


def to_storage(x64, dtype: int) -> np.ndarray:
    """float64 values -> storage array: float32, or uint16 bit patterns for bf16/f16."""
    x32 = np.asarray(x64, dtype=np.float32)
    if dtype == F32:
        return np.ascontiguousarray(x32)
    if dtype == BF16:
        return f32_to_bf16_bits(x32)
    if dtype == F16:
        return np.ascontiguousarray(np.asarray(x64, dtype=np.float64).astype(np.float16)).view(np.uint16)
    raise ValueError(f"unknown dtype code {dtype}")


def widen(stored, dtype: int) -> np.ndarray:
    """Storage array -> exact float64 values."""
    if dtype == F32:
        return np.asarray(stored, dtype=np.float32).astype(np.float64)
    if dtype == BF16:
        return bf16_bits_to_f32(stored).astype(np.float64)
    if dtype == F16:
        return np.ascontiguousarray(stored, dtype=np.uint16).view(np.float16).astype(np.float64)
    raise ValueError(f"unknown dtype code {dtype}")


def storage_itemsize(dtype: int) -> int:
    return 4 if dtype == F32 else 2


# --------------------------------------------------------------------------
# signal / image families
# --------------------------------------------------------------------------
def white_signal(rng: np.random.Generator, shape) -> np.ndarray:
    """i.i.d. N(0, 1) in float64."""
    return rng.standard_normal(shape)


def sine_mix_signal(rng: np.random.Generator, n: int, fs: float = 1000.0) -> np.ndarray:
    """Sum of K ~ U{3..10} sinusoids, f ~ U[0.5, 50] Hz, A ~ U[0.5, 1.5],
    phase ~ U[0, 2pi), sampled at fs, plus N(0, 0.1^2) noise (float64)."""
    k = int(rng.integers(3, 11))
    f = rng.uniform(0.5, 50.0, k)
    amp = rng.uniform(0.5, 1.5, k)
    ph = rng.uniform(0.0, 2.0 * np.pi, k)
    t = np.arange(n, dtype=np.float64) / fs
    x = np.zeros(n, dtype=np.float64)
    for i in range(k):
        x += amp[i] * np.sin(2.0 * np.pi * f[i] * t + ph[i])
    x += rng.normal(0.0, 0.1, n)
    return x


def smooth_image(rng: np.random.Generator, h: int, w: int, terms: int = 8,
                 amplitude: float = 100.0) -> np.ndarray:
    """sum_i amplitude*sin(2pi(fx_i*x/w + fy_i*y/h) + phi_i) + 0.1*U[0,255] (float64).

    fx, fy ~ U[0.5, 16] cycles per image with a random sign, phi ~ U[0, 2pi).
    The sine of a sum is expanded into row and column factors so that a
    4096 x 4096 field costs two outer products per term."""
    fx = rng.uniform(0.5, 16.0, terms) * rng.choice([-1.0, 1.0], terms)
    fy = rng.uniform(0.5, 16.0, terms) * rng.choice([-1.0, 1.0], terms)
    ph = rng.uniform(0.0, 2.0 * np.pi, terms)
    xs = np.arange(w, dtype=np.float64) / w
    ys = np.arange(h, dtype=np.float64) / h
    img = np.zeros((h, w), dtype=np.float64)
    for i in range(terms):
        cx = 2.0 * np.pi * fx[i] * xs
        cy = 2.0 * np.pi * fy[i] * ys + ph[i]
        img += amplitude * (np.outer(np.cos(cy), np.sin(cx)) + np.outer(np.sin(cy), np.cos(cx)))
    img += 0.1 * rng.uniform(0.0, 255.0, (h, w))
    return img


def phantom_volume(rng: np.random.Generator, d: int, h: int, w: int, organs: int = 8) -> np.ndarray:
    """A CT-like volume [d, h, w] (float64): air 0, a body ellipsoid of 1.0
    (radii 0.45 of each side, centred), `organs` ellipsoids inside it with
    radii U[0.04, 0.18] of each side and intensities U[-0.5, 0.8] added,
    plus N(0, 0.02^2) noise.  Stand-in for the medical volumes of the
    paper's application; the intensities mimic normalised Hounsfield units."""
    zs = (np.arange(d, dtype=np.float64) + 0.5) / d
    ys = (np.arange(h, dtype=np.float64) + 0.5) / h
    xs = (np.arange(w, dtype=np.float64) + 0.5) / w

    def ellipsoid(c, r):
        qz = ((zs - c[0]) / r[0]) ** 2
        qy = ((ys - c[1]) / r[1]) ** 2
        qx = ((xs - c[2]) / r[2]) ** 2
        return (qz[:, None, None] + qy[None, :, None] + qx[None, None, :]) < 1.0

    v = np.zeros((d, h, w), dtype=np.float64)
    v[ellipsoid((0.5, 0.5, 0.5), (0.45, 0.45, 0.45))] = 1.0
    for _ in range(organs):
        c = rng.uniform(0.3, 0.7, 3)
        r = rng.uniform(0.04, 0.18, 3)
        v[ellipsoid(c, r)] += rng.uniform(-0.5, 0.8)
    v += rng.normal(0.0, 0.02, (d, h, w))
    return v


def uneven_even_sizes(rng: np.random.Generator, count: int, lo: int = 128,
                      hi: int = 1024):
    """count pairs (H, W), each 2*U{lo..hi} independently (even sizes)."""
    hs = 2 * rng.integers(lo, hi + 1, count)
    ws = 2 * rng.integers(lo, hi + 1, count)
    return [(int(a), int(b)) for a, b in zip(hs, ws)]


def dyadic_lengths(rng: np.random.Generator, count: int, kmin: int = 10,
                   kmax: int = 20):
    """count lengths 2^k with k ~ U{kmin..kmax}."""
    ks = rng.integers(kmin, kmax + 1, count)
    return [1 << int(k) for k in ks]


# --------------------------------------------------------------------------
# the five benchmark workloads
# --------------------------------------------------------------------------
CONFIGS = {
    1: dict(name="1d-white-65536-L16", dim=1, n=65536, levels=16, dtype=F32),
    2: dict(name="2d-smooth-4096x4096-L5", dim=2, h=4096, w=4096, levels=5, dtype=F32),
    3: dict(name="1d-batched-uneven-1024x2^[10,20]-fulldepth", dim=1, count=1024, dtype=F32),
    4: dict(name="2d-autograd-64x3x512x512-L3", dim=2, h=512, w=512, batch=192, levels=3, dtype=F32),
    5: dict(name="2d-batched-bf16-512-uneven-L4", dim=2, count=512, levels=4, dtype=BF16),
}


def config1():
    """One N(0,1) float32 signal of 65536 samples; 16 levels."""
    rng = rng_for(1)
    return to_storage(white_signal(rng, 65536), F32)


def config2(h: int = 4096, w: int = 4096):
    """One float32 smooth image (8 sinusoids, amplitude 100, + 0.1*U[0,255]); 5 levels."""
    rng = rng_for(2)
    return to_storage(smooth_image(rng, h, w), F32)


def config3(count: int = 1024, kmin: int = 10, kmax: int = 20):
    """count float32 sine-mix signals of lengths 2^k, k ~ U{kmin..kmax}; full depth.

    Returns a list of float32 arrays (levels = log2 of each length)."""
    rng = rng_for(3)
    lengths = dyadic_lengths(rng, count, kmin, kmax)
    return [to_storage(sine_mix_signal(rng, n), F32) for n in lengths]


def config4(batch: int = 192, h: int = 512, w: int = 512):
    """An N(0,1) float32 tensor [batch, h, w] (64 x 3 channels of 512^2); 3 levels."""
    rng = rng_for(4)
    out = np.empty((batch, h, w), dtype=np.float32)
    for b in range(batch):
        out[b] = rng.standard_normal((h, w))
    return out


def config5(count: int = 512, lo: int = 128, hi: int = 1024, dtype: int = BF16,
            with_grad: bool = True):
    """count U[0,1] images with even H, W ~ 2*U{lo..hi}, stored as bf16 bits
    (uint16), plus an N(0,1) upstream gradient per image in the same format.

    Returns (images, grads); grads is None when with_grad is False."""
    rng = rng_for(5)
    sizes = uneven_even_sizes(rng, count, lo, hi)
    imgs, grads = [], []
    for (h, w) in sizes:
        imgs.append(to_storage(rng.uniform(0.0, 1.0, (h, w)), dtype))
        if with_grad:
            grads.append(to_storage(rng.standard_normal((h, w)), dtype))
    return imgs, (grads if with_grad else None)
