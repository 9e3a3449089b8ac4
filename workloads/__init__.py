"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package holds no wavelet arithmetic: it only draws random numbers and
converts between storage formats (float32, bfloat16 bit patterns, float16).
Both the GPU path and the FP64 oracle are fed the same bytes from here.
"""
from .generators import *  # noqa: F401,F403
