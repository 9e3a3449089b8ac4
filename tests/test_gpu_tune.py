"""The autotuners on the GPU.

haar_tune_2d / haar_tune_1d time every candidate tile or chunk shape on the
caller's stream and record the fastest in the process-wide table; the plain
calls then consult that table.  Each test tunes one problem, checks that the
table holds the returned choice under the problem's key, and checks the
tuned plain call against the oracle."""
import json

import numpy as np
import pytest

import oracle
from gpu_util import (band_views, check_lowp_coeffs, check_lowp_signal, check_signal, rms, to_device,
                      to_host, torch_dtype)
from workloads import generators as G

pytestmark = pytest.mark.gpu

DTYPES = [G.F32, G.BF16, G.F16]


def _table(tmp_path):
    from paper_1002_2184_amd import _abi
    path = tmp_path / "table.json"
    assert _abi.haar_tune_save(str(path)) == 0
    return json.loads(path.read_text())


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("inverse", [False, True])
def test_tune_2d_then_plain_call(dt, inverse, tmp_path):
    from paper_1002_2184_amd import _abi
    from paper_1002_2184_amd import transform as T
    batch, h, w, L = 3, 200, 520, 4
    choice = T.tune_2d((batch, h, w), L, dtype=torch_dtype(dt), inverse=inverse)
    assert 0 <= choice < _abi.haar_tune_candidates_2d(dt)
    key = f"2d:{G.DTYPE_NAMES[dt]}:{'inv' if inverse else 'fwd'}:L{L}:h8:w10"
    assert _table(tmp_path)[key] == choice
    rng = np.random.default_rng(77 + dt + 5 * inverse)
    xs = G.to_storage(rng.standard_normal((batch, h, w)) * 3.0 + 1.0, dt)
    xw = G.widen(xs, dt)
    if not inverse:
        ref = oracle.fwd_2d(xw, L)
        got = G.widen(to_host(T.fwd2d(to_device(xs, dt), L), dt), dt)
        for b in range(batch):
            what = f"tuned fwd2d (candidate {choice}) item {b}"
            if dt == G.F32:
                check_signal(got[b], ref[b], rms(xw[b]), dt, what)
            else:
                check_lowp_coeffs(got[b], ref[b], rms(xw[b]), dt, band_views((h, w), L), what)
    else:
        cs = G.to_storage(oracle.fwd_2d(xw, L), dt)
        cw = G.widen(cs, dt)
        ref = oracle.inv_2d(cw, L)
        got = G.widen(to_host(T.inv2d(to_device(cs, dt), L), dt), dt)
        for b in range(batch):
            what = f"tuned inv2d (candidate {choice}) item {b}"
            (check_signal if dt == G.F32 else check_lowp_signal)(got[b], ref[b], rms(cw[b]), dt, what)


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("inverse", [False, True])
def test_tune_1d_then_plain_call(dt, inverse, tmp_path):
    from paper_1002_2184_amd import _abi
    from paper_1002_2184_amd import transform as T
    batch, n, L = 4, 50000, 14
    choice = T.tune_1d((batch, n), L, dtype=torch_dtype(dt), inverse=inverse)
    assert 0 <= choice < _abi.haar_tune_candidates_1d()
    key = f"1d:{G.DTYPE_NAMES[dt]}:{'inv' if inverse else 'fwd'}:L{L}:n16"
    assert _table(tmp_path)[key] == choice
    rng = np.random.default_rng(91 + dt + 5 * inverse)
    xs = G.to_storage(rng.standard_normal((batch, n)) * 2.0 - 0.5, dt)
    xw = G.widen(xs, dt)
    if not inverse:
        ref = oracle.fwd_1d(xw, L)
        got = G.widen(to_host(T.fwd1d(to_device(xs, dt), L), dt), dt)
        for b in range(batch):
            what = f"tuned fwd1d (candidate {choice}) item {b}"
            if dt == G.F32:
                check_signal(got[b], ref[b], rms(xw[b]), dt, what)
            else:
                check_lowp_coeffs(got[b], ref[b], rms(xw[b]), dt, band_views(n, L), what)
    else:
        cs = G.to_storage(oracle.fwd_1d(xw, L), dt)
        cw = G.widen(cs, dt)
        ref = oracle.inv_1d(cw, L)
        got = G.widen(to_host(T.inv1d(to_device(cs, dt), L), dt), dt)
        for b in range(batch):
            what = f"tuned inv1d (candidate {choice}) item {b}"
            (check_signal if dt == G.F32 else check_lowp_signal)(got[b], ref[b], rms(cw[b]), dt, what)
