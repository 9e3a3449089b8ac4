"""Batched uneven transforms (plans, one persistent launch per execute) against the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import (band_views, check_lowp_coeffs, check_lowp_signal, check_signal, rms, to_device,
                      to_host)
from workloads import generators as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_1002_2184_amd import plan
    return plan


SHAPES_2D = [(64, 96), (33, 300), (256, 512), (7, 5), (100, 102), (130, 66), (512, 257), (32, 256)]


def _lv(shapes, L):
    return [min(L, int(np.ceil(np.log2(max(h, w))))) for (h, w) in shapes]


def _imgs(dt, shapes, seed):
    rng = np.random.default_rng(seed)
    return [G.to_storage(rng.standard_normal(s) * 2.0 + 1.0, dt) for s in shapes]


@pytest.mark.parametrize("dt", [G.F32, G.BF16, G.F16])
@pytest.mark.parametrize("L", [1, 3, 5])
def test_plan2d_matches_oracle(P, dt, L):
    import torch
    shapes = [(h, w) for (h, w) in SHAPES_2D if max(h, w) >= (1 << L) or L == 1]
    xs = _imgs(dt, shapes, seed=L + 10 * dt)
    xd = [to_device(x, dt) for x in xs]
    yd = [torch.empty_like(x) for x in xd]
    plan = P.Plan2D(xd, yd, L)
    for rep in range(3):                       # counters reset by the kernel itself
        for y in yd:
            y.fill_(float("nan"))
        plan.execute()
        torch.cuda.synchronize()
        for x, y, s in zip(xs, yd, shapes):
            xw = G.widen(x, dt)
            ref = oracle.fwd_2d(xw, L)
            yw = G.widen(to_host(y, dt), dt)
            if dt == G.F32:
                check_signal(yw, ref, rms(xw), dt, f"plan fwd {s} L={L} rep {rep}")
            else:
                check_lowp_coeffs(yw, ref, rms(xw), dt, band_views(s, L), f"plan fwd {s} L={L}")
    # inverse plan on the oracle's stored coefficients
    cs = [G.to_storage(oracle.fwd_2d(G.widen(x, dt), L), dt) for x in xs]
    cd = [to_device(c, dt) for c in cs]
    zd = [torch.empty_like(c) for c in cd]
    iplan = P.Plan2D(cd, zd, L, inverse=True)
    iplan.execute()
    torch.cuda.synchronize()
    for c, z, s in zip(cs, zd, shapes):
        cw = G.widen(c, dt)
        xref = oracle.inv_2d(cw, L)
        zw = G.widen(to_host(z, dt), dt)
        (check_signal if dt == G.F32 else check_lowp_signal)(zw, xref, rms(cw), dt, f"plan inv {s}")


def test_plan2d_configs_and_tune(P):
    import torch
    xs = _imgs(G.F32, SHAPES_2D, seed=3)
    xd = [to_device(x, G.F32) for x in xs]
    yd = [torch.empty_like(x) for x in xd]
    lv = _lv(SHAPES_2D, 4)
    plan = P.Plan2D(xd, yd, lv)
    refs = [oracle.fwd_2d(x.astype(np.float64), L) for x, L in zip(xs, lv)]
    # tile shape + 2 * schedule (strided, atomic claiming, one tile per WG,
    # one tile per WG XCD-contiguous with write-back stores, one tile per WG
    # XCD-contiguous)
    for cfg in range(10):
        plan.set_config(cfg)
        plan.execute()
        torch.cuda.synchronize()
        for y, r, x in zip(yd, refs, xs):
            check_signal(to_host(y, G.F32).astype(np.float64), r, rms(x), G.F32, f"config {cfg}")
    choice = plan.tune()
    assert choice in range(10)
    plan.execute()
    torch.cuda.synchronize()
    for y, r, x in zip(yd, refs, xs):
        check_signal(to_host(y, G.F32).astype(np.float64), r, rms(x), G.F32, "tuned")
    tiles, grid = plan.info()
    assert tiles > 0 and 1 <= grid <= tiles


@pytest.mark.parametrize("dt", [G.F32, G.BF16])
@pytest.mark.parametrize("inverse", [False, True])
def test_plan2d_every_config_both_directions(P, dt, inverse):
    """All 10 configurations (2 tile shapes x 5 schedules) of an analysis and of
    a synthesis plan, two executes each, on images whose rows mostly start
    inside a cache line (odd and even widths, widths not a multiple of 64)."""
    import torch
    shapes = SHAPES_2D + [(96, 1030), (18, 2050), (300, 44)]
    L = 4
    lv = _lv(shapes, L)
    xs = _imgs(dt, shapes, seed=41 + dt + 2 * inverse)
    if inverse:
        ins = [G.to_storage(oracle.fwd_2d(G.widen(x, dt), l), dt) for x, l in zip(xs, lv)]
        refs = [oracle.inv_2d(G.widen(c, dt), l) for c, l in zip(ins, lv)]
    else:
        ins = xs
        refs = [oracle.fwd_2d(G.widen(x, dt), l) for x, l in zip(xs, lv)]
    xd = [to_device(x, dt) for x in ins]
    yd = [torch.empty_like(x) for x in xd]
    plan = P.Plan2D(xd, yd, lv, inverse=inverse)
    for cfg in range(10):
        plan.set_config(cfg)
        for rep in range(2):
            for y in yd:
                y.fill_(float("nan"))
            plan.execute()
            torch.cuda.synchronize()
            for x, y, r, s, l in zip(ins, yd, refs, shapes, lv):
                yw = G.widen(to_host(y, dt), dt)
                scale = rms(G.widen(x, dt))
                what = f"{'inv' if inverse else 'fwd'} config {cfg} rep {rep} {s} L={l}"
                if dt == G.F32:
                    check_signal(yw, r, scale, dt, what)
                elif inverse:
                    check_lowp_signal(yw, r, scale, dt, what)
                else:
                    check_lowp_coeffs(yw, r, scale, dt, band_views(s, l), what)


LENGTHS_1D = [1 << 20, 65536, 100003, 8192, 5000, 4096, 4095, 1024, 777, 1 << 17, 3 * 4096]


def _sigs(dt, lengths, seed):
    rng = np.random.default_rng(seed)
    return [G.to_storage(rng.standard_normal(n) + 0.3, dt) for n in lengths]


@pytest.mark.parametrize("dt", [G.F32, G.BF16, G.F16])
def test_plan1d_full_depth_matches_oracle(P, dt):
    import torch
    xs = _sigs(dt, LENGTHS_1D, seed=5 + dt)
    levels = [int(np.ceil(np.log2(n))) for n in LENGTHS_1D]
    xd = [to_device(x, dt) for x in xs]
    yd = [torch.empty_like(x) for x in xd]
    plan = P.Plan1D(xd, yd, levels)
    for rep in range(2):
        for y in yd:
            y.fill_(float("nan"))
        plan.execute()
        torch.cuda.synchronize()
        for x, y, L in zip(xs, yd, levels):
            xw = G.widen(x, dt)
            ref = oracle.fwd_1d(xw, L)
            yw = G.widen(to_host(y, dt), dt)
            if dt == G.F32:
                check_signal(yw, ref, rms(xw), dt, f"plan1d fwd n={x.size} L={L} rep {rep}")
            else:
                # items deeper than 12 levels keep their level-12 values in FP32
                # between the two kernels: every coefficient within 1 ulp
                check_lowp_coeffs(yw, ref, rms(xw), dt, band_views(x.size, L), f"plan1d fwd n={x.size}")
    # the synthesis plan on the oracle's stored coefficients (items deeper than
    # 12 levels walk their ancestor path through the 16-bit coefficients)
    cs = [G.to_storage(oracle.fwd_1d(G.widen(x, dt), L), dt) for x, L in zip(xs, levels)]
    cd = [to_device(c, dt) for c in cs]
    zd = [torch.empty_like(c) for c in cd]
    iplan = P.Plan1D(cd, zd, levels, inverse=True)
    chk = check_signal if dt == G.F32 else check_lowp_signal
    for rep in range(2):
        for z in zd:
            z.fill_(float("nan"))
        iplan.execute()
        torch.cuda.synchronize()
        for c, z, L in zip(cs, zd, levels):
            cw = G.widen(c, dt)
            chk(G.widen(to_host(z, dt), dt), oracle.inv_1d(cw, L), rms(cw), dt,
                f"plan1d inv n={c.size} L={L} rep {rep}")


def test_plan1d_schedules(P):
    """The three work-list schedules (strided, atomic claiming, one chunk per
    work-group) give the oracle's result, executed twice each (the claiming
    counters reset themselves)."""
    import torch
    lengths = [1 << 16, 5000, 4096, 70000, 777]
    levels = [16, 13, 12, 14, 10]
    xs = _sigs(G.F32, lengths, seed=19)
    xd = [to_device(x, G.F32) for x in xs]
    yd = [torch.empty_like(x) for x in xd]
    plan = P.Plan1D(xd, yd, levels)
    refs = [oracle.fwd_1d(x.astype(np.float64), L) for x, L in zip(xs, levels)]
    cs = [to_device(G.to_storage(r, G.F32), G.F32) for r in refs]
    zd = [torch.empty_like(c) for c in cs]
    iplan = P.Plan1D(cs, zd, levels, inverse=True)
    for sched in (0, 1, 2, 0):
        plan.set_config(sched)
        iplan.set_config(sched)
        for rep in range(2):
            for y in yd + zd:
                y.fill_(float("nan"))
            plan.execute()
            iplan.execute()
            torch.cuda.synchronize()
            for x, y, z, r, L in zip(xs, yd, zd, refs, levels):
                what = f"schedule {sched} n={x.size} L={L} rep {rep}"
                check_signal(to_host(y, G.F32).astype(np.float64), r, rms(x), G.F32, what)
                xref = oracle.inv_1d(G.widen(G.to_storage(r, G.F32), G.F32), L)
                check_signal(to_host(z, G.F32).astype(np.float64), xref, rms(x), G.F32, what + " inv")
    assert plan.tune() in (0, 1, 2)


def test_plan1d_partial_levels(P):
    import torch
    lengths = [50000, 4096, 123, 70000]
    levels = [7, 12, 5, 14]
    xs = _sigs(G.F32, lengths, seed=9)
    xd = [to_device(x, G.F32) for x in xs]
    yd = [torch.empty_like(x) for x in xd]
    P.Plan1D(xd, yd, levels).execute()
    torch.cuda.synchronize()
    for x, y, L in zip(xs, yd, levels):
        check_signal(to_host(y, G.F32).astype(np.float64), oracle.fwd_1d(x.astype(np.float64), L),
                     rms(x), G.F32, f"n={x.size} L={L}")


def test_plan_graph_replay(P):
    """Capture execute() of a 2D and a 1D plan in one graph; replay 3 times with
    eager work in between; every replay equals the eager result."""
    import torch
    xs2 = [to_device(x, G.F32) for x in _imgs(G.F32, SHAPES_2D[:5], seed=11)]
    ys2 = [torch.empty_like(x) for x in xs2]
    xs1 = [to_device(x, G.F32) for x in _sigs(G.F32, [1 << 18, 5000, 4096], seed=12)]
    ys1 = [torch.empty_like(x) for x in xs1]
    p2 = P.Plan2D(xs2, ys2, _lv(SHAPES_2D[:5], 5))
    p1 = P.Plan1D(xs1, ys1, [18, 13, 12])
    p2.set_config(3)                  # atomic claiming: the counters must reset themselves
    p1.set_config(1)
    p2.execute()
    p1.execute()
    torch.cuda.synchronize()
    eager = [y.clone() for y in ys2 + ys1]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            p2.execute()
            p1.execute()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        for y in ys2 + ys1:
            y.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()          # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for a, b in zip(ys2 + ys1, eager):
            assert torch.equal(a, b), f"replay {rep} differs from eager"


def test_config3_sample(P):
    """A 48-signal sample of the batched uneven 1D workload (2^10..2^20, full depth)."""
    import torch
    sigs = G.config3(count=48)
    levels = [int(np.log2(s.size)) for s in sigs]
    xd = [to_device(s, G.F32) for s in sigs]
    yd = [torch.empty_like(x) for x in xd]
    P.Plan1D(xd, yd, levels).execute()
    torch.cuda.synchronize()
    worst = 0.0
    for s, y, L in zip(sigs, yd, levels):
        xw = s.astype(np.float64)
        worst = max(worst, check_signal(to_host(y, G.F32).astype(np.float64), oracle.fwd_1d(xw, L),
                                        rms(xw), G.F32, f"config3 n={s.size}"))
    print(f"config3 sample worst err/RMS {worst:.3e}")


def test_config5_sample_per_band(P):
    """A 24-image sample of the BF16 batched workload: per-level/per-band gate,
    the signal-domain max-abs gate on the backward (U[0,1] images), 1 ulp."""
    import torch
    imgs, grads = G.config5(count=24)
    shapes = [im.shape for im in imgs]
    xd = [to_device(x, G.BF16) for x in imgs]
    yd = [torch.empty_like(x) for x in xd]
    P.Plan2D(xd, yd, 4).execute()
    gd = [to_device(g, G.BF16) for g in grads]
    zd = [torch.empty_like(g) for g in gd]
    P.Plan2D(gd, zd, 4, inverse=True).execute()
    torch.cuda.synchronize()
    per_level = {}       # level (0 = LL_4) -> worst (max err / band peak, RMS err / band RMS)
    bwd_worst = 0.0
    for x, y, g, z, s in zip(imgs, yd, grads, zd, shapes):
        xw = G.widen(x, G.BF16)
        ref = oracle.fwd_2d(xw, 4)
        table = check_lowp_coeffs(G.widen(to_host(y, G.BF16), G.BF16), ref, rms(xw), G.BF16,
                                  band_views(tuple(s), 4), f"config5 fwd {s}", band_gate=True)
        for key, v in table.items():
            lev = 0 if key == "LL" else key[1]
            a, b = per_level.get(lev, (0.0, 0.0))
            per_level[lev] = (max(a, v["max_err_over_band_peak"]), max(b, v["rms_err_over_band_rms"]))
        gw = G.widen(g, G.BF16)
        gref = oracle.inv_2d(gw, 4)
        zw = G.widen(to_host(z, G.BF16), G.BF16)
        bwd_worst = max(bwd_worst, check_lowp_signal(zw, gref, rms(gw), G.BF16, f"config5 bwd {s}"))
    # the per-level error report of the BF16 batch (worst over the sample)
    print("\nBF16 batch, error of the stored coefficients against the FP64 oracle, worst of 24 images:")
    for lev in sorted(per_level):
        a, b = per_level[lev]
        name = "LL_4" if lev == 0 else f"level {lev} (HL, LH, HH)"
        print(f"  {name:>22}: max err / max|band| {a:.2e}, RMS err / RMS band {b:.2e}")
    print(f"  backward (synthesis of the BF16 gradient): max err / RMS(g) {bwd_worst:.2e}")
        # images are U[0, 1]: the literal max-abs signal gate also holds for a
        # round trip of the image itself
    rt = [torch.empty_like(y) for y in yd]
    P.Plan2D(yd, rt, 4, inverse=True).execute()
    torch.cuda.synchronize()
    for x, r, s in zip(imgs, rt, shapes):
        xw = G.widen(x, G.BF16)
        check_signal(G.widen(to_host(r, G.BF16), G.BF16), xw, rms(xw), G.BF16, f"config5 round trip {s}")
