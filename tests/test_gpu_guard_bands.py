"""Guard bands around the outputs of every entry point: a stray store of an
edge tile, a ragged chunk or a deep pass would land in memory next to the
output.  Each output here is a view into a larger buffer whose head and tail
(GUARD elements each) hold a canary bit pattern, a NaN that no transform of
finite data produces.  After each call the host checks that

* both guard bands still hold the canary, bit for bit (no store outside the
  output);
* no canary is left inside the output (every output element was written);
* the input is unchanged (out-of-place contract).

The values themselves are checked against the oracle by the parity files;
here a loose check (round trip or oracle within the parity gates on small
shapes) keeps the calls honest."""
import numpy as np
import pytest

import oracle
from gpu_util import check_lowp_signal, check_signal, rms, to_device, to_host
from workloads import generators as G

pytestmark = pytest.mark.gpu

GUARD = 4096
CANARY = {G.F32: 0x7FA5A5A5, G.BF16: 0x7FA5, G.F16: 0x7E5A}


class Guarded:
    """An output of `shape` inside a buffer with canary-filled guard bands."""

    def __init__(self, shape, dt):
        import torch
        self.dt, self.shape = dt, tuple(shape)
        self.n = int(np.prod(shape)) if len(shape) else 1
        if dt == G.F32:
            bits = np.full(self.n + 2 * GUARD, CANARY[dt], dtype=np.uint32).view(np.int32)
            self.buf = torch.from_numpy(bits).cuda().view(torch.float32)
        else:
            bits = np.full(self.n + 2 * GUARD, CANARY[dt], dtype=np.uint16).view(np.int16)
            tdt = torch.bfloat16 if dt == G.BF16 else torch.float16
            self.buf = torch.from_numpy(bits).cuda().view(tdt)
        self.view = self.buf[GUARD:GUARD + self.n].view(self.shape)

    def check(self, what):
        import torch
        torch.cuda.synchronize()
        w = 32 if self.dt == G.F32 else 16
        raw = self.buf.view(torch.int32 if w == 32 else torch.int16).cpu().numpy()
        raw = raw.view(np.uint32 if w == 32 else np.uint16)
        head, body, tail = raw[:GUARD], raw[GUARD:GUARD + self.n], raw[GUARD + self.n:]
        c = CANARY[self.dt]
        assert np.all(head == c), f"{what}: {int(np.sum(head != c))} stores before the output"
        assert np.all(tail == c), f"{what}: {int(np.sum(tail != c))} stores after the output"
        left = int(np.sum(body == c))
        assert left == 0, f"{what}: {left} output elements never written"
        return to_host(self.view, self.dt)


def mlev(*sizes):
    """Deepest meaningful level count: ceil(log2(largest size))."""
    m = max(sizes)
    return int(np.ceil(np.log2(m))) if m > 1 else 0


def _input(shape, dt, seed):
    rng = np.random.default_rng(seed)
    return G.to_storage(rng.standard_normal(shape) * 2.0 + 0.5, dt)


def _unchanged(xd, xs, dt, what):
    assert np.array_equal(to_host(xd, dt), xs), f"{what}: input modified"


DTS = [G.F32, G.BF16, G.F16]
SHAPES_1D = [(3, 1), (2, 17), (1, 4095), (2, 4097), (1, 12289), (1, 70001)]
SHAPES_2D = [(2, 1, 7), (1, 33, 257), (2, 95, 513), (1, 64, 1030), (1, 300, 700)]
SHAPES_3D = [(1, 9, 17, 33), (2, 16, 16, 16), (1, 20, 40, 70)]


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("shape", SHAPES_1D, ids=str)
def test_guard_1d(T, dt, shape):
    n = shape[-1]
    for L in sorted({min(1, mlev(n)), min(5, mlev(n)), mlev(n)}):
        xs = _input(shape, dt, n + L)
        xd = to_device(xs, dt)
        y = Guarded(shape, dt)
        T.fwd1d(xd, L, out=y.view)
        yh = y.check(f"fwd1d {shape} L={L}")
        _unchanged(xd, xs, dt, f"fwd1d {shape} L={L}")
        z = Guarded(shape, dt)
        T.inv1d(y.view, L, out=z.view)
        z.check(f"inv1d {shape} L={L}")
        _unchanged(y.view, yh, dt, f"inv1d {shape} L={L}")
        if dt == G.F32:
            xw = xs.astype(np.float64)
            for b in range(shape[0]):
                check_signal(G.widen(yh, dt)[b], oracle.fwd_1d(xw[b], L), rms(xw[b]), dt, "fwd1d values")


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("shape", SHAPES_2D, ids=str)
def test_guard_2d(T, dt, shape):
    h, w = shape[-2:]
    for L in sorted({min(1, mlev(h, w)), min(5, mlev(h, w)), mlev(h, w)}):
        xs = _input(shape, dt, h * w + L)
        xd = to_device(xs, dt)
        y = Guarded(shape, dt)
        T.fwd2d(xd, L, out=y.view)
        yh = y.check(f"fwd2d {shape} L={L}")
        _unchanged(xd, xs, dt, f"fwd2d {shape} L={L}")
        z = Guarded(shape, dt)
        T.inv2d(y.view, L, out=z.view)
        zh = z.check(f"inv2d {shape} L={L}")
        _unchanged(y.view, yh, dt, f"inv2d {shape} L={L}")
        xw = G.widen(xs, dt)
        ref = oracle.inv_2d(G.widen(yh, dt), L)
        for b in range(shape[0]):
            if dt == G.F32:
                check_signal(G.widen(zh, dt)[b], ref[b], rms(xw[b]), dt, "inv2d values")
            else:
                check_lowp_signal(G.widen(zh, dt)[b], ref[b], rms(xw[b]), dt, "inv2d values")


@pytest.mark.parametrize("dt", [G.F32, G.BF16])
def test_guard_2d_every_tile_config(T, dt):
    """Every tile shape of the tuner's table, forced, on a shape with edge tiles."""
    from paper_1002_2184_amd import _abi
    shape, L = (2, 70, 530), 5
    xs = _input(shape, dt, 99)
    xd = to_device(xs, dt)
    try:
        for c in range(_abi.haar_tune_candidates_2d(dt)):
            assert _abi.haar_force_config_2d(dt, c) == 0
            y = Guarded(shape, dt)
            T.fwd2d(xd, L, out=y.view)
            yh = y.check(f"config {c} fwd2d")
            z = Guarded(shape, dt)
            T.inv2d(y.view, L, out=z.view)
            z.check(f"config {c} inv2d")
            _unchanged(y.view, yh, dt, f"config {c} inv2d")
    finally:
        _abi.haar_force_config_2d(dt, -1)


@pytest.mark.parametrize("dt", DTS)
@pytest.mark.parametrize("shape", SHAPES_3D, ids=str)
def test_guard_3d(T, dt, shape):
    d, h, w = shape[-3:]
    for L in sorted({min(1, mlev(d, h, w)), min(3, mlev(d, h, w)), mlev(d, h, w)}):
        xs = _input(shape, dt, d * h * w + L)
        xd = to_device(xs, dt)
        y = Guarded(shape, dt)
        T.fwd3d(xd, L, out=y.view)
        yh = y.check(f"fwd3d {shape} L={L}")
        _unchanged(xd, xs, dt, f"fwd3d {shape} L={L}")
        z = Guarded(shape, dt)
        T.inv3d(y.view, L, out=z.view)
        z.check(f"inv3d {shape} L={L}")
        _unchanged(y.view, yh, dt, f"inv3d {shape} L={L}")


@pytest.mark.parametrize("dt", DTS)
def test_guard_fused(T, dt):
    """Fused shrinkage (1D, 2D), the training step (both entry points) and
    the direct bank."""
    from paper_1002_2184_amd import _abi
    import torch
    for shape, L in (((2, 4100), 12), ((1, 777), 5)):
        xs = _input(shape, dt, 7 + L)
        xd = to_device(xs, dt)
        y = Guarded(shape, dt)
        T.shrink1d(xd, L, 0.3, "soft", out=y.view)
        y.check(f"shrink1d {shape}")
        _unchanged(xd, xs, dt, "shrink1d")
        y = Guarded(shape, dt)
        T.direct1d(xd, min(L, 8), out=y.view)
        yh = y.check(f"direct1d fwd {shape}")
        z = Guarded(shape, dt)
        T.direct1d(y.view, min(L, 8), inverse=True, out=z.view)
        z.check(f"direct1d inv {shape}")
        _unchanged(y.view, yh, dt, "direct1d inv")
    for shape, L in (((2, 70, 530), 5), ((1, 33, 1025), 3)):
        xs = _input(shape, dt, 11 + L)
        xd = to_device(xs, dt)
        y = Guarded(shape, dt)
        T.shrink2d(xd, L, 0.3, "hard", out=y.view)
        y.check(f"shrink2d {shape}")
        _unchanged(xd, xs, dt, "shrink2d")
        y = Guarded(shape, dt)
        T.l1_grad2d(xd, L, out=y.view)
        y.check(f"l1_grad2d {shape}")
        _unchanged(xd, xs, dt, "l1_grad2d")
        g = Guarded(shape, dt)
        batch = shape[0]
        loss = torch.empty(batch, dtype=torch.float64, device="cuda")
        st = torch.cuda.current_stream().cuda_stream
        _abi.check(_abi.haar_l1_grad_2d_noalloc(xd.data_ptr(), g.view.data_ptr(), loss.data_ptr(),
                                                shape[1], shape[2], L, batch, dt, st))
        g.check(f"l1_grad2d_noalloc {shape}")
        _unchanged(xd, xs, dt, "l1_grad2d_noalloc")


@pytest.mark.parametrize("dt", [G.F32, G.BF16])
def test_guard_plans(dt):
    """Plans of uneven items, every item's output guarded, both directions."""
    from paper_1002_2184_amd import plan as P
    rng = np.random.default_rng(5150 + dt)
    shapes2 = [(int(rng.integers(2, 300)), int(rng.integers(2, 900))) for _ in range(12)] + [(256, 512)]
    xs = [_input(s, dt, i) for i, s in enumerate(shapes2)]
    xd = [to_device(a, dt) for a in xs]
    for inverse in (False, True):
        outs = [Guarded(s, dt) for s in shapes2]
        lv = [min(4, mlev(*s)) for s in shapes2]
        P.Plan2D(xd, [o.view for o in outs], lv, inverse=inverse).execute()
        for i, o in enumerate(outs):
            o.check(f"plan2d item {i} {shapes2[i]} inverse={inverse}")
            _unchanged(xd[i], xs[i], dt, f"plan2d item {i}")
    lens = [int(rng.integers(2, 20000)) for _ in range(12)] + [1 << 17]
    ys = [_input((n,), dt, n) for n in lens]
    yd = [to_device(a, dt) for a in ys]
    lv1 = [min(mlev(n), 20) for n in lens]
    for inverse in (False, True):
        outs = [Guarded((n,), dt) for n in lens]
        P.Plan1D(yd, [o.view for o in outs], lv1, inverse=inverse).execute()
        for i, o in enumerate(outs):
            o.check(f"plan1d item {i} n={lens[i]} inverse={inverse}")
            _unchanged(yd[i], ys[i], dt, f"plan1d item {i}")


@pytest.fixture(scope="module")
def T():
    from paper_1002_2184_amd import transform
    return transform
