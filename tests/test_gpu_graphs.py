"""Graph capture of the entry points that use stream-ordered scratch
(hipMallocAsync / hipFreeAsync inside the call): deep 2D and 3D transforms
and the fused training step.  One graph holds them all; it is replayed
three times with eager work in between, and every replay must equal the
eager result bit for bit (the same kernels run in the same order)."""
import numpy as np
import pytest

from workloads import generators as G

pytestmark = pytest.mark.gpu


def test_scratch_entry_points_replay_in_a_graph():
    import torch
    from paper_1002_2184_amd import transform as T
    rng = np.random.default_rng(21)
    x2 = torch.tensor(rng.standard_normal((2, 300, 520)), dtype=torch.float32, device="cuda")
    x3 = torch.tensor(G.phantom_volume(rng, 40, 48, 200)[None], dtype=torch.float32, device="cuda")
    xb = x3.to(torch.bfloat16)
    y2, z2 = torch.empty_like(x2), torch.empty_like(x2)
    y3, z3 = torch.empty_like(x3), torch.empty_like(x3)
    yb = torch.empty_like(xb)
    g2 = torch.empty_like(x2)

    def work():
        T.fwd2d(x2, 8, out=y2)              # two passes through FP32 scratch
        T.inv2d(y2, 8, out=z2)
        T.fwd3d(x3, 7, out=y3)              # three passes through FP64 scratch
        T.inv3d(y3, 7, out=z3)
        T.fwd3d(xb, 5, out=yb)
        loss, _ = T.l1_grad2d(x2, 3, out=g2)   # tile loss partials in scratch
        return loss

    loss_eager = work().clone()
    torch.cuda.synchronize()
    outs = (y2, z2, y3, z3, yb, g2)
    eager = [t.clone() for t in outs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            loss_g = work()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        for t in outs:
            t.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()          # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for a, b in zip(outs, eager):
            assert torch.equal(a, b), f"replay {rep} differs from eager"
        assert torch.equal(loss_g, loss_eager), f"replay {rep}: loss differs"
