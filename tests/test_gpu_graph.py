"""The mobility captured into a HIP graph and replayed.

fcm_mobility is stream-ordered, allocates nothing and makes no host
synchronisation, so a caller may capture it (here through torch's stream
capture): the graph holds the sort, the spread, the FFT passes, the
interpolation and the pair correction, whose side stream joins the capture
through the plan's fork and join events.  Each replay, with new positions,
forces and torques written into the captured input buffers between replays (and
an eager call of the same plan, a host synchronisation, between them), must
equal the eager call on the same inputs bitwise.  Also fcm_mobility_repeat.
The graphs refer to the plan's buffers, side stream and events, so they are
destroyed before the plan is.
"""

import numpy as np
import pytest

from gpu_common import host

pytestmark = pytest.mark.gpu

CASES = {
    # pair correction on the side stream; M_G = 10 on a tiled 64^3 grid
    "cube64": dict(N=700, L=32.0, grid=64, Sigma=0.75, M_G=10, R_c=4.0),
    # row-major 54^3 grid (LDS FFT passes), FP64 and FP32
    "cube54": dict(N=300, L=27.0, grid=54, Sigma=0.8, M_G=12, R_c=5.0),
    # no pair correction (R_c = 0): no side stream in the graph
    "nopair48": dict(N=200, L=24.0, grid=48, Sigma=0.7, M_G=8, R_c=0.0),
}


def _inputs(c, k):
    rng = np.random.default_rng(4400 + k)
    return (rng.uniform(-0.5, 1.5, size=(c["N"], 3)) * c["L"], rng.normal(size=(c["N"], 3)),
            rng.normal(size=(c["N"], 3)))


@pytest.mark.parametrize("precision", [1, 0], ids=["fp32", "fp64"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_captured_mobility_equals_eager(name, precision):
    import torch
    from paper_2310_12651_amd import Plan
    c = CASES[name]
    plan = Plan(c["N"], c["L"], 1.0, c["Sigma"], c["grid"], c["R_c"], support=c["M_G"], precision=precision)
    graphs = []
    try:
        N = c["N"]
        Y, F, T = (torch.empty((N, 3), dtype=torch.float64, device="cuda") for _ in range(3))
        V, W = torch.empty_like(Y), torch.empty_like(Y)
        for t, x in zip((Y, F, T), _inputs(c, 0)):
            t.copy_(torch.as_tensor(x))
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            plan.mobility(Y, F, T, V, W)          # eager warm-up on the capture stream
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        graphs.append(g)
        with torch.cuda.graph(g, stream=s):
            plan.mobility(Y, F, T, V, W)
        assert plan.last_error() == 0
        for k in range(1, 5):
            for t, x in zip((Y, F, T), _inputs(c, k)):
                t.copy_(torch.as_tensor(x))
            Ve, We = plan.mobility(Y, F, T)       # eager, into fresh outputs
            Ve, We = host(Ve), host(We)
            V.fill_(float("nan"))
            W.fill_(float("nan"))
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(host(V), Ve) and np.array_equal(host(W), We), (name, k)
        # the repeated mobility (new forces at the last positions) captured too
        g2 = torch.cuda.CUDAGraph()
        graphs.append(g2)
        plan.mobility(Y, F, T, V, W)
        torch.cuda.synchronize()
        with torch.cuda.graph(g2, stream=s):
            plan.mobility_repeat(F, T, V, W)
        for k in range(5, 8):
            _, Fk, Tk = _inputs(c, k)
            F.copy_(torch.as_tensor(Fk))
            T.copy_(torch.as_tensor(Tk))
            Ve, We = plan.mobility_repeat(F, T)
            Ve, We = host(Ve), host(We)
            V.fill_(float("nan"))
            W.fill_(float("nan"))
            g2.replay()
            torch.cuda.synchronize()
            assert np.array_equal(host(V), Ve) and np.array_equal(host(W), We), (name, k)
        assert plan.last_error() == 0
    finally:
        # every graph goes before the plan whose buffers, stream and events it uses
        torch.cuda.synchronize()
        for gr in graphs:
            gr.reset()
        g = g2 = None
        graphs.clear()
        plan.close()
