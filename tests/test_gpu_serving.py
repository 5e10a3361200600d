"""The request server: every result is the same alone and in the mix, plans
are re-bound and evicted under a tight device-memory budget, and a request
whose plan cannot fit the budget fails cleanly.  Requests on rectangular boxes
(the paper's rod and filament grids) equal their plans alone and the oracle."""

import numpy as np
import pytest

import workloads
from gpu_common import dev, host

pytestmark = pytest.mark.gpu


def _stream(n=24):
    reqs = workloads.serving_stream(n, n_lo=200, n_hi=4000)
    out = []
    for r in reqs:
        Y, F, T = workloads.request_inputs(r)
        out.append((r, dev(Y), dev(F), dev(T)))
    return out


def _alone(r, Y, F, T, precision):
    from paper_2310_12651_amd import Plan
    plan = Plan(r["N"], r["L"], r["a"], r["Sigma"], r["grid"], r["R_c"], support=r["M_G"],
                precision=precision)
    V, W = plan.mobility(Y, F, T)
    out = host(V), host(W)
    plan.close()
    return out


@pytest.mark.parametrize("precision,slots,tight", [(1, 4, False), (0, 3, False), (1, 2, True)],
                         ids=["fp32-4slots", "fp64-3slots", "fp32-tight-budget"])
def test_mix_equals_alone(precision, slots, tight):
    import torch
    from paper_2310_12651_amd.serving import Server
    items = _stream()
    # tight: room for the largest plan and a little more, so plans must be evicted
    budget = int(1.3 * max(12 * r["grid"] ** 3 for r, *_ in items)) + 4 * 10 ** 6 if tight else 0
    srv = Server(slots=slots, precision=precision, max_bytes=budget)
    outs, tickets = [], []
    for r, Y, F, T in items:
        V = torch.empty((r["N"], 3), dtype=torch.float64, device="cuda")
        W = torch.empty_like(V)
        outs.append((V, W))
        tickets.append(srv.submit(r["N"], r["L"], r["a"], r["Sigma"], r["grid"], r["R_c"], Y, F, T, V, W,
                                  support=r["M_G"]))
    for t in tickets:
        st, q, run = srv.wait(t)
        assert st == 0
    stats = srv.stats()
    srv.close()
    assert stats["completed"] == len(items) and stats["failed"] == 0
    if tight:
        assert stats["plans_evicted"] > 0
    for (r, Y, F, T), (V, W) in zip(items, outs):
        Va, Wa = _alone(r, Y, F, T, precision)
        assert np.array_equal(host(V), Va) and np.array_equal(host(W), Wa)


def test_request_too_large_for_budget_fails_cleanly():
    import torch
    from paper_2310_12651_amd.serving import Server
    r, Y, F, T = _stream(1)[0]
    srv = Server(slots=1, max_bytes=10 ** 6)
    V = torch.empty((r["N"], 3), dtype=torch.float64, device="cuda")
    t = srv.submit(r["N"], r["L"], r["a"], r["Sigma"], r["grid"], r["R_c"], Y, F, T, V, None,
                   support=r["M_G"])
    st, _, _ = srv.wait(t)
    assert st == -2   # FCM_ENOMEM
    srv.close()


def test_nonfinite_request_fails_alone():
    """A request with a NaN position completes with FCM_ENONFINITE; the other
    requests of the mix still equal their results alone, and a ticket that has
    been waited for cannot be waited for again."""
    import torch
    from paper_2310_12651_amd import FCM_EINVAL, FCM_ENONFINITE
    from paper_2310_12651_amd.serving import Server
    items = _stream(8)
    bad = 3
    srv = Server(slots=3, precision=1)
    outs, tickets = [], []
    for i, (r, Y, F, T) in enumerate(items):
        if i == bad:
            Y = Y.clone()
            Y[r["N"] // 2, 1] = float("nan")
        V = torch.empty((r["N"], 3), dtype=torch.float64, device="cuda")
        W = torch.empty_like(V)
        outs.append((V, W))
        tickets.append(srv.submit(r["N"], r["L"], r["a"], r["Sigma"], r["grid"], r["R_c"], Y, F, T, V, W,
                                  support=r["M_G"]))
    status = [srv.wait(t)[0] for t in tickets]
    assert srv.wait(tickets[0])[0] == FCM_EINVAL
    stats = srv.stats()
    srv.close()
    assert status[bad] == FCM_ENONFINITE
    assert all(s == 0 for i, s in enumerate(status) if i != bad), status
    assert stats["failed"] == 1 and stats["completed"] == len(items) - 1
    for i, ((r, Y, F, T), (V, W)) in enumerate(zip(items, outs)):
        if i == bad:
            continue
        Va, Wa = _alone(r, Y, F, T, 1)
        assert np.array_equal(host(V), Va) and np.array_equal(host(W), Wa)


def test_request_waits_for_callers_stream():
    """Inputs written by a kernel still queued on the caller's stream at
    submit are read only after it: the server waits on that stream."""
    import torch
    from paper_2310_12651_amd.serving import Server
    r, Y, F, T = _stream(1)[0]
    Va, Wa = _alone(r, Y, F, T, 1)
    srv = Server(slots=2, precision=1)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        torch.cuda._sleep(20_000_000)          # hold the stream (~10 ms) before the inputs exist
        F2 = F * 1.0
        T2 = T * 1.0
        V = torch.empty((r["N"], 3), dtype=torch.float64, device="cuda")
        W = torch.empty_like(V)
        t = srv.submit(r["N"], r["L"], r["a"], r["Sigma"], r["grid"], r["R_c"], Y, F2, T2, V, W,
                       support=r["M_G"])
    st, _, _ = srv.wait(t)
    srv.close()
    assert st == 0
    assert np.array_equal(host(V), Va) and np.array_equal(host(W), Wa)


# Requests on rectangular boxes (fcm_server_submit_box) beside cubic ones: the
# paper's rod and filament grids (Sec. 6.3), a thin box whose x and y sizes equal
# the cube's, and a second request on that thin box.
BOX_ITEMS = [
    dict(N=300, L=32.0, grid=64, Sigma=0.7, M_G=10, R_c=3.5),
    dict(N=200, L=(32.0, 32.0, 8.0), grid=(64, 64, 16), Sigma=0.7, M_G=10, R_c=3.5),
    dict(N=800, L=(512.0, 512.0, 8.0), grid=(512, 512, 8), Sigma=1.0, M_G=10, R_c=3.9),
    dict(N=600, L=(204.8, 204.8, 12.8), grid=(256, 256, 16), Sigma=0.8, M_G=10, R_c=4.4),
    dict(N=150, L=(32.0, 32.0, 8.0), grid=(64, 64, 16), Sigma=0.7, M_G=10, R_c=3.5),
]


def _box_inputs(k, c):
    rng = np.random.default_rng(9100 + k)
    L = np.broadcast_to(np.asarray(c["L"], dtype=float), (3,))
    Y = rng.uniform(-0.5, 1.5, size=(c["N"], 3)) * L
    return dev(Y), dev(rng.normal(size=(c["N"], 3))), dev(rng.normal(size=(c["N"], 3)))


@pytest.mark.parametrize("precision", [1, 0], ids=["fp32", "fp64"])
def test_box_requests_equal_alone(precision):
    """Served box and cube requests equal their plans run alone, bitwise; a
    cached plan is re-bound only to a request with the same three grid sizes
    (the thin box shares the cube's x size but gets its own plan)."""
    import torch
    from paper_2310_12651_amd import Plan
    from paper_2310_12651_amd.serving import Server
    srv = Server(slots=1, precision=precision)
    items, tickets = [], []
    for k, c in enumerate(BOX_ITEMS):
        Y, F, T = _box_inputs(k, c)
        V = torch.empty((c["N"], 3), dtype=torch.float64, device="cuda")
        W = torch.empty_like(V)
        items.append((c, Y, F, T, V, W))
        tickets.append(srv.submit(c["N"], c["L"], 1.0, c["Sigma"], c["grid"], c["R_c"], Y, F, T, V, W,
                                  support=c["M_G"]))
    status = [srv.wait(t)[0] for t in tickets]
    stats = srv.stats()
    srv.close()
    assert status == [0] * len(BOX_ITEMS), status
    assert stats["plans_built"] == 4 and stats["plans_rebound"] == 1, stats
    for c, Y, F, T, V, W in items:
        plan = Plan(c["N"], c["L"], 1.0, c["Sigma"], c["grid"], c["R_c"], support=c["M_G"],
                    precision=precision)
        Va, Wa = plan.mobility(Y, F, T)
        Va, Wa = host(Va), host(Wa)
        plan.close()
        assert np.array_equal(host(V), Va) and np.array_equal(host(W), Wa), c


def test_box_request_validation():
    """A box with unequal grid spacings, or a support longer than its x axis,
    is refused at submit (FCM_EINVAL), as fcm_plan_box refuses it."""
    import torch
    from paper_2310_12651_amd import FCM_EINVAL, FCMError
    from paper_2310_12651_amd.serving import Server
    c = BOX_ITEMS[1]
    Y, F, T = _box_inputs(1, c)
    V = torch.empty((c["N"], 3), dtype=torch.float64, device="cuda")
    srv = Server(slots=1)
    try:
        for L, grid, MG in [((32.0, 32.0, 9.0), (64, 64, 16), 10), ((4.0, 32.0, 8.0), (8, 64, 16), 10)]:
            with pytest.raises(FCMError) as e:
                srv.submit(c["N"], L, 1.0, 0.6, grid, 1.9, Y, F, T, V, None, support=MG)
            assert e.value.status == FCM_EINVAL
        assert srv.stats()["submitted"] == 0
    finally:
        srv.close()


@pytest.mark.parametrize("k", [2, 3], ids=["rods512x512x8", "fil256x256x16"])
def test_served_box_request_matches_oracle(k):
    """A served request on the paper's rod grid (support longer than the z
    axis) and on its filament grid against the oracle's mobility: FP64 1e-10
    and FP32 bulk 1e-5 normwise on V and Omega."""
    import torch
    from gpu_common import normwise
    from oracle import fastfcm as ff
    from paper_2310_12651_amd.serving import Server
    c = BOX_ITEMS[k]
    Y, F, T = _box_inputs(k, c)
    p = ff.Params(L=c["L"], M=c["grid"], a=1.0, Sigma=c["Sigma"], M_G=c["M_G"], R_c=c["R_c"])
    Vr, Wr = ff.mobility(p, host(Y), host(F), host(T))
    for precision, tol in [(0, 1e-10), (1, 1e-5)]:
        srv = Server(slots=2, precision=precision)
        V = torch.empty((c["N"], 3), dtype=torch.float64, device="cuda")
        W = torch.empty_like(V)
        t = srv.submit(c["N"], c["L"], 1.0, c["Sigma"], c["grid"], c["R_c"], Y, F, T, V, W, support=c["M_G"])
        st, _, _ = srv.wait(t)
        srv.close()
        assert st == 0
        ev, ew = normwise(host(V), Vr), normwise(host(W), Wr)
        assert ev < tol and ew < tol, (precision, ev, ew)
