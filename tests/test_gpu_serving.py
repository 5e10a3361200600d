"""The request server: every result is the same alone and in the mix, plans
are re-bound and evicted under a tight device-memory budget, and a request
whose plan cannot fit the budget fails cleanly."""

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
