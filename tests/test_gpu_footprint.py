"""The exact plan footprint (fcm_plan_footprint_box) against the device
memory a plan actually takes (hipMemGetInfo before and after fcm_plan_box)."""

import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,L,Sigma,grid,rc,prec", [
    (100_000, 161.2, 0.6297, 256, 3.4633, 1),
    (100_000, 161.2, 0.6297, 256, 3.4633, 0),
    (10_000, 161.2, 1.2594, 128, 6.93, 1),
    (20_000, (96.0, 48.0, 36.0), 1.0, (96, 48, 36), 5.5, 1),
], ids=["dense-fp32", "dense-fp64", "dilute-fp32", "box-fp32"])
def test_footprint_equals_allocation(N, L, Sigma, grid, rc, prec):
    import torch
    from paper_2310_12651_amd import Plan, _lib
    o = _lib.fcm_options_default()
    o.precision = prec
    fp = _lib.fcm_plan_footprint_box(N, L, 1.0, Sigma, grid, rc, o)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    plan = Plan(N, L, 1.0, Sigma, grid, rc, precision=prec)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    plan.close()
    drop = free0 - free1
    print(f"footprint {fp} drop {drop} diff {drop - fp}", flush=True)
    # 17 device buffers, each rounded up to the allocator's granularity, plus
    # the plan's side stream and events
    assert fp <= drop <= fp + 17 * (2 << 20) + (8 << 20)
