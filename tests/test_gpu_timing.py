"""Stage timing through the C ABI (fcm_plan_set_timing / fcm_plan_stage_times):
every stage timed, one stage timed (the others read zero), invalid modes
refused, and timing leaves the results bitwise unchanged."""

import numpy as np
import pytest

import workloads
from gpu_common import dev, host, make_plan

pytestmark = pytest.mark.gpu


def test_stage_timing_modes():
    from paper_2310_12651_amd import STAGES, library
    w = workloads.workload(0)
    plan = make_plan(w, 1)
    Y, F, T = dev(w["Y"]), dev(w["F"]), dev(w["T"])
    V0, W0 = plan.mobility(Y, F, T)
    V0, W0 = host(V0), host(W0)

    plan.set_timing(True)
    for _ in range(3):
        V, W = plan.mobility(Y, F, T)
    st, n = plan.stage_times()
    assert n == 3
    # the fused x-y pass leaves the y stages empty only where it runs; every
    # other stage, the pair correction included, takes time
    for s in ("sort", "spread", "fft_x_fwd", "fft_z_solve", "fft_x_inv", "interp", "pair"):
        assert st[s] > 0.0, s
    assert np.array_equal(host(V), V0) and np.array_equal(host(W), W0)

    for one in ("spread", "interp", "pair"):
        plan.set_timing(True, stage=one)
        for _ in range(2):
            V, W = plan.mobility(Y, F, T)
        st, n = plan.stage_times()
        assert n == 2 and st[one] > 0.0
        assert all(st[s] == 0.0 for s in STAGES if s != one), (one, st)
        assert np.array_equal(host(V), V0) and np.array_equal(host(W), W0)

    plan.set_timing(False)
    lib = library()
    for bad in (-1, 2 + len(STAGES)):
        assert lib.fcm_plan_set_timing(plan.handle, bad) != 0
