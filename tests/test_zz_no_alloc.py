"""The allocation-free entry point fcm_mobility_static (called through the C
ABI) against fcm_mobility on a plan with the same arguments: two calls in a
row, the second smaller (the static scratch keeps the first call's contents),
in FP32 bulk and FP64; and a problem too large for the scratch is refused."""

import ctypes

import numpy as np
import pytest

import workloads
from gpu_common import dev, host, make_plan, normwise

pytestmark = pytest.mark.gpu


def _static(w, precision):
    import torch
    from paper_2310_12651_amd import _lib
    lib = _lib.library()
    o = _lib.fcm_options_default()
    o.support, o.precision = int(w["M_G"]), int(precision)
    N = w["N"]
    Y, F, T = dev(w["Y"]), dev(w["F"]), dev(w["T"])
    V = torch.empty((N, 3), dtype=torch.float64, device="cuda")
    W = torch.empty_like(V)
    st = lib.fcm_mobility_static(N, w["L"], w["a"], w["Sigma"], w["grid"], w["R_c"], ctypes.byref(o),
                                 ctypes.c_void_p(Y.data_ptr()), ctypes.c_void_p(F.data_ptr()),
                                 ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(V.data_ptr()),
                                 ctypes.c_void_p(W.data_ptr()),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, host(V), host(W)


def _planned(w, precision):
    plan = make_plan(w, precision)
    V, W = plan.mobility(dev(w["Y"]), dev(w["F"]), dev(w["T"]))
    out = host(V), host(W)
    plan.close()
    return out


@pytest.mark.parametrize("precision,tol", [(1, 1e-5), (0, 1e-10)], ids=["fp32", "fp64"])
def test_static_equals_planned_twice_second_smaller(precision, tol):
    for w in (workloads.workload(1), workloads.workload(0)):     # 10^4 on 128^3, then 64 on 32^3
        print(f"static {w['name']} precision={precision}", flush=True)
        st, V, W = _static(w, precision)
        assert st == 0
        Vp, Wp = _planned(w, precision)
        assert normwise(V, Vp) < tol and normwise(W, Wp) < tol, (normwise(V, Vp), normwise(W, Wp))


def test_static_refuses_problem_beyond_scratch():
    from paper_2310_12651_amd import FCM_ESCRATCH
    w = workloads.workload(2)          # 10^5 particles on 256^3: ~330 MB of buffers
    st, _, _ = _static(w, 1)
    assert st == FCM_ESCRATCH
