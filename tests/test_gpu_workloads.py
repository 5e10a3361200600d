"""Parity at the full sizes of the workloads, in the launch configuration the
benchmark times (default plans, FP32 bulk and FP64).

Dilute N = 10^4 (128^3): every particle against the oracle.  Dense N = 10^5
(256^3) and rods N = 60 000 (192^3): the oracle spreads all particles, solves
on the full grid and evaluates interpolation and pair correction on a seeded
subsample; the GPU values of those particles must match.  Bars: FP64 1e-10,
FP32 bulk 1e-5 normwise (and the paper's mean error measure < 1e-4).
"""

import numpy as np
import pytest

import workloads
from gpu_common import dev, eps_mean, host, make_plan, normwise, oracle_params
from oracle import fastfcm as ff

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[1, 2, 3], ids=["dilute", "dense", "rods"])
def full(request):
    w = workloads.workload(request.param)
    p = oracle_params(w)
    rng = np.random.default_rng(77)
    sub = None if request.param == 1 else np.sort(rng.choice(w["N"], size=600, replace=False))
    V, W = ff.mobility(p, w["Y"], w["F"], w["T"], targets=sub)
    return dict(w=w, sub=sub, V=V, W=W)


@pytest.mark.parametrize("prec,tol", [(0, 1e-10), (1, 1e-5)], ids=["fp64", "fp32"])
def test_full_size_parity(full, prec, tol):
    w, sub = full["w"], full["sub"]
    plan = make_plan(w, prec)
    V, W = plan.mobility(dev(w["Y"]), dev(w["F"]), dev(w["T"]))
    Vh, Wh = host(V), host(W)
    if sub is not None:
        Vh, Wh = Vh[sub], Wh[sub]
    print(f"{w['name']} prec={prec} relV={normwise(Vh, full['V']):.2e} relW={normwise(Wh, full['W']):.2e}")
    assert normwise(Vh, full["V"]) < tol
    if np.abs(full["W"]).max() > 0:
        assert normwise(Wh, full["W"]) < tol
    assert eps_mean(Vh, full["V"]) < 1e-4
    plan.close()


def test_fp32_kahan_modes_agree(full):
    """Plain, Kahan-compensated and FP64-accumulated FP32 spreading agree with
    the oracle to the FP32 bar."""
    w, sub = full["w"], full["sub"]
    for mode in (0, 1, 2):
        plan = make_plan(w, 1, kahan=mode)
        V, _ = plan.mobility(dev(w["Y"]), dev(w["F"]), dev(w["T"]))
        Vh = host(V)
        if sub is not None:
            Vh = Vh[sub]
        assert normwise(Vh, full["V"]) < 1e-5, mode
        plan.close()
