"""Brownian velocities on the GPU (fcm_brownian) against the oracle, on the
same noise: the grid part (fluctuating FCM through the square-root solve) and
the pair part (Lanczos square root of the VF correction matrix) of the
positive splitting (Sec. 3.3, Sec. 7)."""

import math

import numpy as np
import pytest

import workloads
from gpu_common import dev, host, make_plan, normwise, oracle_params, oracle_to_gpu_grid
from oracle import brownian as br
from oracle import fastfcm as ff

pytestmark = pytest.mark.gpu

A = 1.0
SIG = A / math.sqrt(math.pi)
SIGD = A / (6.0 * math.sqrt(math.pi)) ** (1.0 / 3.0)


def _noise(p, N, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(3,) + tuple(p.Mv)), rng.normal(size=(N, 3))


def _grid_tensor(plan, xi):
    import torch
    return torch.as_tensor(oracle_to_gpu_grid(xi), dtype=plan.grid_dtype, device="cuda").contiguous()


@pytest.mark.parametrize("prec, tol", [("fp64", 1e-9), ("fp32", 1e-5)])
def test_brownian_matches_oracle(prec, tol):
    w = workloads.workload(0)
    p = oracle_params(w)
    xg, xp = _noise(p, w["N"], 5)
    kT = 1.3
    plan = make_plan(w, 0 if prec == "fp64" else 1)
    V, it = plan.brownian(dev(w["Y"]), _grid_tensor(plan, xg), dev(xp), kT, tol=1e-12)
    Vg = br.brownian_grid(p, w["Y"], xg, kT)
    Vp = br.brownian_pair(p, w["Y"], xp, kT)
    assert 1 < it < 48
    assert normwise(host(V), Vg + Vp) < tol
    # the pair part alone (kT enters both parts as sqrt(2 kT)): zero grid noise
    V0, _ = plan.brownian(dev(w["Y"]), _grid_tensor(plan, 0.0 * xg), dev(xp), kT, tol=1e-12)
    assert normwise(host(V0), Vp) < 1e-9


def test_brownian_standard_fcm_has_no_pair_part():
    w = dict(workloads.workload(0))
    w.update(Sigma=SIG, R_c=0.0, M_G=14, grid=48)
    p = oracle_params(w, Sigma_D=SIGD)
    xg, _ = _noise(p, w["N"], 8)
    plan = make_plan(w, 0, sigma_D_grid=SIGD)
    V, it = plan.brownian(dev(w["Y"]), _grid_tensor(plan, xg), None, 0.5)
    assert it == 0
    assert normwise(host(V), br.brownian_grid(p, w["Y"], xg, 0.5)) < 1e-10


def test_brownian_in_a_rectangular_box():
    from paper_2310_12651_amd import Plan
    rng = np.random.default_rng(12)
    L, M, N = (24.0, 16.0, 12.0), (48, 32, 24), 25
    Y = np.stack([rng.uniform(0, l, size=N) for l in L], 1)
    p = ff.Params(L=L, M=M, a=A, Sigma=0.75, M_G=14, R_c=5.9)
    xg, xp = _noise(p, N, 13)
    plan = Plan(N, L, A, 0.75, M, 5.9, support=14, precision=0)
    V, _ = plan.brownian(dev(Y), _grid_tensor(plan, xg), dev(xp), 2.0, tol=1e-12)
    assert normwise(host(V), br.brownian(p, Y, xg, xp, 2.0)) < 1e-9


@pytest.mark.parametrize("M", [(96,) * 3, (108,) * 3, (128,) * 3, (144,) * 3, (162,) * 3, (192,) * 3,
                               (216,) * 3, (288,) * 3, (324,) * 3, (384,) * 3, (64, 64, 16), (32, 32, 8)],
                         ids=lambda M: "x".join(map(str, M)))
def test_brownian_grid_part_fp32_register_z_passes(M):
    """The grid part in FP32 on grids whose z pass takes one component per
    thread group (96^3, 108^3, 144^3, 192^3, 216^3 and 288^3 with the split
    line; 128^3, 162^3, 324^3 and 384^3 with the four-step of the y pass) or one
    column per thread (square boxes with 16 and 8 z points), where the
    projection takes the square root of the Stokes
    multiplier: standard FCM (no pair part) against the oracle on the same
    noise.  The oracle's FFT runs on scipy threads at these sizes."""
    import os

    from paper_2310_12651_amd import FCM_FP32_BULK, Plan
    N, kT = 40, 0.7
    L = tuple(m * SIG for m in M)
    rng = np.random.default_rng(sum(M))
    Y = rng.uniform(0.0, 1.0, size=(N, 3)) * np.array(L)
    p = ff.Params(L=L, M=M, a=A, Sigma=SIG, M_G=10, R_c=0.0, Sigma_D=SIGD)
    xg = rng.normal(size=(3,) + tuple(M))
    plan = Plan(N, L, A, SIG, M, 0.0, support=10, precision=FCM_FP32_BULK, sigma_D_grid=SIGD)
    try:
        V, it = plan.brownian(dev(Y), _grid_tensor(plan, xg), None, kT)
        Vh = host(V)
    finally:
        plan.close()
    assert it == 0
    ref = br.brownian_grid(p, Y, xg, kT, workers=min(16, os.cpu_count() or 1))
    assert normwise(Vh, ref) < 1e-5, (M, normwise(Vh, ref))
