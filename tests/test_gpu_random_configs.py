"""Parity of the whole mobility with the FP64 oracle on seeded random
configurations: a sweep beside the hand-picked cases of test_gpu_parity.py.

Each case draws a grid (cubic among the register and LDS FFT sizes, or a
rectangular box with one grid spacing), a spacing dx and Sigma / dx in
[0.9, 1.6] (never below sigma), a support M_G in [6, 16], sometimes a wider
torque width Sigma_D and eta != 1, a cutoff R_c in [1.5, 0.45 L_min], N
log-uniform in [1, 400] with positions uniform over three box lengths (so
they wrap; centres may overlap, where the pair blocks take their r -> 0
limits), and torques on or off.  Bars as in test_gpu_parity.py: FP64 1e-10
and FP32 1e-5 normwise on V; Omega the same in FP64 where it does not
cancel, else (and in FP32) against max(|Omega|, |V| / a).
"""

import math
import zlib

import numpy as np
import pytest

from gpu_common import dev, host, normwise
from oracle import cgrid
from oracle import fastfcm as ff

pytestmark = pytest.mark.gpu

A = 1.0
SIGMA = A / math.sqrt(math.pi)
CUBES = [24, 32, 36, 48, 54, 64, 72, 96, 108, 128]
BOXES = [(48, 32, 24), (64, 64, 16), (36, 48, 24), (32, 32, 8), (96, 64, 32), (54, 36, 18)]
NCASES = 24


def _draw(k):
    rng = np.random.default_rng(zlib.crc32(b"random-configs-%d" % k))
    if rng.uniform() < 0.7:
        M = (int(rng.choice(CUBES)),) * 3
    else:
        M = tuple(int(m) for m in BOXES[int(rng.integers(len(BOXES)))])
    dx = float(rng.uniform(0.4, 0.8))
    L = tuple(m * dx for m in M)
    Sigma = max(1.02 * SIGMA, float(rng.uniform(0.9, 1.6)) * dx)
    SD = None
    if rng.uniform() < 0.3:
        SD = Sigma * float(rng.uniform(1.05, 1.5))
    mg_max = min(16, M[0], M[1])
    if M[2] not in (8, 12, 16):
        mg_max = min(mg_max, M[2])
    MG = int(rng.integers(6, mg_max + 1))
    eta = float(rng.choice([1.0, 0.7, 2.0]))
    Rc = float(rng.uniform(1.5, 0.45 * min(L)))
    N = int(round(math.exp(rng.uniform(0.0, math.log(400.0)))))
    Y = rng.uniform(-1.0, 2.0, size=(N, 3)) * np.array(L)
    F = rng.normal(size=(N, 3))
    T = rng.normal(size=(N, 3)) if rng.uniform() < 0.75 else None
    return dict(k=k, M=M, L=L, Sigma=Sigma, SD=SD, MG=MG, eta=eta, Rc=Rc, N=N, Y=Y, F=F, T=T)


def _oracle(c):
    p = ff.Params(L=c["L"], M=c["M"], a=A, Sigma=c["Sigma"], M_G=c["MG"], R_c=c["Rc"], eta=c["eta"],
                  Sigma_D=c["SD"])
    f = cgrid.spread(p, c["Y"], c["F"], c["T"])
    u = ff.stokes_solve(p, f)
    V, W = ff.interp(p, c["Y"], u)
    dV, dW = ff.pair_correction(p, c["Y"], c["F"], c["T"])
    return V + dV, W + dW


@pytest.fixture(scope="module", params=range(NCASES))
def case(request):
    c = _draw(request.param)
    c["Vr"], c["Wr"] = _oracle(c)
    return c


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_random_config_matches_oracle(case, prec):
    from paper_2310_12651_amd import FCM_FP32_BULK, FCM_FP64, Plan
    c = case
    plan = Plan(c["N"], c["L"], A, c["Sigma"], c["M"], c["Rc"], eta=c["eta"], support=c["MG"],
                precision=FCM_FP64 if prec == "fp64" else FCM_FP32_BULK, sigma_D_grid=c["SD"] or 0.0)
    try:
        V, W = plan.mobility(dev(c["Y"]), dev(c["F"]), None if c["T"] is None else dev(c["T"]))
        Vh, Wh = host(V), host(W)
        assert plan.last_error() == 0
    finally:
        plan.close()
    tol = 1e-10 if prec == "fp64" else 1e-5
    tag = {k: c[k] for k in ("k", "M", "Sigma", "SD", "MG", "eta", "Rc", "N")}
    assert normwise(Vh, c["Vr"]) < tol, (tag, normwise(Vh, c["Vr"]))
    # Omega as in test_gpu_parity.py: plain normwise in FP64 where Omega does
    # not cancel; otherwise, and always in FP32 (single-precision sums cancel
    # to ~1e-7 of it), against max(|Omega|, |V| / a)
    ang = np.linalg.norm(c["Vr"]) / A
    if prec == "fp64" and np.linalg.norm(c["Wr"]) > 1e-6 * ang:
        assert normwise(Wh, c["Wr"]) < tol, (tag, normwise(Wh, c["Wr"]))
    else:
        scale = max(np.linalg.norm(c["Wr"]), ang)
        assert np.linalg.norm(Wh - c["Wr"]) < tol * scale, (tag, np.linalg.norm(Wh - c["Wr"]) / scale)


def test_random_configs_cover_the_space():
    """The draws include boxes, a separate torque width, no torques, eta != 1,
    N = 1-3 and N > 100, and supports from small to 16."""
    cs = [_draw(k) for k in range(NCASES)]
    assert any(len(set(c["M"])) > 1 for c in cs)
    assert any(c["SD"] is not None for c in cs)
    assert any(c["T"] is None for c in cs)
    assert any(c["eta"] != 1.0 for c in cs)
    assert any(c["N"] <= 3 for c in cs) and any(c["N"] > 100 for c in cs)
    assert min(c["MG"] for c in cs) <= 8 and max(c["MG"] for c in cs) >= 14
