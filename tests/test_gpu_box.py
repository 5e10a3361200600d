"""Rectangular periodic boxes on the GPU (fcm_plan_box) against the oracle.

Cases: a box long in x (48 x 18 x 18 points, M_G = 12: the four-lane FP32
interpolation of the row-major layout), a flat one (48 x 32 x 24, M_G = 16), and a thin one (64 x 64 x
16, M_G = 16, so spreading tiles are one point high), and a slab whose y period
equals the support (48 x 12 x 24, M_G = 12: every support covers all of y and the
spreading tiles are one row wide); the paper's rod grid 512 x 512 x 8 with
M_G = 10 and two more boxes whose support is longer than the z axis (M_G = 12
on 8 points, M_G = 16 on 12: the support wraps onto itself), and the paper's
filament grid 256 x 256 x 16, and a 288 x 288 x 16 box (register passes of 288
with a partial last block of x lines); every operator and the whole mobility, FP64 (1e-10 normwise) and FP32 bulk (1e-5).  Also the copy
identity of the oracle's box pins, on the GPU: copies of a cube along one axis
keep the cube's velocities.
"""

import math

import numpy as np
import pytest

import workloads
from gpu_common import dev, gpu_to_oracle_grid, host, normwise, oracle_to_gpu_grid
from oracle import fastfcm as ff

pytestmark = pytest.mark.gpu

A = 1.0
PREC = {"fp64": (0, 1e-10), "fp32": (1, 1e-5)}

BOXES = {
    "long48x18x18": dict(L=(32.0, 12.0, 12.0), M=(48, 18, 18), Sigma=0.75, M_G=12, R_c=5.0, N=30),
    "flat48x32x24": dict(L=(24.0, 16.0, 12.0), M=(48, 32, 24), Sigma=0.75, M_G=16, R_c=5.0, N=40),
    "thin64x64x16": dict(L=(32.0, 32.0, 8.0), M=(64, 64, 16), Sigma=0.7, M_G=16, R_c=3.5, N=40),
    "slab48x12x24": dict(L=(24.0, 6.0, 12.0), M=(48, 12, 24), Sigma=0.75, M_G=12, R_c=2.9, N=20),
    # supports longer than the z axis (they wrap onto themselves and their
    # coinciding points add): the paper's rod grid (Sec. 6.3, 512 x 512 x 8,
    # M_G = 10 at Sigma = dx), and M_G = 12 on 8 and M_G = 16 on 12 z points
    "rods512x512x8": dict(L=(512.0, 512.0, 8.0), M=(512, 512, 8), Sigma=1.0, M_G=10, R_c=3.9, N=2000),
    "fold64x64x8": dict(L=(32.0, 32.0, 4.0), M=(64, 64, 8), Sigma=0.6, M_G=12, R_c=1.95, N=40),
    "fold48x48x12": dict(L=(24.0, 24.0, 6.0), M=(48, 48, 12), Sigma=0.75, M_G=16, R_c=2.9, N=40),
    # the paper's filament grid (Sec. 6.3, 256 x 256 x 16)
    "fil256x256x16": dict(L=(204.8, 204.8, 12.8), M=(256, 256, 16), Sigma=0.8, M_G=10, R_c=4.4, N=1500),
    # register x and y passes of 288 (x lines staged through LDS, the last block
    # of 20 lines partly past the 3 x 288 x 16 lines) around the column z pass
    "sq288x288x16": dict(L=(144.0, 144.0, 8.0), M=(288, 288, 16), Sigma=0.6, M_G=10, R_c=3.0, N=60),
}


def _positions(N, L, rng):
    """Random sequential addition in a rectangular box (minimum image per axis)."""
    L = np.asarray(L)
    out = []
    while len(out) < N:
        p = rng.uniform(0.0, 1.0, size=3) * L
        ok = True
        for q in out:
            d = p - q
            d -= L * np.round(d / L)
            if d @ d < 4.0 * A * A:
                ok = False
                break
        if ok:
            out.append(p)
    return np.array(out)


@pytest.fixture(scope="module", params=sorted(BOXES))
def box(request):
    c = BOXES[request.param]
    rng = np.random.default_rng(sum(map(ord, request.param)))
    Y = _positions(c["N"], c["L"], rng)
    Y[:3] += np.array(c["L"]) * np.array([[1.0, 0.0, -1.0], [-2.0, 1.0, 0.0], [0.0, 0.0, 3.0]])
    F, T = rng.normal(size=(c["N"], 3)), rng.normal(size=(c["N"], 3))
    p = ff.Params(L=c["L"], M=c["M"], a=A, Sigma=c["Sigma"], M_G=c["M_G"], R_c=c["R_c"])
    f = ff.spread(p, Y, F, T)
    u = ff.stokes_solve(p, f)
    V, W = ff.mobility(p, Y, F, T)
    return dict(name=request.param, c=c, Y=Y, F=F, T=T, p=p, f=f, u=u, V=V, W=W)


def _plan(box, prec):
    from paper_2310_12651_amd import Plan
    c = box["c"]
    return Plan(c["N"], c["L"], A, c["Sigma"], c["M"], c["R_c"], support=c["M_G"],
                precision=PREC[prec][0])


def test_box_plan_properties(box):
    c = box["c"]
    plan = _plan(box, "fp64")
    info = plan.box_info()
    assert info["grid"] == tuple(c["M"]) and np.allclose(info["L"], c["L"])
    # m = max(int(L / R_c), 3) per axis (Sec. 4), at most 128 cells per axis
    assert info["cells"] == tuple(min(max(int(l / c["R_c"]), 3), 128) for l in c["L"])
    assert plan.new_grid().shape == (3, c["M"][2], c["M"][1], c["M"][0])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_box_spread_solve_mobility_match_oracle(box, prec):
    import torch
    plan = _plan(box, prec)
    tol = PREC[prec][1]
    Y, F, T = dev(box["Y"]), dev(box["F"]), dev(box["T"])
    g = plan.spread(Y, F, T)
    assert normwise(gpu_to_oracle_grid(host(g)), box["f"]) < tol
    gi = torch.as_tensor(oracle_to_gpu_grid(box["f"]), dtype=plan.grid_dtype, device="cuda")
    plan.solve(gi)
    assert normwise(gpu_to_oracle_grid(host(gi)), box["u"]) < tol
    V, W = plan.mobility(Y, F, T)
    assert normwise(host(V), box["V"]) < tol and normwise(host(W), box["W"]) < tol


@pytest.mark.parametrize("axis, k", [(0, 2), (2, 3)])
def test_box_copies_keep_the_cube_velocities(axis, k):
    from paper_2310_12651_amd import Plan
    rng = np.random.default_rng(7)
    L, M, N = 12.0, 24, 16
    Y = workloads.rsa_positions(N, L, A, rng)
    F, T = rng.normal(size=(N, 3)), rng.normal(size=(N, 3))
    cube = Plan(N, L, A, 0.8, M, 5.0, support=12, precision=0)
    Vc, Wc = cube.mobility(dev(Y), dev(F), dev(T))
    Vc, Wc = host(Vc), host(Wc)
    e = np.zeros(3)
    e[axis] = 1.0
    Lb, Mb = [L] * 3, [M] * 3
    Lb[axis] *= k
    Mb[axis] *= k
    Yb = np.concatenate([Y + j * L * e for j in range(k)])
    boxp = Plan(k * N, Lb, A, 0.8, Mb, 5.0, support=12, precision=0)
    Vb, Wb = boxp.mobility(dev(Yb), dev(np.tile(F, (k, 1))), dev(np.tile(T, (k, 1))))
    Vb, Wb = host(Vb), host(Wb)
    for j in range(k):
        sl = slice(j * N, (j + 1) * N)
        assert np.max(np.abs(Vb[sl] - Vc)) < 1e-12 * np.max(np.abs(Vc))
        assert np.max(np.abs(Wb[sl] - Wc)) < 1e-12 * np.max(np.abs(Wc))


def test_box_unequal_spacing_refused():
    from paper_2310_12651_amd import FCMError, Plan
    with pytest.raises(FCMError):
        Plan(10, (20.0, 20.0, 24.0), A, 1.0, (32, 32, 32), 4.0)
