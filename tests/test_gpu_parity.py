"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: FP64 plans within 1e-10 normwise relative (elementwise checks too);
FP32-bulk plans within 1e-5 normwise relative.  Each operator of the path is
checked on its own (spread, Stokes solve, interpolation, correction) and the
whole mobility end to end, on grids that span several tiles and ragged
tilings (grid sizes with factors of 3, odd supports), wrapped positions,
torques on and off, a separate torque width, standard FCM, a crowded box
(R_c near L/2, many neighbours per particle; with a separate torque width,
about 300 of them), a dense cluster (spreading tiles with ~1500 candidates),
supports M_G = 15 and 16 on
grids whose FP32 mobility runs in the tiled layout (the packed interpolation's
widest form), N = 1, a lattice of grid points given one to six periods
away (the wrap must land exactly where the oracle's does, or a support start
moves by one point), positions up to 1e9 box lengths away, coincident
centres, and pairs within two ulps of the cut-off.
"""

import math
import zlib

import numpy as np
import pytest

import workloads
from gpu_common import (dev, eps_mean, gpu_to_oracle_grid, host, make_plan, maxrel, normwise,
                        oracle_params, oracle_to_gpu_grid)
from oracle import fastfcm as ff

pytestmark = pytest.mark.gpu

A = 1.0
SIG = A / math.sqrt(math.pi)


def _case(name):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    if name == "small":
        return workloads.workload(0), None
    if name == "ragged54":
        L, N = 30.0, 37
        Y = workloads.rsa_positions(N, L, A, rng)
        Y[:5] += L * np.array([[-1.0], [1.0], [2.0], [-3.0], [0.0]])   # outside the box
        w = dict(N=N, L=L, a=A, eta=1.0, grid=54, Sigma=1.3 * L / 54, M_G=9, R_c=7.0,
                 Y=Y, F=rng.normal(size=(N, 3)), T=rng.normal(size=(N, 3)))
        return w, None
    if name == "wideTorque36":
        L, N = 24.0, 50
        Y = workloads.rsa_positions(N, L, A, rng)
        w = dict(N=N, L=L, a=A, eta=0.7, grid=36, Sigma=1.1, M_G=16, R_c=8.0,
                 Y=Y, F=rng.normal(size=(N, 3)), T=rng.normal(size=(N, 3)))
        return w, 1.5
    if name == "standard48":
        L, N = 20.0, 40
        Y = workloads.rsa_positions(N, L, A, rng)
        w = dict(N=N, L=L, a=A, eta=1.0, grid=48, Sigma=SIG, M_G=14, R_c=0.0,
                 Y=Y, F=rng.normal(size=(N, 3)), T=rng.normal(size=(N, 3)))
        return w, None
    if name == "crowded":
        # R_c near L/2: ~130 neighbours per particle, more than the pair scan
        # records per (particle, z layer), so the evaluation's rescan path runs
        L, N = 30.0, 300
        Y = workloads.rsa_positions(N, L, A, rng)
        w = dict(N=N, L=L, a=A, eta=1.0, grid=36, Sigma=1.2, M_G=12, R_c=14.0,
                 Y=Y, F=rng.normal(size=(N, 3)), T=rng.normal(size=(N, 3)))
        return w, None
    if name == "crowded700":
        # ~300 neighbours per particle, ~100 per z layer of the 3 x 3 x 3
        # cells: twice what the scan records, so the evaluation runs several
        # refill passes (each queues up to 12 more hits of a layer)
        L, N = 30.0, 700
        Y = workloads.rsa_positions(N, L, A, rng)
        w = dict(N=N, L=L, a=A, eta=1.0, grid=36, Sigma=1.2, M_G=12, R_c=14.0,
                 Y=Y, F=rng.normal(size=(N, 3)), T=rng.normal(size=(N, 3)))
        return w, 1.4
    if name == "cluster64":
        # 1500 spheres packed in a 6^3 corner region (centres may overlap)
        # and 200 spread over the box: the spreading tiles over the cluster
        # hold ~1500 candidates each (a few tens elsewhere), and the pair
        # search there finds ~800 neighbours a particle (refill passes)
        L, N = 32.0, 1700
        Y = np.concatenate([12.0 + rng.uniform(0.0, 6.0, size=(1500, 3)),
                            rng.uniform(0.0, L, size=(200, 3))])
        w = dict(N=N, L=L, a=A, eta=1.0, grid=64, Sigma=0.75, M_G=12, R_c=3.0,
                 Y=Y, F=rng.normal(size=(N, 3)), T=rng.normal(size=(N, 3)))
        return w, None
    if name == "tiny16":
        # grid narrower than support + tile (16 < 12 + 8): supports meet a
        # spreading tile on both sides of the periodic seam
        L, N = 14.0, 12
        Y = workloads.rsa_positions(N, L, A, rng)
        w = dict(N=N, L=L, a=A, eta=1.0, grid=16, Sigma=1.2 * L / 16, M_G=12, R_c=5.0,
                 Y=Y, F=rng.normal(size=(N, 3)), T=rng.normal(size=(N, 3)))
        return w, None
    if name == "support16":
        # M_G = 16 at Sigma/dx = 1.5 (the serving stream's support) on a grid
        # whose FP32 mobility runs in the tiled layout: packed interpolation
        # with three quads per lane, two particles per wavefront; N odd, so the
        # last wavefront holds one particle
        L, N = 32.0, 45
        Y = workloads.rsa_positions(N, L, A, rng)
        Y[:4] += L * np.array([[1.0], [-1.0], [-2.0], [3.0]])
        w = dict(N=N, L=L, a=A, eta=1.0, grid=64, Sigma=1.5 * L / 64, M_G=16, R_c=4.2,
                 Y=Y, F=rng.normal(size=(N, 3)), T=rng.normal(size=(N, 3)))
        return w, None
    if name == "support15":
        L, N = 36.0, 29
        Y = workloads.rsa_positions(N, L, A, rng)
        w = dict(N=N, L=L, a=A, eta=1.0, grid=72, Sigma=1.4 * L / 72, M_G=15, R_c=4.0,
                 Y=Y, F=rng.normal(size=(N, 3)), T=rng.normal(size=(N, 3)))
        return w, None
    if name == "single64":
        # one particle on a tiled 64^3 grid with M_G = 16: the packed
        # interpolation with one live slot and the fused x-y FFT passes
        w = dict(N=1, L=32.0, a=A, eta=1.0, grid=64, Sigma=0.75, M_G=16, R_c=4.2,
                 Y=np.array([[31.9, 0.3, 17.02]]), F=np.array([[0.4, 1.0, -0.7]]),
                 T=np.array([[-0.2, 0.5, 0.9]]))
        return w, None
    if name == "support14":
        # M_G = 14 on a tiled 96^3 grid (fused x-y passes with three-quad rows)
        L, N = 48.0, 33
        Y = workloads.rsa_positions(N, L, A, rng)
        w = dict(N=N, L=L, a=A, eta=1.0, grid=96, Sigma=1.4 * L / 96, M_G=14, R_c=3.9,
                 Y=Y, F=rng.normal(size=(N, 3)), T=rng.normal(size=(N, 3)))
        return w, None
    if name == "single":
        w = dict(N=1, L=16.0, a=A, eta=1.0, grid=24, Sigma=2 * SIG, M_G=12, R_c=7.5,
                 Y=np.array([[15.9, 0.01, 8.0]]), F=np.array([[1.0, -2.0, 0.5]]),
                 T=np.array([[0.3, 0.2, -1.0]]))
        return w, None
    raise KeyError(name)


CASES = ["small", "ragged54", "wideTorque36", "standard48", "crowded", "crowded700", "cluster64", "tiny16",
         "support16",
         "support15", "support14", "single64", "single"]
PREC = {"fp64": (0, 1e-10), "fp32": (1, 1e-5)}


@pytest.fixture(scope="module", params=CASES)
def case(request):
    w, SD = _case(request.param)
    p = oracle_params(w, Sigma_D=SD)
    f = ff.spread(p, w["Y"], w["F"], w["T"])
    u = ff.stokes_solve(p, f)
    V, W = ff.interp(p, w["Y"], u)
    dV, dW = ff.pair_correction(p, w["Y"], w["F"], w["T"])
    return dict(name=request.param, w=w, SD=SD, p=p, f=f, u=u, Vg=V, Wg=W, dV=dV, dW=dW,
                V=V + dV, W=W + dW)


def _plan(c, prec):
    return make_plan(c["w"], PREC[prec][0], sigma_D_grid=c["SD"] or 0.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_spread_matches_oracle(case, prec):
    w = case["w"]
    plan = _plan(case, prec)
    g = plan.spread(dev(w["Y"]), dev(w["F"]), dev(w["T"]))
    got = gpu_to_oracle_grid(host(g).astype(np.float64))
    tol = PREC[prec][1]
    assert maxrel(got, case["f"]) < tol, (case["name"], prec, maxrel(got, case["f"]))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_solve_matches_oracle(case, prec):
    import torch
    plan = _plan(case, prec)
    g = torch.as_tensor(oracle_to_gpu_grid(case["f"]), device="cuda").to(plan.grid_dtype).contiguous()
    plan.solve(g)
    got = gpu_to_oracle_grid(host(g).astype(np.float64))
    assert normwise(got, case["u"]) < PREC[prec][1], (case["name"], prec, normwise(got, case["u"]))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_interp_matches_oracle(case, prec):
    import torch
    w = case["w"]
    plan = _plan(case, prec)
    g = torch.as_tensor(oracle_to_gpu_grid(case["u"]), device="cuda").to(plan.grid_dtype).contiguous()
    V, W = plan.interp(dev(w["Y"]), g)
    tol = PREC[prec][1]
    assert normwise(host(V), case["Vg"]) < tol
    assert normwise(host(W), case["Wg"]) < tol


def test_correct_matches_oracle(case):
    w = case["w"]
    plan = _plan(case, "fp64")
    import torch
    V = torch.zeros((w["N"], 3), dtype=torch.float64, device="cuda")
    W = torch.zeros_like(V)
    plan.correct(dev(w["Y"]), dev(w["F"]), dev(w["T"]), V, W)
    for got, ref in ((host(V), case["dV"]), (host(W), case["dW"])):
        scale = max(np.abs(ref).max(), 1e-300)
        assert np.abs(got - ref).max() < 1e-12 * scale + 1e-16, (case["name"], np.abs(got - ref).max(), scale)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_mobility_matches_oracle(case, prec):
    w = case["w"]
    plan = _plan(case, prec)
    V, W = plan.mobility(dev(w["Y"]), dev(w["F"]), dev(w["T"]))
    tol = PREC[prec][1]
    Vh, Wh = host(V), host(W)
    assert normwise(Vh, case["V"]) < tol, (case["name"], prec, normwise(Vh, case["V"]))
    assert normwise(Wh, case["W"]) < tol, (case["name"], prec, normwise(Wh, case["W"]))
    if prec == "fp64":
        assert maxrel(Vh, case["V"]) < 1e-9 and maxrel(Wh, case["W"]) < 1e-9
    assert plan.last_error() == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_optional_torque_and_omega(case, prec):
    """T = NULL means zero torques; Omega = NULL skips angular velocities.

    FP64 meets the plain normwise bar on Omega wherever Omega does not cancel.
    A lone particle's Omega from its force vanishes by symmetry up to the
    grid's residual (about 1e-9 of the angular scale |V| / a on 64^3): there the
    rounding of its O(|V| / a) sums bounds the error, in FP64 as in FP32, so the
    error is measured against that scale.  In FP32 the same scale is taken in
    every case (single-precision sums cancel to 1e-7 of it)."""
    w = case["w"]
    p = case["p"]
    tol = PREC[prec][1]
    plan = _plan(case, prec)
    V, W = plan.mobility(dev(w["Y"]), dev(w["F"]), None)
    Vr, Wr = ff.mobility(p, w["Y"], w["F"], None)
    assert normwise(host(V), Vr) < tol
    ang = np.linalg.norm(Vr) / w["a"]
    if prec == "fp64" and np.linalg.norm(Wr) > 1e-6 * ang:
        assert normwise(host(W), Wr) < 1e-10
    else:
        scale = max(np.linalg.norm(Wr), ang)
        assert np.linalg.norm(host(W) - Wr) < tol * scale
    V2, W2 = plan.mobility(dev(w["Y"]), dev(w["F"]), dev(w["T"]), want_omega=False)
    assert W2 is None and normwise(host(V2), case["V"]) < tol


def test_deterministic_and_permutation_invariant():
    w = workloads.workload(0)
    plan = make_plan(w, 0)
    Y, F, T = dev(w["Y"]), dev(w["F"]), dev(w["T"])
    V1, W1 = plan.mobility(Y, F, T)
    V2, W2 = plan.mobility(Y, F, T)
    assert np.array_equal(host(V1), host(V2)) and np.array_equal(host(W1), host(W2))
    perm = np.random.default_rng(5).permutation(w["N"])
    V3, W3 = plan.mobility(dev(w["Y"][perm]), dev(w["F"][perm]), dev(w["T"][perm]))
    assert maxrel(host(V3), host(V1)[perm]) < 1e-12 and maxrel(host(W3), host(W1)[perm]) < 1e-12


def test_spread_interp_adjoint_on_gpu():
    """<u, J~^dagger F + N~^dagger T> = <(F, T), (J~ u, N~ u)> (Sec. 2: spreading
    and interpolation are adjoint) for the FP64 HIP operators."""
    import torch
    w, _ = _case("ragged54")
    plan = make_plan(w, 0)
    rng = np.random.default_rng(8)
    u = rng.normal(size=(3, w["grid"], w["grid"], w["grid"]))
    g = plan.spread(dev(w["Y"]), dev(w["F"]), dev(w["T"]))
    lhs = float(np.sum(host(g) * u)) * (w["L"] / w["grid"]) ** 3
    V, W = plan.interp(dev(w["Y"]), torch.as_tensor(u, device="cuda").contiguous())
    rhs = float(np.sum(host(V) * w["F"]) + np.sum(host(W) * w["T"]))
    assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), 1.0)


def test_nonfinite_position_is_reported():
    w = workloads.workload(0)
    plan = make_plan(w, 1)
    Y = w["Y"].copy()
    Y[3, 1] = np.nan
    plan.mobility(dev(Y), dev(w["F"]), dev(w["T"]))
    assert plan.last_error() == -5
    assert plan.last_error() == 0


def _clustered(n_big=9000, n_mid=600, n_rest=400, seed=11):
    """A box with one dense cluster (more members per grid bin and per pair
    cell than an LDS sort holds), one medium cluster (an LDS sort) and loose
    particles.  Cluster members overlap, which the library allows; they sit on
    jittered lattices so no pair is closer than ~0.04 (the corrections' small-r
    cancellation stays far below the tolerance)."""
    rng = np.random.default_rng(seed)
    L, grid = 40.0, 32                     # dx = 1.25

    def lattice(n, lo, side):
        k = int(math.ceil(n ** (1.0 / 3.0)))
        g = (np.stack(np.meshgrid(*([np.arange(k)] * 3), indexing="ij"), -1).reshape(-1, 3) + 0.5) / k
        g = g[rng.choice(len(g), size=n, replace=False)]
        return lo + side * g + rng.uniform(-0.2, 0.2, size=(n, 3)) * side / k

    # grid cell [10, 11.25)^3: one first support point, one bin; pair cell
    # width 40/20 = 2: [10, 12)^3 holds the whole cluster
    big = lattice(n_big, 10.05, 1.15)
    mid = lattice(n_mid, 25.05, 1.15)
    rest = rng.uniform(0.0, L, size=(n_rest, 3))
    Y = np.concatenate([big, mid, rest])
    Y = Y[rng.permutation(len(Y))]
    N = len(Y)
    return dict(N=N, L=L, a=A, eta=1.0, grid=grid, Sigma=1.5 * SIG, M_G=12, R_c=2.0,
                Y=Y, F=rng.normal(size=(N, 3)), T=rng.normal(size=(N, 3)))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_long_sort_segments_match_oracle(prec):
    """Grid bins and pair cells with 600 and 9000 members take the workgroup
    sorts (LDS bitonic, and rank counting); spread (all particles) and the
    mobility of a subsample agree with the oracle, and the result is the same
    from call to call."""
    w = _clustered()
    p = oracle_params(w)
    plan = make_plan(w, PREC[prec][0])
    Y, F, T = dev(w["Y"]), dev(w["F"]), dev(w["T"])
    f = ff.spread(p, w["Y"], w["F"], w["T"])
    g = host(plan.spread(Y, F, T))
    # FP32: grid points near the big cluster sum 9000 terms
    tol = 1e-10 if prec == "fp64" else 1e-4
    assert normwise(gpu_to_oracle_grid(g), f) < tol
    V1, W1 = plan.mobility(Y, F, T)
    V2, W2 = plan.mobility(Y, F, T)
    V1, W1 = host(V1), host(W1)
    assert np.array_equal(V1, host(V2)) and np.array_equal(W1, host(W2))
    sub = np.sort(np.random.default_rng(3).choice(w["N"], size=60, replace=False))
    Vr, Wr = ff.mobility(p, w["Y"], w["F"], w["T"], targets=sub)
    tol = 1e-9 if prec == "fp64" else 1e-4
    assert normwise(V1[sub], Vr) < tol and normwise(W1[sub], Wr) < tol


def _mid_clusters(sizes=(3, 16, 17, 33, 64, 65, 300), n_rest=100, seed=12):
    """Clusters of the given sizes, each inside one pair cell (width 2) and one
    grid cell (dx = 1.25), so pair cells hold exactly those counts (loose
    particles rarely join) across the thread (<= 16), wavefront (17..64) and
    workgroup (> 64) sorts; grid bins (8 x 8 x 16 support starts) hold one or
    two clusters."""
    rng = np.random.default_rng(seed)
    L, grid = 40.0, 32
    corners = [(10, 10, 10), (20, 10, 10), (10, 20, 10), (10, 10, 20), (30, 10, 10), (20, 20, 20),
               (30, 30, 30)]
    parts = []
    for n, c in zip(sizes, corners):
        k = int(math.ceil(n ** (1.0 / 3.0)))
        g = (np.stack(np.meshgrid(*([np.arange(k)] * 3), indexing="ij"), -1).reshape(-1, 3) + 0.5) / k
        g = g[rng.choice(len(g), size=n, replace=False)]
        parts.append(np.array(c) + 0.05 + 1.15 * g + rng.uniform(-0.2, 0.2, size=(n, 3)) * 1.15 / k)
    parts.append(rng.uniform(0.0, L, size=(n_rest, 3)))
    Y = np.concatenate(parts)
    Y = Y[rng.permutation(len(Y))]
    N = len(Y)
    return dict(N=N, L=L, a=A, eta=1.0, grid=grid, Sigma=1.5 * SIG, M_G=12, R_c=2.0,
                Y=Y, F=rng.normal(size=(N, 3)), T=rng.normal(size=(N, 3)))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_mid_sort_segments_match_oracle(prec):
    """Pair cells of 3, 16, 17, 33, 64, 65 and 300 members (both sides of the
    thread/wavefront and wavefront/workgroup limits of the segment sorts):
    spread and the mobility of every cluster's members agree with the oracle,
    repeated calls are bitwise equal, and a permuted input gives the permuted
    result."""
    w = _mid_clusters()
    p = oracle_params(w)
    plan = make_plan(w, PREC[prec][0])
    Y, F, T = dev(w["Y"]), dev(w["F"]), dev(w["T"])
    f = ff.spread(p, w["Y"], w["F"], w["T"])
    tol = PREC[prec][1]
    assert normwise(gpu_to_oracle_grid(host(plan.spread(Y, F, T))), f) < tol
    V1, W1 = plan.mobility(Y, F, T)
    V2, W2 = plan.mobility(Y, F, T)
    V1, W1 = host(V1), host(W1)
    assert np.array_equal(V1, host(V2)) and np.array_equal(W1, host(W2))
    sub = np.sort(np.random.default_rng(4).choice(w["N"], size=80, replace=False))
    Vr, Wr = ff.mobility(p, w["Y"], w["F"], w["T"], targets=sub)
    tol_m = 1e-9 if prec == "fp64" else 1e-5
    assert normwise(V1[sub], Vr) < tol_m and normwise(W1[sub], Wr) < tol_m
    perm = np.random.default_rng(6).permutation(w["N"])
    V3, W3 = plan.mobility(dev(w["Y"][perm]), dev(w["F"][perm]), dev(w["T"][perm]))
    tol_p = 1e-12 if prec == "fp64" else 1e-5
    assert maxrel(host(V3), V1[perm]) < tol_p and maxrel(host(W3), W1[perm]) < tol_p


def test_standard_fcm_widths_recognised():
    """Standard FCM passed with the torque width rounded differently (one part
    in 1e14) is recognised as such: no correction, results equal to those of
    the exact width."""
    w = _case("standard48")[0]
    sd = A / (6.0 * math.sqrt(math.pi)) ** (1.0 / 3.0)
    Y, F, T = dev(w["Y"]), dev(w["F"]), dev(w["T"])
    out = []
    for s in (sd, sd * (1.0 + 1e-14), sd * (1.0 - 1e-14)):
        plan = make_plan(w, 0, sigma_D_grid=s)
        assert plan.info()["cells_per_axis"] == 1
        V, W = plan.mobility(Y, F, T)
        out.append((host(V), host(W)))
    for V, W in out[1:]:
        assert np.array_equal(V, out[0][0]) and np.array_equal(W, out[0][1])
    p = oracle_params(w, Sigma_D=sd)
    Vr, Wr = ff.mobility(p, w["Y"], w["F"], w["T"])
    assert normwise(out[0][0], Vr) < 1e-10 and normwise(out[0][1], Wr) < 1e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_mobility_repeat_equals_full_call(prec):
    """fcm_mobility_repeat reuses the last call's sort, records and pair lists:
    for new forces and torques it returns exactly what fcm_mobility returns at
    the same positions (also without torques or Omega), and it is refused
    once another call has sorted other positions."""
    w = _case("crowded")[0]
    plan = make_plan(w, PREC[prec][0])
    rng = np.random.default_rng(21)
    Y = dev(w["Y"])
    F1, T1 = dev(w["F"]), dev(w["T"])
    F2, T2 = dev(rng.normal(size=(w["N"], 3))), dev(rng.normal(size=(w["N"], 3)))
    plan.mobility(Y, F1, T1)
    Vr, Wr = plan.mobility_repeat(F2, T2)
    Vr, Wr = host(Vr), host(Wr)
    V0r, _ = plan.mobility_repeat(F2, None, want_omega=False)
    V0r = host(V0r)
    Vf, Wf = plan.mobility(Y, F2, T2)
    assert np.array_equal(Vr, host(Vf)) and np.array_equal(Wr, host(Wf))
    V0f, _ = plan.mobility(Y, F2, None, want_omega=False)
    assert np.array_equal(V0r, host(V0f))
    # and against the oracle at the same positions
    Vo, Wo = ff.mobility(oracle_params(w), w["Y"], host(F2), host(T2))
    assert normwise(Vr, Vo) < PREC[prec][1] and normwise(Wr, Wo) < PREC[prec][1]
    # a stage call sorts again: the reuse ends
    plan.interp(Y, plan.new_grid().zero_())
    from paper_2310_12651_amd import FCMError
    with pytest.raises(FCMError):
        plan.mobility_repeat(F2, T2)


def _lattice_case(M, dx, N, seed):
    """N distinct grid points j dx with odd indices, each coordinate shifted by
    n L, n in [-6, 6]; in eight of them one coordinate is n L exactly (four)
    or one ulp below it (four), which wraps to 0 or just below L: next to the
    odd sites, so no two particles come closer than dx."""
    rng = np.random.default_rng(seed)
    L = M * dx
    h = M // 2
    sites = rng.choice(h ** 3, size=N, replace=False)
    j = 2 * np.stack([sites % h, (sites // h) % h, sites // (h * h)], 1).astype(np.float64) + 1.0
    n = rng.integers(-6, 7, size=(N, 3)).astype(np.float64)
    Y = j * dx + n * L
    for i in range(8):
        a = i % 3
        Y[i, a] = n[i, a] * L if i < 4 else n[i, a] * L - np.spacing(abs(n[i, a] * L) + L)
    d = Y[:, None, :] - Y[None, :, :]
    d -= L * np.round(d / L)
    r = np.sqrt(np.sum(d * d, -1)) + np.eye(N) * L
    assert r.min() > 0.99 * dx, r.min()
    return Y, L, rng


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("M,dx,MG", [(54, 0.3, 10), (64, 0.35, 12)], ids=["rowmajor54", "tiled64"])
def test_lattice_positions_periods_away_match_oracle(M, dx, MG, prec):
    """Support starts are integers decided at grid points: the position wraps
    by the exact remainder on both sides, so each support lies where the
    oracle puts it (a window one point off changes V by the kernel's tail)."""
    Y, L, rng = _lattice_case(M, dx, 80, zlib.crc32(b"lattice%d" % M))
    F, T = rng.normal(size=(len(Y), 3)), rng.normal(size=(len(Y), 3))
    p = ff.Params(L=L, M=M, a=A, Sigma=2.0 * dx, M_G=MG, R_c=2.9)
    Vr, Wr = ff.mobility(p, Y, F, T)
    w = dict(N=len(Y), L=L, a=A, Sigma=2.0 * dx, grid=M, M_G=MG, R_c=2.9)
    plan = make_plan(w, 0 if prec == "fp64" else 1)
    try:
        V, W = plan.mobility(dev(Y), dev(F), dev(T))
        V, W = host(V), host(W)
        assert plan.last_error() == 0
    finally:
        plan.close()
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert normwise(V, Vr) < tol and normwise(W, Wr) < tol, (normwise(V, Vr), normwise(W, Wr))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_coincident_centres_match_oracle(prec):
    """Distinct particles at exactly the same point (ten pairs and a triple
    among 40): the pair corrections take App. B's r -> 0 limits on both sides
    (the oracle's closed forms divide by r, so it switches to the limits at
    r = 0; the kernel below 1e-3 sigma)."""
    rng = np.random.default_rng(zlib.crc32(b"coincident"))
    L, M = 14.0, 36
    Y = rng.uniform(-L, 2.0 * L, size=(40, 3))
    for i in range(10):
        Y[2 * i + 1] = Y[2 * i]
    Y[21] = Y[22] = Y[20]
    F, T = rng.normal(size=(40, 3)), rng.normal(size=(40, 3))
    w = dict(N=40, L=L, a=A, Sigma=0.75, grid=M, M_G=10, R_c=4.5)
    Vr, Wr = ff.mobility(oracle_params(w), Y, F, T)
    assert np.isfinite(Vr).all() and np.isfinite(Wr).all()
    plan = make_plan(w, 0 if prec == "fp64" else 1)
    try:
        V, W = plan.mobility(dev(Y), dev(F), dev(T))
        V, W = host(V), host(W)
    finally:
        plan.close()
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert normwise(V, Vr) < tol and normwise(W, Wr) < tol, (normwise(V, Vr), normwise(W, Wr))


def _cutoff_case(L, Rc, npairs, seed):
    """Pairs whose separation is R_c to within two ulps, spread over the box."""
    rng = np.random.default_rng(seed)
    P = rng.uniform(0.0, L, size=(npairs, 3))
    d = rng.normal(size=(npairs, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    Q = P + Rc * d * (1.0 + rng.integers(-2, 3, size=(npairs, 1)) * 2.0 ** -52)
    return np.concatenate([P, Q]), rng


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pairs_at_the_cutoff_match_oracle(prec):
    """The cut-off r < R_c decides a pair within ulps of R_c as the oracle
    does: r^2 summed (x0^2 + x1^2) + x2^2 with each step rounded, against the
    smallest double whose square root reaches R_c (a fused r^2, or r^2 <
    R_c * R_c, flips about one such pair in twenty; a flipped pair moves V by
    the correction at R_c, ~1e-4 here)."""
    L, Rc = 24.0, 2.5
    Y, rng = _cutoff_case(L, Rc, 60, zlib.crc32(b"cutoff"))
    F, T = rng.normal(size=(len(Y), 3)), rng.normal(size=(len(Y), 3))
    w = dict(N=len(Y), L=L, a=A, Sigma=0.75, grid=48, M_G=10, R_c=Rc)
    Vr, Wr = ff.mobility(oracle_params(w), Y, F, T)
    plan = make_plan(w, 0 if prec == "fp64" else 1)
    try:
        V, W = plan.mobility(dev(Y), dev(F), dev(T))
        V, W = host(V), host(W)
    finally:
        plan.close()
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert normwise(V, Vr) < tol and normwise(W, Wr) < tol, (normwise(V, Vr), normwise(W, Wr))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_far_positions_match_oracle(prec):
    """Finite positions up to 1e9 box lengths away wrap by the exact remainder
    on both sides (no position is too far to wrap), and such a call raises no
    flag; infinities still do."""
    rng = np.random.default_rng(zlib.crc32(b"far"))
    L, N = 20.0, 40
    Y = rng.uniform(0.0, L, size=(N, 3)) + L * np.round(10.0 ** rng.uniform(0.0, 9.0, size=(N, 3)) *
                                                         rng.choice([-1.0, 1.0], size=(N, 3)))
    F, T = rng.normal(size=(N, 3)), rng.normal(size=(N, 3))
    w = dict(N=N, L=L, a=A, Sigma=0.8, grid=48, M_G=10, R_c=4.0)
    Vr, Wr = ff.mobility(oracle_params(w), Y, F, T)
    plan = make_plan(w, 0 if prec == "fp64" else 1)
    try:
        V, W = plan.mobility(dev(Y), dev(F), dev(T))
        V, W = host(V), host(W)
        assert plan.last_error() == 0
        Yi = Y.copy()
        Yi[5, 2] = np.inf
        plan.mobility(dev(Yi), dev(F), dev(T))
        assert plan.last_error() == -5
    finally:
        plan.close()
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert normwise(V, Vr) < tol and normwise(W, Wr) < tol, (normwise(V, Vr), normwise(W, Wr))
