"""Grid sizes whose FFT passes run in registers (FP32): the Stokes solve of the
FP32 and the FP64 path (whose passes use the LDS kernels) against the oracle's
at every size, 64^3 to 432^3 (the request stream's largest grids), and the
whole mobility, where the solve hands the interpolation a tiled field, against
the FP64 path.  Above 432^3, up to the largest cube a plan accepts (1024^3;
LDS passes), the solve of single Fourier modes, one per solve, against their
closed form (ff.stokes_plane_wave), at 4096 sampled grid points.

Inputs: a white-noise field (seeded) for the solve; 400 random particles with
N(0, 1) forces and torques in a box of side M (dx = 1, Sigma = 1, M_G = 10,
R_c = 5.5) for the mobility; seeded modes for the large grids, one at a time
(FP64: along x, along y one below the Nyquist index, a mixed one with a z
index one below Nyquist, a random one; FP32: along x and two mixed ones).
"""

import math
import os
import zlib

import numpy as np
import pytest

from gpu_common import dev, gpu_to_oracle_grid, host, normwise, oracle_to_gpu_grid
from oracle import fastfcm as ff

pytestmark = pytest.mark.gpu

REGISTER_SIZES = [64, 72, 96, 108, 128, 144, 162, 192, 216, 256, 288, 324, 384, 432]
# threads of the oracle's FFT at the largest sizes (the host's share is 16)
WORKERS = max(1, min(16, os.cpu_count() or 1))


def _plan(M, N, precision, R_c=0.0):
    from paper_2310_12651_amd import Plan
    return Plan(N, float(M), 1.0, 1.0, M, R_c, support=10, precision=precision)


@pytest.mark.parametrize("M", REGISTER_SIZES)
def test_solve_fp32_register_passes(M):
    import torch
    rng = np.random.default_rng(zlib.crc32(f"solve{M}".encode()))
    f = rng.normal(size=(3, M, M, M))
    g32 = torch.as_tensor(oracle_to_gpu_grid(f), device="cuda").float().contiguous()
    g64 = torch.as_tensor(oracle_to_gpu_grid(f), device="cuda").double().contiguous()
    p32, p64 = _plan(M, 1, 1), _plan(M, 1, 0)
    p32.solve(g32)
    p64.solve(g64)
    p32.close()
    p64.close()
    u32 = host(g32).astype(np.float64)
    u64 = host(g64)
    del g32, g64
    assert normwise(u32, u64) < 1e-5, (M, normwise(u32, u64))
    u = ff.stokes_solve(ff.Params(L=float(M), M=M, a=1.0, Sigma=1.0, M_G=10, R_c=0.0), f,
                        workers=WORKERS)
    e64 = normwise(gpu_to_oracle_grid(u64), u)
    e32 = normwise(gpu_to_oracle_grid(u32), u)
    print(f"solve M={M} fp64={e64:.2e} fp32={e32:.2e}", flush=True)
    assert e64 < 1e-10, M
    assert e32 < 1e-5, M


@pytest.mark.parametrize("M", REGISTER_SIZES)
def test_mobility_fp32_register_passes(M):
    N = 400
    rng = np.random.default_rng(zlib.crc32(f"mob{M}".encode()))
    Y = rng.uniform(0.0, float(M), size=(N, 3))
    F = rng.normal(size=(N, 3))
    T = rng.normal(size=(N, 3))
    out = {}
    for prec in (1, 0):
        plan = _plan(M, N, prec, R_c=5.5)
        V, W = plan.mobility(dev(Y), dev(F), dev(T))
        out[prec] = (host(V), host(W))
        plan.close()
    assert normwise(out[1][0], out[0][0]) < 1e-5, M
    assert normwise(out[1][1], out[0][1]) < 1e-5, M


LARGE_SIZES = [486, 512, 576, 648, 768, 864, 972, 1024]


def _large_modes(M, prec):
    """Seeded modes: FP64 takes one along x, one along y one below the Nyquist
    index, a mixed one with a z index one below Nyquist and a random one; FP32
    takes the mode along x and two mixed ones (|j_d| <= M/6): a mode along one
    axis with a large index rounds to FP32 in a one-dimensional pattern whose
    low-k content the solve amplifies by |j|^2 (1e-4 at 768^3 with an
    independent single-precision FFT too), which fields spread from Gaussians
    do not have."""
    rng = np.random.default_rng(zlib.crc32(f"large{M}-{prec}".encode()))
    h = M // 2 - 1
    if prec == 0:
        js = [(1, 0, 0), (0, h, 0), (-(M // 3), 7, h - 2), tuple(int(v) for v in rng.integers(-h, h + 1, size=3))]
    else:
        q = M // 8
        js = [(1, 0, 0), (-(M // 6), 7, q), tuple(int(v) for v in rng.integers(-q, q + 1, size=3))]
    return [(j, rng.normal(size=3), float(rng.uniform(0.0, 2.0 * np.pi))) for j in js]


@pytest.mark.parametrize("M", LARGE_SIZES)
def test_solve_large_grids_against_plane_waves(M):
    """One solve per mode, each against its own closed form (in a sum of modes
    the solve divides by k^2, so rounding of the larger modes' forcing lands
    on the smallest k amplified by up to (M / 2)^2)."""
    import torch
    p = ff.Params(L=float(M), M=M, a=1.0, Sigma=1.0, M_G=10, R_c=0.0)
    idx = np.random.default_rng(zlib.crc32(f"pts{M}".encode())).integers(0, M, size=(4096, 3))
    n = torch.arange(M, device="cuda")
    it = torch.as_tensor(idx, device="cuda")
    for prec, tol in [(1, 1e-5), (0, 1e-10)]:
        plan = _plan(M, 1, prec)
        try:
            for j, A, phi in _large_modes(M, prec):
                # the field (3, z, y, x): A_c cos(2 pi ((j . n) mod M) / M + phi)
                ph = (j[0] * n[None, None, :] + j[1] * n[None, :, None] + j[2] * n[:, None, None]) % M
                wave = torch.cos(ph.to(torch.float64) * (2.0 * math.pi / M) + phi)
                del ph
                g = torch.stack([(float(A[c]) * wave).to(plan.grid_dtype) for c in range(3)])
                del wave
                plan.solve(g)
                uh = host(g[:, it[:, 2], it[:, 1], it[:, 0]].T).astype(np.float64)
                del g
                e = normwise(uh, ff.stokes_plane_wave(p, j, A, phi, idx))
                print(f"large solve M={M} prec={prec} j={j} err={e:.2e}", flush=True)
                assert e < tol, (M, prec, j, e)
        finally:
            plan.close()
            torch.cuda.empty_cache()


@pytest.mark.parametrize("M,Mb", [(1024, 128), (972, 162), (864, 108)])
def test_mobility_largest_grids_by_periodic_copies(M, Mb):
    """The whole mobility on the largest cubes (every stage at these sizes:
    sort, spread and interpolation on the row-major field, LDS passes, pair
    correction with 128 cells an axis) against the oracle: (M/Mb)^3 copies of
    an Mb^3 cube fill the M^3 box, and by periodicity every copy's particles
    move as the cube's, which the oracle computes (FP64 1e-10, FP32 1e-5)."""
    k = M // Mb
    rng = np.random.default_rng(zlib.crc32(f"copies{M}".encode()))
    N = 6
    Y = rng.uniform(0.0, float(Mb), size=(N, 3))
    F, T = rng.normal(size=(N, 3)), rng.normal(size=(N, 3))
    p = ff.Params(L=float(Mb), M=Mb, a=1.0, Sigma=1.0, M_G=10, R_c=5.5)
    Vr, Wr = ff.mobility(p, Y, F, T)
    shifts = np.stack(np.meshgrid(*[np.arange(k)] * 3, indexing="ij"), -1).reshape(-1, 1, 3) * float(Mb)
    Yb = (Y[None] + shifts).reshape(-1, 3)
    Fb, Tb = np.tile(F, (k ** 3, 1)), np.tile(T, (k ** 3, 1))
    for prec, tol in [(1, 1e-5), (0, 1e-10)]:
        from paper_2310_12651_amd import Plan
        plan = Plan(len(Yb), float(M), 1.0, 1.0, M, 5.5, support=10, precision=prec)
        try:
            V, W = plan.mobility(dev(Yb), dev(Fb), dev(Tb))
            Vb, Wb = host(V).reshape(k ** 3, N, 3), host(W).reshape(k ** 3, N, 3)
            assert plan.last_error() == 0
        finally:
            plan.close()
        ev = max(normwise(Vb[c], Vr) for c in range(k ** 3))
        ew = max(normwise(Wb[c], Wr) for c in range(k ** 3))
        print(f"copies M={M} prec={prec} V={ev:.2e} W={ew:.2e}", flush=True)
        assert ev < tol and ew < tol, (M, prec, ev, ew)
