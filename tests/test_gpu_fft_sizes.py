"""Grid sizes whose FFT passes run in registers (FP32): the Stokes solve of the
FP32 and the FP64 path (whose passes use the LDS kernels) against the oracle's
at every size, 64^3 to 432^3 (the request stream's largest grids), and the
whole mobility, where the solve hands the interpolation a tiled field, against
the FP64 path.

Inputs: a white-noise field (seeded) for the solve; 400 random particles with
N(0, 1) forces and torques in a box of side M (dx = 1, Sigma = 1, M_G = 10,
R_c = 5.5) for the mobility.
"""

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
