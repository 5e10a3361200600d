"""Statistical pins of the oracle against the paper's calibration (Sec. 5.1).

The paper tabulates, for a random suspension at volume fraction 8 %, the grid
resolution (Sigma/dx, M_G) that keeps the mean relative velocity error
eps = mean_n |V_n - U_n| / |U_n| below a tolerance (Table 1), and the slope
lambda_eps of the cut-off line R_c = lambda_eps Sigma that does the same for
the pair correction (Table 2).  These tests rebuild both measurements with the
oracle on a small suspension (300 spheres at 8 %, random sequential addition)
and require the errors at the paper's tabulated parameters to be of the
tabulated size: within a factor 2 of eps for the Table 1 rows eps = 1e-2,
1e-3, 1e-4, and within a factor 3 for every Table 2 row at Sigma ~ 2 sigma.

The reference U is fast FCM with every error source pushed far below 1e-8:
Sigma/dx = 1.6 with M_G = 24 (window half-width 7.5 Sigma) and all pairs
within 0.499 L corrected (the corrections there are below e^-30).  Table 1's
rows eps = 1e-6 and 1e-8 (M_G = 12 and 14) are not pinned: with this
library's support window (start = floor(Y/dx - M_G/2) + 1) those M_G truncate
the Gaussian at 5 Sigma on the near side and give eps ~ 1e-5; the library's
own calibration is measured separately on the GPU.
"""

import math

import numpy as np
import pytest

import workloads
from golden_tables import table
from oracle import fastfcm as ff

A = 1.0
SIG = A / math.sqrt(math.pi)


@pytest.fixture(scope="module")
def suspension():
    N, phi = 300, 0.08
    L = workloads.box_for_fraction(N, A, phi)
    rng = np.random.default_rng(77)
    Y = workloads.rsa_positions(N, L, A, rng)
    F = rng.normal(size=(N, 3))
    return dict(N=N, L=L, Y=Y, F=F)


def _velocities(s, Sigma0, ratio, MG, R_c=None, lam=None):
    """Force-only fast FCM with Sigma/dx = ratio exactly (Sigma close to Sigma0)."""
    L = s["L"]
    M = int(math.ceil(L * ratio / Sigma0 - 1e-9))
    Sigma = ratio * L / M
    if R_c is None:
        R_c = min(lam * Sigma, 0.499 * L)
    p = ff.Params(L=L, M=M, a=A, Sigma=Sigma, M_G=MG, R_c=R_c)
    V, _ = ff.mobility(p, s["Y"], s["F"], None)
    return V


def _eps(V, U):
    return float(np.mean(np.linalg.norm(V - U, axis=1) / np.linalg.norm(U, axis=1)))


@pytest.fixture(scope="module")
def reference(suspension):
    return _velocities(suspension, 2.0 * SIG, 1.6, 24, R_c=0.499 * suspension["L"])


# the paper's printed rows (tests/golden/, Sec. 5.1 Table 1 and Sec. 5.2 Table 2)
T1 = table("table1_grid_resolution.txt")
T2 = table("table2_cutoff_slope.txt")


@pytest.mark.parametrize("ratio, MG, eps", [(r[1], int(r[2]), r[0]) for r in T1 if r[0] >= 1e-4])
def test_table1_grid_resolution_rows(suspension, reference, ratio, MG, eps):
    """Table 1: the grid part at (Sigma/dx, M_G) of a row, all pairs corrected."""
    V = _velocities(suspension, 2.0 * SIG, ratio, MG, R_c=0.499 * suspension["L"])
    e = _eps(V, reference)
    assert 0.5 * eps < e < 2.0 * eps, e


def test_table1_error_falls_with_resolution(suspension, reference):
    """Both parameters matter: lowering either below the 1e-4 row raises eps."""
    e0 = _eps(_velocities(suspension, 2.0 * SIG, 0.99, 10, R_c=0.499 * suspension["L"]), reference)
    e_dx = _eps(_velocities(suspension, 2.0 * SIG, 0.8, 10, R_c=0.499 * suspension["L"]), reference)
    e_mg = _eps(_velocities(suspension, 2.0 * SIG, 0.99, 8, R_c=0.499 * suspension["L"]), reference)
    assert e_dx > 5 * e0 and e_mg > 5 * e0


@pytest.mark.parametrize("lam, eps", [(r[2], r[0]) for r in T2])   # the phi = 8 % column
def test_table2_cutoff_slope_rows(suspension, reference, lam, eps):
    """Table 2 (phi = 8 %): R_c = lambda_eps Sigma with the grid resolved
    (Sigma/dx = 1.6, M_G = 20) gives an error of the row's size."""
    V = _velocities(suspension, 2.0 * SIG, 1.6, 20, lam=lam)
    e = _eps(V, reference)
    assert eps / 3.0 < e < 3.0 * eps, e


def test_request_stream_uses_table3():
    """The request stream's width rule is Table 3's optimum (Sec. 5.2)."""
    T3 = table("table3_optimal_width.txt")
    assert np.allclose(workloads._T3_PHI, T3[:, 0]) and np.allclose(workloads._T3_RATIO, T3[:, 1])
