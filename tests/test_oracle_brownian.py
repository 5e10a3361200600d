"""Pins of the oracle's Brownian velocities (positive splitting, Sec. 3.3).

* The grid part is a linear map B_g of the grid noise; built column by
  column from unit noise fields, B_g B_g^T equals 2 kT times the grid
  mobility M~ assembled from unit forces through spread, solve and
  interpolation (fluctuation-dissipation on the grid).
* The pair matrix C equals, column by column, the correction the fast-FCM
  mobility adds for a unit force (pairs within R_c and the self term), and
  it is positive definite, as the paper shows for the VF block.
* Hence the two parts together have covariance 2 kT M.
"""

import math

import numpy as np
import pytest

import workloads
from oracle import brownian as br
from oracle import fastfcm as ff

A = 1.0


@pytest.fixture(scope="module")
def small():
    rng = np.random.default_rng(99)
    L, M, N = 8.0, 8, 3
    Y = workloads.rsa_positions(N, L, A, rng)
    p = ff.Params(L=L, M=M, a=A, Sigma=0.9, M_G=8, R_c=3.9)
    return dict(p=p, Y=Y, N=N)


def _unit_forces(N):
    for j in range(3 * N):
        F = np.zeros((N, 3))
        F.flat[j] = 1.0
        yield j, F


def test_grid_part_covariance_is_2kT_grid_mobility(small):
    p, Y, N = small["p"], small["Y"], small["N"]
    kT = 0.7
    Mx, My, Mz = p.Mv
    cols = []
    for c in range(3):
        for i in range(Mx * My * Mz):
            xi = np.zeros((3, Mx * My * Mz))
            xi[c, i] = 1.0
            cols.append(br.brownian_grid(p, Y, xi.reshape(3, Mx, My, Mz), kT).ravel())
    B = np.array(cols).T                        # 3N x 3 M^3
    Mt = np.zeros((3 * N, 3 * N))
    for j, F in _unit_forces(N):
        V, _ = ff.mobility(p, Y, F, None, with_correction=False)
        Mt[:, j] = V.ravel()
    assert np.allclose(B @ B.T, 2.0 * kT * Mt, rtol=0, atol=1e-12 * np.abs(Mt).max())


def test_pair_matrix_is_the_correction_and_positive(small):
    p, Y, N = small["p"], small["Y"], small["N"]
    C = br.pair_matrix(p, Y)
    for j, F in _unit_forces(N):
        V1, _ = ff.mobility(p, Y, F, None)
        V0, _ = ff.mobility(p, Y, F, None, with_correction=False)
        assert np.allclose(C[:, j], (V1 - V0).ravel(), rtol=0, atol=1e-13 * np.abs(C).max())
    assert np.allclose(C, C.T, rtol=0, atol=1e-14 * np.abs(C).max())
    assert np.linalg.eigvalsh(C).min() > 0.0


def test_square_root_and_total_covariance(small):
    p, Y, N = small["p"], small["Y"], small["N"]
    C = br.pair_matrix(p, Y)
    S = br.sqrt_spd(C)
    assert np.allclose(S @ S, C, rtol=0, atol=1e-13 * np.abs(C).max())
    kT = 1.3
    cols = [br.brownian_pair(p, Y, np.eye(3 * N)[j].reshape(N, 3), kT).ravel() for j in range(3 * N)]
    Bp = np.array(cols).T
    assert np.allclose(Bp @ Bp.T, 2.0 * kT * C, rtol=0, atol=1e-12 * np.abs(C).max())
