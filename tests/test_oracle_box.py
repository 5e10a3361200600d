"""Rectangular boxes in the oracle, pinned by an exact identity.

A periodic suspension in a cube of side L is the same periodic suspension as
its copy in a box of sides (k L, L, L) holding k translated copies of every
particle (with the same forces and torques), on a grid with the same spacing:
every Fourier mode of the copied field is a mode of the cube's, the modes with
index M/2 of the cube are those the long axis zeroes, and with R_c < L/2 the
pairs within R_c are the same.  So the velocities of the copies equal the
cube's, to rounding.  This checks the per-axis wave numbers, windows, Nyquist
planes, cell counts and minimum images of the oracle.
"""

import math

import numpy as np
import pytest

import workloads
from oracle import fastfcm as ff

A = 1.0
SIG = A / math.sqrt(math.pi)


@pytest.fixture(scope="module")
def cube():
    rng = np.random.default_rng(4242)
    L, M, N = 14.0, 24, 20
    Y = workloads.rsa_positions(N, L, A, rng)
    F = rng.normal(size=(N, 3))
    T = rng.normal(size=(N, 3))
    p = ff.Params(L=L, M=M, a=A, Sigma=1.5 * SIG, M_G=12, R_c=6.0)
    V, W = ff.mobility(p, Y, F, T)
    return dict(L=L, M=M, N=N, Y=Y, F=F, T=T, p=p, V=V, W=W)


@pytest.mark.parametrize("axis, k", [(0, 2), (1, 3), (2, 2)])
def test_copies_along_one_axis_keep_the_cube_velocities(cube, axis, k):
    L, M, N = cube["L"], cube["M"], cube["N"]
    e = np.zeros(3)
    e[axis] = 1.0
    Lb = [L] * 3
    Mb = [M] * 3
    Lb[axis] *= k
    Mb[axis] *= k
    Y = np.concatenate([cube["Y"] + j * L * e for j in range(k)])
    F = np.tile(cube["F"], (k, 1))
    T = np.tile(cube["T"], (k, 1))
    p = ff.Params(L=Lb, M=Mb, a=A, Sigma=1.5 * SIG, M_G=12, R_c=6.0)
    assert not p.cubic
    V, W = ff.mobility(p, Y, F, T)
    for j in range(k):
        sl = slice(j * N, (j + 1) * N)
        assert np.max(np.abs(V[sl] - cube["V"])) < 1e-12 * np.max(np.abs(cube["V"]))
        assert np.max(np.abs(W[sl] - cube["W"])) < 1e-12 * np.max(np.abs(cube["W"]))


def test_unequal_spacing_is_refused():
    with pytest.raises(ValueError):
        ff.Params(L=[10.0, 10.0, 12.0], M=[20, 20, 20], a=A, Sigma=1.0, M_G=10, R_c=3.0)


def test_box_cells_per_axis():
    assert list(ff.cell_counts([30.0, 12.0, 9.0], 4.0)) == [7, 3, 3]
    keys = ff.hash_particles(np.array([[29.0, 11.0, 8.9]]), [30.0, 12.0, 9.0], [7, 3, 3])
    assert keys[0] == 6 + (2 + 2 * 3) * 7
