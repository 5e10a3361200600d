"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins
notice each one.  Every mutation below must move some pinned quantity well
beyond the tolerance its pin uses."""

import math

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import fastfcm as ff
from oracle import lattice

A = 1.0
SIG = A / math.sqrt(math.pi)
L = 20.0
Y4 = np.array([[2.1, 3.3, 4.9], [6.0, 8.2, 3.1], [11.7, 1.9, 15.2], [15.5, 16.0, 9.4]])


@pytest.fixture(scope="module")
def exact():
    return lattice.mobility_matrix(Y4, L, A)


def _fast_error(exact_M):
    p = ff.Params(L=L, M=27, a=A, Sigma=2 * SIG, M_G=20, R_c=8.6 * 2 * SIG)
    N = len(Y4)
    Mat = np.zeros((6 * N, 6 * N))
    for col in range(6 * N):
        F = np.zeros((N, 3))
        T = np.zeros((N, 3))
        (F if col < 3 * N else T).flat[col % (3 * N)] = 1.0
        V, W = ff.mobility(p, Y4, F, T)
        Mat[:3 * N, col] = V.ravel()
        Mat[3 * N:, col] = W.ravel()
    return np.linalg.norm(Mat - exact_M) / np.linalg.norm(exact_M)


def test_unmutated_oracle_passes(exact):
    assert _fast_error(exact) < 1e-8


MUTATIONS = {
    # sign of the torque spreading flipped (Sec. 3.4 printed with both signs)
    "torque_sign": lambda mp: mp.setattr(ff, "_particle_weights", _wrap_weights(torque_scale=-1.0)),
    # Laplacian modification of the force kernel dropped
    "no_laplacian": lambda mp: mp.setattr(ff, "_particle_weights", _wrap_weights(drop_lap=True)),
    # missing 1/2 in the Omega-T correction
    "OT_half": lambda mp: mp.setattr(cf, "correction_OT", _scaled(cf.correction_OT, 2.0)),
    # literal erf arguments r/(sigma sqrt2) of the printed correction_VF
    "VF_erf_args": lambda mp: mp.setattr(cf, "correction_VF", _literal_vf),
    # self correction with the wrong sign of its Q term
    "self_sign": lambda mp: mp.setattr(cf, "self_correction_VF", _bad_self),
    # Nyquist modes kept
    "nyquist": lambda mp: mp.setattr(ff, "stokes_solve", _keep_nyquist),
    # transposed V-T block
    "VT_transpose": lambda mp: mp.setattr(cf, "correction_VT", lambda x, *a, **k: cf.correction_OF(x, *a, **k).swapaxes(-1, -2)),
}

_orig_weights = ff._particle_weights
_orig_solve = ff.stokes_solve


def _wrap_weights(torque_scale=1.0, drop_lap=False):
    def w(p, Yw):
        flat, dmod, dtor, d = _orig_weights(p, Yw)
        if drop_lap:
            r2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
            dmod = cf.gaussian(np.sqrt(r2), p.Sigma)
        return flat, dmod, torque_scale * dtor, d
    return w


def _scaled(f, s):
    return lambda *a, **k: s * f(*a, **k)


def _literal_vf(x, sigma, Sigma, eta=1.0):
    from scipy.special import erf
    xx, r, I, xh = cf._geometry(x)
    G = cf.oseen(x, eta)
    LG = cf.lap_oseen(x, eta)
    dE = (erf(r / (sigma * math.sqrt(2))) - erf(r / (Sigma * math.sqrt(2))))[..., None, None]
    s1, s2 = sigma * math.sqrt(2), Sigma * math.sqrt(2)
    d = sigma ** 2 - Sigma ** 2
    # Q2 = Q - Q1, Q1 = erf(r / s2 sqrt2) lap G
    Q2 = cf.Q(x, s2, eta) - (cf.lap_oseen(x, eta) * erf(r / (s2 * math.sqrt(2)))[..., None, None])
    return (G + sigma ** 2 * LG) * dE + cf.S3_part(x, s1, eta) - cf.S3_part(x, s2, eta) \
        - d * Q2 - 0.25 * d * d * cf.T(x, s2, eta)


def _bad_self(a, sigma, Sigma, eta=1.0):
    sp = Sigma * math.sqrt(math.pi)
    d = sigma ** 2 - Sigma ** 2
    return (1 / (6 * math.pi * eta * a) - 1 / (6 * math.pi * eta * sp) - d / (12 * eta * sp ** 3)
            - d * d / (32 * eta * Sigma ** 5 * math.pi ** 1.5))


def _keep_nyquist(p, f):
    fh = np.fft.fftn(f, axes=(1, 2, 3))
    k = ff.wavenumbers(p)
    kx, ky, kz = k[:, None, None], k[None, :, None], k[None, None, :]
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    k2s = np.where(k2 == 0, 1.0, k2)
    kd = (kx * fh[0] + ky * fh[1] + kz * fh[2]) / k2s
    uh = np.stack([(fh[0] - kx * kd), (fh[1] - ky * kd), (fh[2] - kz * kd)]) / (p.eta * k2s)
    uh[:, 0, 0, 0] = 0
    return np.real(np.fft.ifftn(uh, axes=(1, 2, 3)))


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, exact, monkeypatch):
    MUTATIONS[name](monkeypatch)
    if name == "nyquist":
        # an odd grid has no Nyquist mode; the even-grid pin is the DFT check
        from test_oracle_grid import _dft_stokes
        p = ff.Params(L=5.0, M=6, a=A, Sigma=0.8, M_G=4, R_c=0.0)
        f = np.random.default_rng(1).normal(size=(3, 6, 6, 6))
        u = ff.stokes_solve(p, f)
        assert np.abs(u - _dft_stokes(p, f)).max() > 1e-6 * np.abs(u).max()
        return
    assert _fast_error(exact) > 1e-6, name
