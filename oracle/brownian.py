"""Brownian velocities of fast FCM, plain FP64 (test infrastructure only).

The positive splitting of Sec. 3.3 (the grid part M~ and the correction
M - M~ are both symmetric positive definite) is what makes fast FCM usable
for Brownian simulations (Sec. 3.3, Sec. 7): a velocity with covariance
2 kT M is the sum of independent draws with covariances 2 kT M~ (fluctuating
FCM on the grid) and 2 kT (M - M~) (a square root of the pair correction,
which the GPU path approximates by the Lanczos method, Sec. 7).  This module
takes the random numbers as inputs and covers force-free particles' velocity
part only (the VF block; the torque-coupled correction is not shown positive
by the paper).

Grid part.  With the discrete mobility M~_h = dV W G W^T (W the kernel
weights Delta~ at the grid points, dV = dx^3, G the grid Stokes solve
IFFT[P(k) / (eta k^2) FFT[.]], P = I - k k^T / k^2, k = 0 and the Nyquist
planes removed), a unit-variance real field xi on the grid gives
    V_grid = sqrt(2 kT / dV) * dV W G^(1/2) xi,   G^(1/2) = IFFT[P(k) / sqrt(eta k^2) FFT[.]]
whose covariance is 2 kT dV W G W^T = 2 kT M~_h (P^2 = P).

Pair part.  The 3N x 3N matrix C of the VF pair corrections (closed forms of
Sec. 3.2 for pairs closer than R_c, plus the self term of App. B on the
diagonal); V_pair = sqrt(2 kT) C^(1/2) xi_p with the symmetric square root from
an eigendecomposition.
"""

import numpy as np

from . import closed_forms as cf
from .fastfcm import interp, min_image, wrap


def grid_sqrt_solve(p, xi, workers=None):
    """G^(1/2) xi on the grid: xi and the result have shape (3, Mx, My, Mz).
    ``workers``: None uses numpy's FFT (one thread); a number uses scipy's FFT
    with that many threads (the same transform, for the largest grids)."""
    if workers is None:
        fftn, ifftn = np.fft.fftn, np.fft.ifftn
    else:
        import scipy.fft as sfft
        fftn = lambda a, axes: sfft.fftn(a, axes=axes, workers=workers)
        ifftn = lambda a, axes: sfft.ifftn(a, axes=axes, workers=workers)
    fh = fftn(np.asarray(xi, dtype=np.float64), axes=(1, 2, 3))
    Mx, My, Mz = p.Mv
    kx = (2.0 * np.pi * np.fft.fftfreq(Mx, d=1.0 / Mx) / p.Lv[0])[:, None, None]
    ky = (2.0 * np.pi * np.fft.fftfreq(My, d=1.0 / My) / p.Lv[1])[None, :, None]
    kz = (2.0 * np.pi * np.fft.fftfreq(Mz, d=1.0 / Mz) / p.Lv[2])[None, None, :]
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    k2s = np.where(k2 == 0.0, 1.0, k2)
    kdotf = (kx * fh[0] + ky * fh[1] + kz * fh[2]) / k2s
    s = 1.0 / np.sqrt(p.eta * k2s)
    uh = np.empty_like(fh)
    uh[0] = (fh[0] - kx * kdotf) * s
    uh[1] = (fh[1] - ky * kdotf) * s
    uh[2] = (fh[2] - kz * kdotf) * s
    uh[:, 0, 0, 0] = 0.0
    if Mx % 2 == 0:
        uh[:, Mx // 2, :, :] = 0.0
    if My % 2 == 0:
        uh[:, :, My // 2, :] = 0.0
    if Mz % 2 == 0:
        uh[:, :, :, Mz // 2] = 0.0
    return np.real(ifftn(uh, axes=(1, 2, 3)))


def brownian_grid(p, Y, xi, kT, workers=None):
    """sqrt(2 kT / dV) J~[G^(1/2) xi] at the particles (N x 3)."""
    V, _ = interp(p, Y, grid_sqrt_solve(p, xi, workers), want_omega=False)
    return np.sqrt(2.0 * kT / p.dx ** 3) * V


def pair_matrix(p, Y):
    """The 3N x 3N VF correction matrix: correction_VF(Y_n - Y_m) for pairs
    with minimum-image distance < R_c (Sec. 3.2), self term c_VF I (App. B)
    on the diagonal blocks."""
    Yw = wrap(Y, p.Lv)
    N = len(Yw)
    C = np.zeros((3 * N, 3 * N))
    cvf = cf.self_correction_VF(p.a, p.sigma, p.Sigma, p.eta)
    for n in range(N):
        C[3 * n:3 * n + 3, 3 * n:3 * n + 3] += cvf * np.eye(3)
        if p.R_c <= 0.0:
            continue
        x = min_image(Yw[n][None, :] - Yw, p.Lv)
        r = np.sqrt(np.sum(x * x, axis=1))
        for m in np.nonzero((r < p.R_c) & (np.arange(N) != n))[0]:
            C[3 * n:3 * n + 3, 3 * m:3 * m + 3] = cf.correction_VF(x[m][None, :], p.sigma, p.Sigma, p.eta)[0]
    return C


def sqrt_spd(C):
    """Symmetric square root of a symmetric positive semi-definite matrix."""
    w, Q = np.linalg.eigh(0.5 * (C + C.T))
    return (Q * np.sqrt(np.clip(w, 0.0, None))) @ Q.T


def brownian_pair(p, Y, xi_p, kT):
    """sqrt(2 kT) C^(1/2) xi_p (N x 3)."""
    C = pair_matrix(p, Y)
    return (np.sqrt(2.0 * kT) * sqrt_spd(C) @ np.asarray(xi_p, dtype=np.float64).ravel()).reshape(-1, 3)


def brownian(p, Y, xi_grid, xi_pair, kT):
    """Brownian velocities V_grid + V_pair with covariance 2 kT M (VF block)."""
    return brownian_grid(p, Y, xi_grid, kT) + brownian_pair(p, Y, xi_pair, kT)
