"""Closed-form FCM pair mobilities and fast-FCM corrections, plain FP64.

TEST INFRASTRUCTURE ONLY (see the package header).

Conventions.  ``x`` is an array of separation vectors of shape (..., 3) with
x = Y_n - Y_m; every function returns the 3x3 blocks, shape (..., 3, 3), that
map the force (or torque) on particle m to the velocity (or angular velocity)
of particle n.  ``Delta(r; s) = (2 pi s^2)^(-3/2) exp(-r^2 / 2 s^2)`` is the
FCM Gaussian of Sec. 2.  ``eta`` is the viscosity.

The forms follow Sec. 2.2 (S, Q, G), Sec. 3.2 (T) and Sec. 3.4 (R, K, P).
Readings of garbled passages, each checked by the pins in tests/:

* correction_VF (Sec. 3.2): the error-function arguments are those of
  S(x; sigma*sqrt 2), i.e. erf(r / 2 sigma) and erf(r / 2 Sigma).  This module
  does not use the printed expanded form at all: the correction is written as
  the plain difference of the pair mobilities, M - M~, which is its definition.
* correction_WT (Sec. 3.4) carries the factor 1/2 of M^{Omega T} = P/2.
* R is half the vorticity (the local rotation rate) of the Gaussian-force flow
  and P is the full vorticity of the Gaussian-torque flow; M^{Omega T} = P/2.
"""

import numpy as np
from scipy.special import erf


def gaussian(r, s):
    """FCM Gaussian Delta(r; s) (Sec. 2, first equation)."""
    return (2.0 * np.pi * s * s) ** -1.5 * np.exp(-r * r / (2.0 * s * s))


def _geometry(x):
    x = np.asarray(x, dtype=np.float64)
    r = np.sqrt(np.sum(x * x, axis=-1))
    xhat = x / r[..., None]
    I = np.broadcast_to(np.eye(3), x.shape[:-1] + (3, 3))
    xx = xhat[..., :, None] * xhat[..., None, :]
    return x, r, I, xx


def cross_matrix(x):
    """The matrix (-x cross) of Sec. 3.4: rows (0,x3,-x2), (-x3,0,x1), (x2,-x1,0).

    Applied to a vector F it gives F x x.
    """
    x = np.asarray(x, dtype=np.float64)
    z = np.zeros(x.shape[:-1])
    x1, x2, x3 = x[..., 0], x[..., 1], x[..., 2]
    return np.stack([np.stack([z, x3, -x2], -1),
                     np.stack([-x3, z, x1], -1),
                     np.stack([x2, -x1, z], -1)], -2)


def oseen(x, eta=1.0):
    """Oseen tensor G (Sec. 2.2)."""
    x, r, I, xx = _geometry(x)
    return (I + xx) / (8.0 * np.pi * eta * r)[..., None, None]


def lap_oseen(x, eta=1.0):
    """Laplacian of the Oseen tensor, (1/4 pi eta r^3)(I - 3 xx/r^2) (Sec. 2.2)."""
    x, r, I, xx = _geometry(x)
    return (I - 3.0 * xx) / (4.0 * np.pi * eta * r ** 3)[..., None, None]


def S(x, s, eta=1.0):
    """Flow of a Gaussian force of width s: S = S1 + S2 + S3 (eqs. S1-S3)."""
    x, r, I, xx = _geometry(x)
    E = erf(r / (s * np.sqrt(2.0)))[..., None, None]
    D = gaussian(r, s)[..., None, None]
    rr = r[..., None, None]
    S1 = (I + xx) * E / (8.0 * np.pi * eta * rr)
    S2 = (I - 3.0 * xx) * s * s * E / (8.0 * np.pi * eta * rr ** 3)
    S3 = -(s * s / (2.0 * eta)) * (I - 3.0 * xx) * (s * s / rr ** 2) * D
    return S1 + S2 + S3


def S3_part(x, s, eta=1.0):
    """The Gaussian term S3 alone (eq. S3)."""
    x, r, I, xx = _geometry(x)
    D = gaussian(r, s)[..., None, None]
    rr = r[..., None, None]
    return -(s * s / (2.0 * eta)) * (I - 3.0 * xx) * (s * s / rr ** 2) * D


def Q(x, s, eta=1.0):
    """Flow of the force distribution H lap Delta(x; s): Q = Q1 + Q2 (eqs. Q1, Q2)."""
    x, r, I, xx = _geometry(x)
    E = erf(r / (s * np.sqrt(2.0)))[..., None, None]
    D = gaussian(r, s)[..., None, None]
    rr = r[..., None, None]
    Q1 = (I - 3.0 * xx) * E / (4.0 * np.pi * eta * rr ** 3)
    Q2 = -((1.0 + s * s / rr ** 2) * I - (1.0 + 3.0 * s * s / rr ** 2) * xx) * D / eta
    return Q1 + Q2


def T(x, s, eta=1.0):
    """The bi-Laplacian term T of the modified pair mobility (Sec. 3.2)."""
    x, r, I, xx = _geometry(x)
    D = gaussian(r, s)[..., None, None]
    xxT = x[..., :, None] * x[..., None, :]
    rr = r[..., None, None]
    return (2.0 * I + (xxT - rr ** 2 * I) / (s * s)) * D / (eta * s * s)


def R(x, s, eta=1.0):
    """Rotation rate of the Gaussian-force flow, eq. R (Sec. 3.4)."""
    x, r, I, xx = _geometry(x)
    E = erf(r / (s * np.sqrt(2.0)))
    D = gaussian(r, s)
    f = (E - 4.0 * np.pi * r * s * s * D) / (8.0 * np.pi * eta * r ** 3)
    return f[..., None, None] * cross_matrix(x)


def K(x, s, eta=1.0):
    """K = lap R, eq. V of Sec. 3.4: -(1/2 s^2 eta) Delta(x; s) (-x cross)."""
    x, r, I, xx = _geometry(x)
    D = gaussian(r, s)
    return (-D / (2.0 * s * s * eta))[..., None, None] * cross_matrix(x)


def P(x, s, eta=1.0):
    """Vorticity of the Gaussian-torque flow: P = P1 + P2 (eqs. P1, P2)."""
    x, r, I, xx = _geometry(x)
    E = erf(r / (s * np.sqrt(2.0)))[..., None, None]
    D = gaussian(r, s)[..., None, None]
    rr = r[..., None, None]
    P1 = (-I + 3.0 * xx) * E / (8.0 * np.pi * eta * rr ** 3)
    P2 = ((s * s + rr ** 2) * I - (3.0 * s * s + rr ** 2) * xx) * D / (2.0 * eta * rr ** 2)
    return P1 + P2


# --- FCM pair mobilities (eq. M_VF, Sec. 3.4, App. A) ---------------------

def fcm_pair_VF(x, sigma, eta=1.0):
    """M^{VF}_{nm} = S(Y_n - Y_m; sigma sqrt 2) (eq. M_VF)."""
    return S(x, sigma * np.sqrt(2.0), eta)


def fcm_pair_OF(x, sigma, sigma_D, eta=1.0):
    """M^{Omega F}_{nm} = R(Y_n - Y_m; sqrt(sigma^2 + sigma_D^2)) (Sec. 3.4)."""
    return R(x, np.sqrt(sigma ** 2 + sigma_D ** 2), eta)


def fcm_pair_VT(x, sigma, sigma_D, eta=1.0):
    """M^{VT}_{nm} = (M^{Omega F}_{mn})^T (Sec. 3.4), evaluated from -x."""
    return np.swapaxes(fcm_pair_OF(-np.asarray(x, dtype=np.float64), sigma, sigma_D, eta), -1, -2)


def fcm_pair_OT(x, sigma_D, eta=1.0):
    """M^{Omega T}_{nm} = P(Y_n - Y_m; sigma_D sqrt 2) / 2 (Sec. 3.4)."""
    return 0.5 * P(x, sigma_D * np.sqrt(2.0), eta)


# --- modified (grid) pair mobilities: the part fast FCM puts on the grid ----

def modified_pair_VF(x, sigma, Sigma, eta=1.0):
    """M~^{VF}_{nm} = S(Sigma sqrt2) + (sigma^2-Sigma^2) Q(Sigma sqrt2)
    + ((sigma^2-Sigma^2)^2/4) T(Sigma sqrt2) (Sec. 3.2)."""
    s2 = Sigma * np.sqrt(2.0)
    d = sigma ** 2 - Sigma ** 2
    return S(x, s2, eta) + d * Q(x, s2, eta) + 0.25 * d * d * T(x, s2, eta)


def modified_pair_OF(x, sigma, Sigma, Sigma_D, eta=1.0):
    """M~^{Omega F}_{nm} = R(st) + ((sigma^2-Sigma^2)/2) K(st),
    st = sqrt(Sigma^2 + Sigma_D^2) (eq. correction_WF read as M - M~)."""
    st = np.sqrt(Sigma ** 2 + Sigma_D ** 2)
    return R(x, st, eta) + 0.5 * (sigma ** 2 - Sigma ** 2) * K(x, st, eta)


def modified_pair_OT(x, Sigma_D, eta=1.0):
    """M~^{Omega T}_{nm} = P(Sigma_D sqrt 2) / 2 (Sec. 3.4)."""
    return 0.5 * P(x, Sigma_D * np.sqrt(2.0), eta)


# --- corrections M - M~ (eqs. correction_VF, correction_WF, correction_WT) ---

def correction_VF(x, sigma, Sigma, eta=1.0):
    """M^{VF} - M~^{VF} (eq. correction_VF), as the difference of definitions."""
    return fcm_pair_VF(x, sigma, eta) - modified_pair_VF(x, sigma, Sigma, eta)


def correction_OF(x, sigma, sigma_D, Sigma, Sigma_D, eta=1.0):
    """M^{Omega F} - M~^{Omega F} (eq. correction_WF)."""
    return fcm_pair_OF(x, sigma, sigma_D, eta) - modified_pair_OF(x, sigma, Sigma, Sigma_D, eta)


def correction_VT(x, sigma, sigma_D, Sigma, Sigma_D, eta=1.0):
    """M^{VT} - M~^{VT}: the transpose relation of Sec. 3.4 applied to both parts."""
    xm = -np.asarray(x, dtype=np.float64)
    return np.swapaxes(correction_OF(xm, sigma, sigma_D, Sigma, Sigma_D, eta), -1, -2)


def correction_OT(x, sigma_D, Sigma_D, eta=1.0):
    """M^{Omega T} - M~^{Omega T} = [P(sigma_D sqrt2) - P(Sigma_D sqrt2)] / 2
    (eq. correction_WT with the factor 1/2 of M^{Omega T} = P/2)."""
    return fcm_pair_OT(x, sigma_D, eta) - modified_pair_OT(x, Sigma_D, eta)


def self_correction_VF(a, sigma, Sigma, eta=1.0):
    """r -> 0 limit of correction_VF (App. B, eq. correction_VF_limit); times I."""
    sp = Sigma * np.sqrt(np.pi)
    d = sigma ** 2 - Sigma ** 2
    return (1.0 / (6.0 * np.pi * eta * a) - 1.0 / (6.0 * np.pi * eta * sp)
            + d / (12.0 * eta * sp ** 3) - d * d / (32.0 * eta * Sigma ** 5 * np.pi ** 1.5))


def self_correction_OT(a, Sigma_D, eta=1.0):
    """r -> 0 limit of correction_WT (App. B, eq. correction_WT_limit); times I.

    The printed limit is written with Sigma; it is the torque-kernel width
    Sigma_D (equal to Sigma in the paper's runs) that enters it.
    """
    return 1.0 / (8.0 * np.pi * eta * a ** 3) - 1.0 / (48.0 * eta * (Sigma_D * np.sqrt(np.pi)) ** 3)
