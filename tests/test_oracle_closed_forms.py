"""Pins of the oracle's closed forms against what the paper and mathematics fix.

* Each pair-mobility closed form equals its spectral definition (App. A):
  a 1-D Fourier-Bessel integral evaluated by quadrature, independent of the
  closed form.
* Far-field limits (Oseen tensor, rotlet) and the single-particle identities
  a = sigma sqrt(pi) => S(0; sigma sqrt2) = 1/(6 pi eta a) (Sec. 2) and
  sigma_D => P(0; sigma_D sqrt2)/2 = 1/(8 pi eta a^3) (Sec. 3.4).
* The r -> 0 limits of the corrections equal the printed App. B scalars.
* The fast-FCM splitting function is in (0, 1] and non-increasing (Sec. 3.3).
* The stored cut-off of the 64-sphere workload is reproduced.
"""

import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import spherical_jn

from oracle import closed_forms as cf
from oracle import derive

A = 1.0
SIG = A / math.sqrt(math.pi)
SIG_D = A / (6.0 * math.sqrt(math.pi)) ** (1.0 / 3.0)
ETA = 1.3   # a non-unit viscosity catches a dropped 1/eta


def _radial(fun, r, kmax):
    """int_0^kmax fun(k) dk by adaptive quadrature split at Bessel periods."""
    edges = np.linspace(0.0, kmax, int(kmax * r / np.pi) + 8)
    tot = 0.0
    for a0, b0 in zip(edges[:-1], edges[1:]):
        v, _ = integrate.quad(fun, a0, b0, epsabs=1e-16, epsrel=1e-13, limit=200)
        tot += v
    return tot


def spectral_tensor(r, weight, kpow):
    """(1/2 pi^2) int k^kpow w(k) [(j0 - j1/(kr)) I + j2 xx] dk at x = r e_hat,
    returned as the (A, B) coefficients of A I + B xhat xhat^T.

    This is (2 pi)^-3 int exp(i k.x) w(k) k^(kpow-2) (I - k^ k^^T) d^3k with the
    angular integral done analytically."""
    kmax = 40.0
    fa = lambda k: k ** kpow * weight(k) * (spherical_jn(0, k * r) - spherical_jn(1, k * r) / (k * r))
    fb = lambda k: k ** kpow * weight(k) * spherical_jn(2, k * r)
    return _radial(fa, r, kmax) / (2 * np.pi ** 2), _radial(fb, r, kmax) / (2 * np.pi ** 2)


def spectral_rot(r, weight, kpow):
    """(1/4 pi^2) int k^kpow w(k) j1(kr) dk: the coefficient c with
    (2 pi)^-3 int exp(i k.x) w(k) k^(kpow-2) (i k x) d^3k / 2 = -c (xhat x)."""
    kmax = 40.0
    f = lambda k: k ** kpow * weight(k) * spherical_jn(1, k * r)
    return _radial(f, r, kmax) / (4 * np.pi ** 2)


def _AB(Mx):
    """Coefficients of A I + B xhat xhat^T for x along (1,1,1)/sqrt3."""
    # at xhat = (1,1,1)/sqrt3: diag = A + B/3, offdiag = B/3
    off = Mx[0, 1]
    return Mx[0, 0] - off, 3.0 * off


DIAG = np.ones(3) / math.sqrt(3.0)
RADII = [0.3, 1.0, 2.5, 6.0]


@pytest.mark.parametrize("r", RADII)
@pytest.mark.parametrize("s", [0.8, 1.6])
def test_S_Q_T_match_fourier_definition(r, s):
    w = lambda k: np.exp(-0.5 * s * s * k * k) / ETA
    x = r * DIAG
    for fun, kp in ((cf.S, 0), (cf.Q, 2), (cf.T, 4)):
        A_, B_ = _AB(fun(x, s, ETA))
        a_ref, b_ref = spectral_tensor(r, w, kp)
        sign = -1.0 if kp == 2 else 1.0        # Q: transform of lap is -k^2
        scale = max(abs(a_ref), abs(b_ref), 1e-30)
        assert abs(A_ - sign * a_ref) < 1e-11 * scale + 1e-15, (fun.__name__, A_, sign * a_ref)
        assert abs(B_ - sign * b_ref) < 1e-11 * scale + 1e-15, (fun.__name__, B_, sign * b_ref)


@pytest.mark.parametrize("r", RADII)
@pytest.mark.parametrize("s", [0.7, 1.5])
def test_P_matches_fourier_definition(r, s):
    # vorticity of the flow of (1/2) curl(T Delta): (1/2 eta) (I - k^k^) Delta^(k)
    w = lambda k: 0.5 * np.exp(-0.5 * s * s * k * k) / ETA
    A_, B_ = _AB(cf.P(r * DIAG, s, ETA))
    a_ref, b_ref = spectral_tensor(r, w, 2)
    scale = max(abs(a_ref), abs(b_ref))
    assert abs(A_ - a_ref) < 1e-11 * scale and abs(B_ - b_ref) < 1e-11 * scale


@pytest.mark.parametrize("r", RADII)
@pytest.mark.parametrize("s", [0.7, 1.5])
def test_R_and_K_match_fourier_definition(r, s):
    # Omega = (1/2) i k x u^,  u^ = (I - k^k^) F w / (eta k^2)
    w = lambda k: np.exp(-0.5 * s * s * k * k) / ETA
    x = r * DIAG
    F = np.array([0.3, -1.1, 0.7])
    for fun, kp in ((cf.R, 1), (cf.K, 3)):
        got = fun(x, s, ETA) @ F
        c = spectral_rot(r, w, kp)
        ref = -c * np.cross(DIAG, F) * (-1.0 if kp == 3 else 1.0)
        assert np.allclose(got, ref, rtol=0, atol=1e-11 * np.abs(ref).max() + 1e-15), (fun.__name__, got, ref)


def test_far_field_limits():
    x = np.array([7.0, -3.0, 11.0])
    s = 0.5
    # beyond the Gaussian the flow is the Stokeslet plus its degenerate quadrupole
    assert np.allclose(cf.S(x, s, ETA), cf.oseen(x, ETA) + 0.5 * s * s * cf.lap_oseen(x, ETA),
                       rtol=1e-14, atol=0)
    r = np.linalg.norm(x)
    rotlet = cf.cross_matrix(x) / (8 * np.pi * ETA * r ** 3)
    assert np.allclose(cf.R(x, s, ETA), rotlet, rtol=1e-14, atol=0)
    # P -> (3 xx - I)/(8 pi eta r^3): the rotation field of a point rotlet, doubled
    xh = x / r
    assert np.allclose(cf.P(x, s, ETA), (3 * np.outer(xh, xh) - np.eye(3)) / (8 * np.pi * ETA * r ** 3),
                       rtol=1e-13, atol=0)


def test_single_particle_mobilities():
    # near r = 0 the closed forms cancel like 1/r^2; 1e-3 sigma keeps ~1e-9
    x = 1e-3 * SIG * DIAG
    # (the approach to the limit is quadratic in r: ~1e-7 here)
    assert np.abs(cf.fcm_pair_VF(x, SIG, ETA) * (6 * np.pi * ETA * A) - np.eye(3)).max() < 1e-6
    assert np.abs(cf.fcm_pair_OT(x, SIG_D, ETA) * (8 * np.pi * ETA * A ** 3) - np.eye(3)).max() < 1e-6


@pytest.mark.parametrize("ratio", [1.5, 2.0, 4.0])
def test_self_corrections_are_limits_of_pair_corrections(ratio):
    """App. B scalars are the r -> 0 limits; the approach is quadratic in r, so a
    Richardson step from r = 2e-3 sigma and 1e-3 sigma removes the r^2 term."""
    Sg = ratio * SIG

    def lim(fun):
        f1 = fun(2e-3 * SIG * DIAG)
        f2 = fun(1e-3 * SIG * DIAG)
        return (4.0 * f2 - f1) / 3.0

    lim_vf = lim(lambda x: cf.correction_VF(x, SIG, Sg, ETA))
    lim_ot = lim(lambda x: cf.correction_OT(x, SIG_D, Sg, ETA))
    ref_vf = cf.self_correction_VF(A, SIG, Sg, ETA)
    ref_ot = cf.self_correction_OT(A, Sg, ETA)
    assert np.abs(lim_vf - ref_vf * np.eye(3)).max() < 1e-7 * abs(ref_vf)
    assert np.abs(lim_ot - ref_ot * np.eye(3)).max() < 1e-7 * abs(ref_ot)
    # the Omega-F correction is odd in x and vanishes linearly at r = 0
    o1 = cf.correction_OF(1e-3 * SIG * DIAG, SIG, SIG_D, Sg, Sg, ETA)
    o2 = cf.correction_OF(2e-3 * SIG * DIAG, SIG, SIG_D, Sg, Sg, ETA)
    assert np.abs(o2 - 2.0 * o1).max() < 1e-5 * np.abs(o2).max()


@pytest.mark.parametrize("r", [0.6, 2.0, 5.0])
def test_corrections_match_split_fourier_form(r):
    """M - M~ equals the spectral integral with weight
    exp(-sigma^2 k^2) - (1 - (sigma^2-Sigma^2) k^2/2)^2 exp(-Sigma^2 k^2)
    (Sec. 3.3: the transform of Delta~ is (1 - (sigma^2-Sigma^2) k^2/2) times
    that of Delta(.; Sigma))."""
    Sg = 2.3 * SIG
    SD = 1.7 * SIG_D
    c = 0.5 * (SIG ** 2 - Sg ** 2)
    x = r * DIAG
    wvf = lambda k: (np.exp(-SIG ** 2 * k * k) - (1 - c * k * k) ** 2 * np.exp(-Sg ** 2 * k * k)) / ETA
    a_ref, b_ref = spectral_tensor(r, wvf, 0)
    A_, B_ = _AB(cf.correction_VF(x, SIG, Sg, ETA))
    sc = max(abs(a_ref), abs(b_ref))
    assert abs(A_ - a_ref) < 1e-10 * sc and abs(B_ - b_ref) < 1e-10 * sc
    wot = lambda k: 0.25 * (np.exp(-SIG_D ** 2 * k * k) - np.exp(-SD ** 2 * k * k)) / ETA
    a_ref, b_ref = spectral_tensor(r, wot, 2)
    A_, B_ = _AB(cf.correction_OT(x, SIG_D, SD, ETA))
    sc = max(abs(a_ref), abs(b_ref))
    assert abs(A_ - a_ref) < 1e-10 * sc and abs(B_ - b_ref) < 1e-10 * sc
    wof = lambda k: (np.exp(-0.5 * (SIG ** 2 + SIG_D ** 2) * k * k)
                     - (1 - c * k * k) * np.exp(-0.5 * (Sg ** 2 + SD ** 2) * k * k)) / ETA
    F = np.array([1.0, 0.2, -0.4])
    cref = spectral_rot(r, wof, 1)
    got = cf.correction_OF(x, SIG, SIG_D, Sg, SD, ETA) @ F
    ref = -cref * np.cross(DIAG, F)
    assert np.allclose(got, ref, rtol=0, atol=1e-10 * np.abs(ref).max())
    # V-T correction is the transpose relation of Sec. 3.4
    assert np.allclose(cf.correction_VT(x, SIG, SIG_D, Sg, SD, ETA),
                       cf.correction_OF(-x, SIG, SIG_D, Sg, SD, ETA).T, rtol=1e-14, atol=0)


def test_corrections_decay_and_are_symmetric():
    Sg = 2.0 * SIG
    x = np.array([3.0, -1.0, 2.0])
    C = cf.correction_VF(x, SIG, Sg, ETA)
    assert np.allclose(C, C.T, rtol=1e-14, atol=0)
    assert np.allclose(C, cf.correction_VF(-x, SIG, Sg, ETA), rtol=1e-14, atol=0)
    near = np.abs(cf.correction_VF(3.0 * DIAG, SIG, Sg, ETA)).max()
    far = np.abs(cf.correction_VF(12.0 * DIAG, SIG, Sg, ETA)).max()
    assert far < 1e-8 * near


def test_splitting_function_positive_and_monotone():
    for ratio in (1.2, 2.0, 5.0):
        Sg = ratio * SIG
        k = np.linspace(0.0, np.sqrt(600.0 / (Sg ** 2 - SIG ** 2)), 20001)   # H > 1e-250
        d = SIG ** 2 - Sg ** 2
        p = 1 - d * k * k + 0.25 * d * d * k ** 4
        H = p * np.exp(-(Sg ** 2 - SIG ** 2) * k * k)
        # H is the squared ratio of the kernel transforms (Sec. 3.3)
        ratio_t = (1 - 0.5 * d * k * k) * np.exp(-0.5 * (Sg ** 2 - SIG ** 2) * k * k)
        assert np.allclose(H, ratio_t ** 2, rtol=1e-12, atol=1e-300)
        assert H[0] == 1.0 and np.all(H[1:] > 0) and np.all(H[1:] <= 1.0)
        assert np.all(np.diff(H) <= 1e-15)


def test_stored_small_workload_cutoff():
    import workloads
    rc = derive.cutoff_for_tolerance(A, 2.0 * SIG, 1e-10, 19.9)
    assert abs(rc - workloads.C1_RCUT) < 1e-7
    assert derive.scaled_correction(rc * 1.001, A, 2.0 * SIG) < 1e-10
    assert derive.scaled_correction(rc * 0.99, A, 2.0 * SIG) > 1e-10
