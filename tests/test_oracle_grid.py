"""Pins of the oracle's grid pipeline and of the whole fast-FCM algorithm.

Each test checks the oracle against something other than itself:

* the Fourier Stokes solve against a brute-force discrete Fourier sum, and its
  closed form for single Fourier modes (which the GPU tests use on grids too
  large for the oracle's full solve) against the solve itself;
* spreading against the moment identities of the kernels (total force, and
  first moment x cross f = T, which fixes the sign of the torque spreading,
  Sec. 3.4);
* the assembled grid mobility against exact invariants: symmetry and positive
  semi-definiteness (spreading and interpolation are adjoint, Sec. 3.3), zero
  fluid mean;
* the grid part against the exact periodic lattice sum of the modified kernel;
* full fast FCM against the exact periodic FCM lattice sum (the plain
  definition it approximates, Sec. 3) to the tolerance of Tables 1-2;
* independence of the result from Sigma (Sec. 3, Sec. 5.2);
* a single sphere against Hasimoto's periodic drag (constant recomputed here
  by an independent Ewald sum) and the exact periodic rotation mobility;
* cell-list pair search against brute force over all pairs.
"""

import math
import zlib

import numpy as np
import pytest
from scipy.special import erfc

from oracle import fastfcm as ff
from oracle import lattice

A = 1.0
SIG = A / math.sqrt(math.pi)
SIG_D = A / (6.0 * math.sqrt(math.pi)) ** (1.0 / 3.0)


def _random_config(N, L, seed, min_sep=2.0):
    rng = np.random.default_rng(seed)
    Y = []
    while len(Y) < N:
        p = rng.uniform(0, L, 3)
        ok = True
        for q in Y:
            d = p - q
            d -= L * np.round(d / L)
            if np.linalg.norm(d) < min_sep:
                ok = False
        if ok:
            Y.append(p)
    return np.array(Y)


def _assemble(p, Y, grid_only=False):
    """6N x 6N matrix of the oracle's map (F, T) -> (V, Omega) by unit solves."""
    N = len(Y)
    Mat = np.zeros((6 * N, 6 * N))
    for col in range(6 * N):
        F = np.zeros((N, 3))
        T = np.zeros((N, 3))
        if col < 3 * N:
            F.flat[col] = 1.0
        else:
            T.flat[col - 3 * N] = 1.0
        if grid_only:
            u = ff.stokes_solve(p, ff.spread(p, Y, F, T))
            V, W = ff.interp(p, Y, u)
        else:
            V, W = ff.mobility(p, Y, F, T)
        Mat[:3 * N, col] = V.ravel()
        Mat[3 * N:, col] = W.ravel()
    return Mat


def _dft_stokes(p, f):
    """u = L^{-1} f by explicit O(M^6) discrete Fourier sums (plain definition)."""
    M = p.M
    g = np.arange(M)
    xg = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) * p.dx
    j = np.fft.fftfreq(M, 1.0 / M)
    J = np.stack(np.meshgrid(j, j, j, indexing="ij"), -1).reshape(-1, 3)
    keep = np.all(np.abs(J) != M / 2.0, axis=1) & np.any(J != 0, axis=1)
    k = 2 * np.pi * J[keep] / p.L
    E = np.exp(-1j * (k @ xg.T))                       # (modes, points)
    fh = E @ f.reshape(3, -1).T                          # (modes, 3)
    k2 = np.sum(k * k, 1)
    uh = (fh - k * (np.sum(k * fh, 1) / k2)[:, None]) / (p.eta * k2[:, None])
    u = (np.conj(E).T @ uh).real / M ** 3
    return u.T.reshape(3, M, M, M)


@pytest.mark.parametrize("M", [6, 7])
def test_stokes_solve_equals_direct_fourier_sum(M):
    p = ff.Params(L=5.0, M=M, a=A, Sigma=0.8, M_G=4, R_c=0.0, eta=1.7)
    f = np.random.default_rng(1).normal(size=(3, M, M, M))
    u = ff.stokes_solve(p, f)
    assert np.allclose(u, _dft_stokes(p, f), rtol=0, atol=1e-13 * np.abs(u).max())


@pytest.mark.parametrize("L,M,j", [
    (5.0, 12, (1, 0, 0)), (5.0, 12, (5, -3, 2)), (5.0, 18, (0, 0, -8)),
    ((6.0, 4.0, 3.0), (24, 16, 12), (11, -7, 5)), ((6.0, 4.0, 3.0), (24, 16, 12), (-2, 0, 1)),
])
def test_plane_wave_closed_form_equals_solve(L, M, j):
    """A sum of one mode's closed-form solution over every grid point equals
    the Fourier solve of the sampled mode (cube and box, eta != 1, modes up to
    one below the Nyquist index)."""
    p = ff.Params(L=L, M=M, a=A, Sigma=0.8, M_G=4, R_c=0.0, eta=1.7)
    rng = np.random.default_rng(zlib.crc32(repr((L, M, j)).encode()))
    Av, phi = rng.normal(size=3), rng.uniform(0.0, 2.0 * np.pi)
    Mx, My, Mz = p.Mv
    idx = np.stack(np.meshgrid(np.arange(Mx), np.arange(My), np.arange(Mz), indexing="ij"), -1).reshape(-1, 3)
    # the forcing sampled on the grid: A cos(k.x + phi) at x = idx * dx
    k = 2.0 * np.pi * np.asarray(j) / p.Lv
    wave = np.cos((idx * p.dx) @ k + phi)
    f = (Av[:, None] * wave[None, :]).reshape(3, Mx, My, Mz)
    u = ff.stokes_solve(p, f).reshape(3, -1).T
    uc = ff.stokes_plane_wave(p, j, Av, phi, idx)
    assert np.allclose(u, uc, rtol=0, atol=1e-12 * np.abs(uc).max())
    # divergence-free amplitude and the 1/k^2 decay
    assert abs(np.sum(k * uc[0])) < 1e-12 * np.abs(uc).max() * np.sqrt(k @ k)


def test_plane_wave_rejects_zero_and_nyquist_modes():
    p = ff.Params(L=5.0, M=12, a=A, Sigma=0.8, M_G=4, R_c=0.0)
    for j in [(0, 0, 0), (6, 0, 0), (0, -6, 1)]:
        with pytest.raises(ValueError):
            ff.stokes_plane_wave(p, j, (1.0, 0.0, 0.0), 0.0, np.zeros((1, 3), dtype=np.int64))


def _spread_fns():
    from oracle import cgrid
    return {"numpy": ff.spread, "c": cgrid.spread}


@pytest.mark.parametrize("impl", ["numpy", "c"])
def test_spread_moments_fix_normalisation_and_torque_sign(impl):
    spread = _spread_fns()[impl]
    L, M = 12.0, 32
    Sg = 1.5 * L / M                     # Sigma / dx = 1.5; M_G = 24 cuts at 8 Sigma: e^-32
    p = ff.Params(L=L, M=M, a=A, Sigma=Sg, M_G=24, R_c=0.0)
    Y = np.array([[5.31, 6.07, 4.66]])
    dV = p.dx ** 3
    g = np.arange(M) * p.dx
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), 0)
    F = np.array([[0.4, -1.2, 0.9]])
    f = spread(p, Y, F, None)
    assert np.allclose(dV * f.reshape(3, -1).sum(1), F[0], rtol=0, atol=1e-10)
    T = np.array([[-0.7, 0.3, 1.1]])
    f = spread(p, Y, np.zeros((1, 3)), T)
    d = X - Y[0][:, None, None, None]
    d -= L * np.round(d / L)
    mom = dV * np.cross(d.reshape(3, -1).T, f.reshape(3, -1).T).sum(0)
    assert np.allclose(mom, T[0], rtol=0, atol=1e-10)          # int x cross f = T
    assert abs(dV * f.sum()) < 1e-12                             # no net force


@pytest.mark.parametrize("L,M,MG,Sigma_D,torque", [
    (20.0, 16, 10, None, True),
    ((30.0, 12.0, 18.0), (40, 16, 24), 9, 0.9, True),    # box, odd support, Sigma_D != Sigma
    (17.0, 27, 8, None, False),                         # odd grid, no torques
    (10.0, 12, 12, None, True),                         # support = grid: every axis wraps
], ids=["cube", "box-oddMG-SigmaD", "odd-grid-noT", "support-equals-grid"])
def test_c_spread_equals_numpy_spread(L, M, MG, Sigma_D, torque):
    """The C spreading used for the largest request-stream grids is the same
    operator as the numpy oracle's (positions up to two boxes outside)."""
    spread = _spread_fns()
    p = ff.Params(L=L, M=M, a=A, Sigma=0.8, M_G=MG, R_c=3.0, Sigma_D=Sigma_D)
    rng = np.random.default_rng(31)
    Y = rng.uniform(-25.0, 45.0, (40, 3))
    F = rng.normal(size=(40, 3))
    T = rng.normal(size=(40, 3)) if torque else None
    a = spread["numpy"](p, Y, F, T)
    b = spread["c"](p, Y, F, T)
    assert np.abs(a - b).max() < 1e-14 * np.abs(a).max()


def test_threaded_fft_solve_equals_numpy_solve():
    p = ff.Params(L=(30.0, 20.0, 25.0), M=(30, 20, 25), a=A, Sigma=1.0, M_G=10, R_c=0.0)
    f = np.random.default_rng(5).normal(size=(3, 30, 20, 25))
    a = ff.stokes_solve(p, f)
    b = ff.stokes_solve(p, f, workers=4)
    assert np.abs(a - b).max() < 1e-14 * np.abs(a).max()


def test_grid_mobility_symmetric_psd_and_fluid_mean_zero():
    L, M = 14.0, 16
    p = ff.Params(L=L, M=M, a=A, Sigma=1.3 * L / M, M_G=10, R_c=0.0)
    Y = _random_config(4, L, seed=3)
    Mh = _assemble(p, Y, grid_only=True)
    assert np.abs(Mh - Mh.T).max() < 1e-13 * np.abs(Mh).max()
    ev = np.linalg.eigvalsh(0.5 * (Mh + Mh.T))
    assert ev.min() > -1e-13 * ev.max()
    rng = np.random.default_rng(9)
    u = ff.stokes_solve(p, ff.spread(p, Y, rng.normal(size=(4, 3)), rng.normal(size=(4, 3))))
    assert np.abs(u.reshape(3, -1).mean(1)).max() < 1e-15 * np.abs(u).max()


def test_grid_part_converges_to_modified_lattice_sum():
    """At Sigma/dx = 1.5, M_G = 20 (cut at 6.7 Sigma) the grid part equals the
    exact periodic M~ (lattice sum of the modified kernels) to ~1e-9 (Table 1
    extrapolated)."""
    L, M = 12.0, 24
    Sg = 1.5 * L / M
    p = ff.Params(L=L, M=M, a=A, Sigma=Sg, M_G=20, R_c=0.0)
    Y = _random_config(3, L, seed=5)
    Mh = _assemble(p, Y, grid_only=True)
    Mex = lattice.mobility_matrix(Y, L, A, Sigma=Sg, modified=True)
    assert np.abs(Mh - Mex).max() < 2e-8 * np.abs(Mex).max()


@pytest.fixture(scope="module")
def exact_case():
    L = 20.0
    Y = _random_config(4, L, seed=11)
    return L, Y, lattice.mobility_matrix(Y, L, A)


def _fast(L, Y, ratio, M, MG, lam):
    Sg = ratio * SIG
    p = ff.Params(L=L, M=M, a=A, Sigma=Sg, M_G=MG, R_c=lam * Sg if ratio > 1 else 0.0)
    return _assemble(p, Y)


def test_fast_fcm_matches_exact_periodic_fcm(exact_case):
    """Sigma = 2 sigma, Sigma/dx = 1.52, M_G = 20 (cut beyond 6 Sigma),
    R_c = 8.6 Sigma (Table 2, 1e-8): the full fast-FCM matrix, torque blocks
    included, matches the lattice sum of exact periodic FCM."""
    L, Y, Mex = exact_case
    Mf = _fast(L, Y, 2.0, 27, 20, 8.6)
    err = np.linalg.norm(Mf - Mex) / np.linalg.norm(Mex)
    assert err < 1e-8, err
    N3 = 3 * len(Y)
    for blk in (np.s_[:N3, :N3], np.s_[N3:, N3:], np.s_[N3:, :N3], np.s_[:N3, N3:]):
        assert np.abs(Mf[blk] - Mex[blk]).max() < 1e-6 * np.abs(Mex[blk]).max()
    # symmetric to rounding: grid part adjoint, corrections pairwise symmetric
    assert np.abs(Mf - Mf.T).max() < 1e-13 * np.abs(Mf).max()
    assert np.linalg.eigvalsh(0.5 * (Mf + Mf.T)).min() > 0


def test_results_independent_of_Sigma(exact_case):
    """Standard FCM (Sigma = sigma, no correction) and fast FCM at
    Sigma/sigma = 1.5 agree with the lattice sum, as the Sigma = 2 sigma run
    above does: the result does not depend on Sigma (Sec. 3, Sec. 5.2)."""
    L, Y, Mex = exact_case
    runs = {1.0: _fast(L, Y, 1.0, 54, 20, 0.0),
            1.5: _fast(L, Y, 1.5, 36, 20, 8.6)}
    for ratio, Mf in runs.items():
        err = np.linalg.norm(Mf - Mex) / np.linalg.norm(Mex)
        assert err < 1e-8, (ratio, err)


def hasimoto_constant():
    """C_H = -4 pi L phi_reg(0) for the simple cubic lattice by Ewald summation
    of the periodic Coulomb potential with a neutralising background; the
    trace of the periodic Stokeslet is 2/3 of it (Hasimoto 1959)."""
    L = 1.0
    alpha = math.sqrt(math.pi) / L
    n = np.arange(-6, 7)
    J = np.stack(np.meshgrid(n, n, n, indexing="ij"), -1).reshape(-1, 3)
    J = J[np.any(J != 0, axis=1)]
    k2 = np.sum((2 * np.pi * J / L) ** 2, 1)
    rec = np.sum(np.exp(-k2 / (4 * alpha ** 2)) / k2) / L ** 3
    rn = np.linalg.norm(J * L, axis=1)
    real = np.sum(erfc(alpha * rn) / (4 * np.pi * rn))
    phi = rec + real - alpha / (2 * np.pi ** 1.5) - 1.0 / (4 * alpha ** 2 * L ** 3)
    return -4 * np.pi * L * phi


def test_hasimoto_constant_value():
    assert abs(hasimoto_constant() - 2.837297) < 2e-6


@pytest.mark.parametrize("L,ratio,M,MG,lam", [(10.0, 1.0, 27, 20, 0.0), (20.0, 2.0, 27, 20, 8.6)])
def test_single_sphere_periodic_drag(L, ratio, M, MG, lam):
    """V 6 pi eta a = 1 - C_H a/L + 4 (a/L)^3 and Omega 8 pi eta a^3 =
    1 - (4 pi / 3)(a/L)^3 for FCM in a periodic cube (the Gaussian's sigma^2
    term replaces Hasimoto's point-particle 4 pi/3 (a/L)^3 in translation)."""
    Sg = ratio * SIG
    p = ff.Params(L=L, M=M, a=A, Sigma=Sg, M_G=MG, R_c=lam * Sg if ratio > 1 else 0.0)
    Y = np.array([[3.3, 7.1, 0.4]])
    V, W = ff.mobility(p, Y, np.array([[1.0, 0, 0]]), np.array([[0, 0, 1.0]]))
    al = A / L
    tv = 1 - hasimoto_constant() * al + 4 * al ** 3
    tw = 1 - 4 * np.pi / 3 * al ** 3
    assert abs(V[0, 0] * 6 * np.pi * A - tv) < 1e-8
    assert abs(W[0, 2] * 8 * np.pi * A ** 3 - tw) < 1e-8
    assert np.abs(V[0, 1:]).max() < 1e-9 and np.abs(W[0, :2]).max() < 1e-9


def test_opposite_forces_give_opposite_velocities():
    L = 16.0
    p = ff.Params(L=L, M=24, a=A, Sigma=1.0, M_G=20, R_c=7.9)
    Y = np.array([[2.0, 3.0, 4.0], [5.5, 4.2, 6.1]])
    F = np.array([[0.3, -0.8, 0.5], [-0.3, 0.8, -0.5]])
    V, _ = ff.mobility(p, Y, F, None)
    assert np.abs(V[0] + V[1]).max() < 1e-8 * np.abs(V).max()


@pytest.mark.parametrize("L,Rc", [(24.0, 7.9), (30.0, 5.0)])
def test_cell_list_pair_search_equals_brute_force(L, Rc):
    p = ff.Params(L=L, M=16, a=A, Sigma=1.4, M_G=8, R_c=Rc)
    rng = np.random.default_rng(2)
    N = 120
    Y = rng.uniform(-L, 2 * L, size=(N, 3))         # outside the box: wrapped
    F = rng.normal(size=(N, 3))
    T = rng.normal(size=(N, 3))
    dV, dW = ff.pair_correction(p, Y, F, T)
    from oracle import closed_forms as cf
    Yw = ff.wrap(Y, L)
    bV = np.zeros((N, 3))
    bW = np.zeros((N, 3))
    for n in range(N):
        for m in range(N):
            if m == n:
                continue
            x = ff.min_image(Yw[n] - Yw[m], L)
            if np.linalg.norm(x) < Rc:
                bV[n] += cf.correction_VF(x, p.sigma, p.Sigma) @ F[m] + \
                    cf.correction_VT(x, p.sigma, p.sigma_D, p.Sigma, p.Sigma_D) @ T[m]
                bW[n] += cf.correction_OF(x, p.sigma, p.sigma_D, p.Sigma, p.Sigma_D) @ F[m] + \
                    cf.correction_OT(x, p.sigma_D, p.Sigma_D) @ T[m]
        bV[n] += cf.self_correction_VF(A, p.sigma, p.Sigma) * F[n]
        bW[n] += cf.self_correction_OT(A, p.Sigma_D) * T[n]
    assert np.allclose(dV, bV, rtol=0, atol=1e-14) and np.allclose(dW, bW, rtol=0, atol=1e-14)


def test_targets_subset_matches_full_evaluation():
    L = 20.0
    p = ff.Params(L=L, M=16, a=A, Sigma=1.25, M_G=10, R_c=6.0)
    rng = np.random.default_rng(4)
    Y = _random_config(30, L, seed=6)
    F = rng.normal(size=(30, 3))
    T = rng.normal(size=(30, 3))
    V, W = ff.mobility(p, Y, F, T)
    tg = np.array([7, 2, 19])
    Vs, Ws = ff.mobility(p, Y, F, T, targets=tg)
    assert np.allclose(Vs, V[tg], rtol=0, atol=1e-15) and np.allclose(Ws, W[tg], rtol=0, atol=1e-15)


def test_pair_correction_at_coincident_centres_is_the_limit():
    """Two particles at the same point: the pair correction takes the r -> 0
    limits of App. B, so it is finite (the closed forms divide by r) and equals
    the mean of the corrections with the second particle moved 1e-3 sigma
    either way (the odd force-torque blocks cancel; the rest approaches its
    limit as r^2, and the closed forms still hold 1e-10 there)."""
    p = ff.Params(L=12.0, M=24, a=A, Sigma=0.9, M_G=10, R_c=4.0, eta=1.3, Sigma_D=1.1)
    rng = np.random.default_rng(23)
    Y = rng.uniform(0.0, 12.0, size=(5, 3))
    Y[1] = Y[0]
    F, T = rng.normal(size=(5, 3)), rng.normal(size=(5, 3))
    dV, dW = ff.pair_correction(p, Y, F, T)
    assert np.isfinite(dV).all() and np.isfinite(dW).all()
    step = 1e-3 * p.sigma * np.array([0.48, -0.6, 0.64])
    Yp, Ym = Y.copy(), Y.copy()
    Yp[1] += step
    Ym[1] -= step
    (pV, pW), (mV, mW) = ff.pair_correction(p, Yp, F, T), ff.pair_correction(p, Ym, F, T)
    assert np.abs(dV - 0.5 * (pV + mV)).max() < 1e-6 * np.abs(dV).max()
    assert np.abs(dW - 0.5 * (pW + mW)).max() < 1e-6 * np.abs(dW).max()
    # and the coincident pair contributes the self-correction values
    solo = ff.pair_correction(p, np.delete(Y, 1, axis=0), np.delete(F, 1, axis=0), np.delete(T, 1, axis=0))
    from oracle import closed_forms as cf
    extra = cf.self_correction_VF(A, p.sigma, p.Sigma, p.eta) * F[1]
    assert np.allclose(dV[0] - solo[0][0], extra, rtol=0, atol=1e-13)
