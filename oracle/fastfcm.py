"""Fast FCM, plain FP64 on the CPU: the algorithm of Sec. 4, step by step.

TEST INFRASTRUCTURE ONLY (see the package header).

The steps are those of Sec. 4 in the paper's order: spatial hashing, sorting
into cell lists, applying the modified spreading operator J~^dagger (with the
torque spreading N~^dagger of Sec. 3.4), the inverse Stokes operator in
Fourier space (Sec. 2.1, App. A), the interpolation operators J~ and N~, and
the pairwise correction for pairs closer than R_c, plus the self corrections
of App. B.  numpy's FFT serves as the Fourier transform; nothing is blocked,
fused or reordered.

Grid conventions (the paper leaves them open; these readings are part of the
library's contract and are checked only GPU-against-oracle):

* grid points sit at x_g = (i, j, k) * dx, i, j, k = 0..M-1, dx = L / M, on the
  periodic box [0, L)^3 (Sec. 2.1);
* the M_G support points of a particle at coordinate Y along one axis are
  start, ..., start + M_G - 1 (indices mod M) with
  start = floor(Y/dx - M_G/2) + 1, and the displacement used in the kernel is
  d = (start + j) dx - Y, not a minimum image;
* for even M every Fourier mode whose index equals M/2 along any axis is set
  to zero in the Stokes solve (the projection is odd in that component, so a
  real field cannot represent it), and the k = 0 mode is zero;
* Omega is formed from the real-space gradient of the torque Gaussian
  (integration by parts of (1/2) curl u), which makes N~ the exact transpose of
  N~^dagger on the grid.
"""

from dataclasses import dataclass
import math

import numpy as np

from . import closed_forms as cf


@dataclass
class Params:
    """Fast-FCM parameters (Sec. 5): box L, grid M per axis, support M_G,
    particle radius a, modified widths Sigma (force) and Sigma_D (torque,
    Sec. 3.4; the paper takes Sigma_D = Sigma), cut-off R_c, viscosity eta.

    L and M are one number each for a cube, or three (x, y, z) for a
    rectangular box; the grid spacing L / M must then be the same on all axes.
    """
    L: object
    M: object
    a: float
    Sigma: float
    M_G: int
    R_c: float
    eta: float = 1.0
    Sigma_D: float = None

    def __post_init__(self):
        if self.Sigma_D is None:
            self.Sigma_D = self.Sigma
        Lv = np.broadcast_to(np.asarray(self.L, dtype=np.float64), (3,)).copy()
        Mv = np.broadcast_to(np.asarray(self.M, dtype=np.int64), (3,)).copy()
        h = Lv / Mv
        if np.max(np.abs(h - h[0])) > 1e-12 * h[0]:
            raise ValueError("the grid spacing L/M must be the same on all axes")
        self.Lv, self.Mv = Lv, tuple(int(m) for m in Mv)

    @property
    def cubic(self):
        return self.Mv[0] == self.Mv[1] == self.Mv[2]

    @property
    def sigma(self):
        """FCM force width, a = sigma sqrt(pi) (Sec. 2)."""
        return self.a / math.sqrt(math.pi)

    @property
    def sigma_D(self):
        """FCM torque width sigma_D = a / (6 sqrt pi)^(1/3) (Sec. 3.4)."""
        return self.a / (6.0 * math.sqrt(math.pi)) ** (1.0 / 3.0)

    @property
    def dx(self):
        return float(self.Lv[0] / self.Mv[0])


# --- Sec. 4, steps 1-2: spatial hashing and cell lists ---------------------

def wrap(Y, L):
    """Map positions into the periodic box [0, L) (L one side, or three)."""
    L = np.asarray(L, dtype=np.float64)
    Yw = np.mod(np.asarray(Y, dtype=np.float64), L)
    Yw[Yw >= np.broadcast_to(L, Yw.shape)] = 0.0
    return Yw


def cell_counts(L, R_c):
    """Cells per direction m = max(int(L / R_c), 3) (Sec. 4, spatial hashing),
    per axis when L has three sides."""
    Lv = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    m = np.array([max(int(l / R_c), 3) for l in Lv], dtype=np.int64)
    return int(m[0]) if np.ndim(L) == 0 else m


def hash_particles(Y, L, m):
    """Cell index x_c + (y_c + z_c m_y) m_x of every particle (Sec. 4)."""
    Lv = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
    mv = np.broadcast_to(np.asarray(m, dtype=np.int64), (3,))
    c = np.floor(wrap(Y, Lv) / (Lv / mv)).astype(np.int64)
    c = np.minimum(c, mv - 1)
    return c[:, 0] + (c[:, 1] + c[:, 2] * mv[1]) * mv[0]


def cell_lists(keys, m):
    """Sort by key (stable) and return (order, start) with start[c]..start[c+1]
    the sorted positions of the particles in cell c (Sec. 4, sorting)."""
    ncell = int(np.prod(np.broadcast_to(np.asarray(m, dtype=np.int64), (3,))))
    order = np.argsort(keys, kind="stable")
    start = np.searchsorted(keys[order], np.arange(ncell + 1))
    return order, start


# --- Sec. 2.1 / 3.1 / 3.4: grid operators ----------------------------------

def _window(Yc, dx, M_G, M):
    """Support of one coordinate: grid indices (mod M) and displacements d."""
    start = np.floor(Yc / dx - M_G / 2.0).astype(np.int64) + 1
    j = start[:, None] + np.arange(M_G)[None, :]
    d = j * dx - Yc[:, None]
    return np.mod(j, M), d


def _particle_weights(p, Yw):
    """For a block of particles: flat grid indices and, at every support point,
    the modified force kernel Delta~(d; Sigma) (Sec. 3, definition of Delta~)
    and the torque factor Delta(d; Sigma_D) / (2 Sigma_D^2) with d itself."""
    (Mx, My, Mz), MG = p.Mv, p.M_G
    ix, dxs = _window(Yw[:, 0], p.dx, MG, Mx)
    iy, dys = _window(Yw[:, 1], p.dx, MG, My)
    iz, dzs = _window(Yw[:, 2], p.dx, MG, Mz)
    # full 3-D support, shape (n, MG, MG, MG), axis order (x, y, z)
    flat = (ix[:, :, None, None] * My + iy[:, None, :, None]) * Mz + iz[:, None, None, :]
    dx3 = np.broadcast_to(dxs[:, :, None, None], flat.shape)
    dy3 = np.broadcast_to(dys[:, None, :, None], flat.shape)
    dz3 = np.broadcast_to(dzs[:, None, None, :], flat.shape)
    r2 = dx3 ** 2 + dy3 ** 2 + dz3 ** 2
    S2 = p.Sigma ** 2
    # Delta~ = (1 + (sigma^2 - Sigma^2)/2 lap) Delta(.; Sigma); lap Delta = Delta (r^2/S^4 - 3/S^2)
    dmod = cf.gaussian(np.sqrt(r2), p.Sigma) * (1.0 + 0.5 * (p.sigma ** 2 - S2) * (r2 / S2 ** 2 - 3.0 / S2))
    # -(1/2) T x grad Delta(.; Sigma_D) = (1 / 2 Sigma_D^2) Delta (T x d)
    dtor = cf.gaussian(np.sqrt(r2), p.Sigma_D) / (2.0 * p.Sigma_D ** 2)
    return flat, dmod, dtor, (dx3, dy3, dz3)


def spread(p, Y, F, T=None, chunk=2048):
    """J~^dagger[F] + N~^dagger[T] on the grid (Sec. 3.1 eq. force_kernel_mod,
    Sec. 3.4 eq. torque_kernel_mod), truncated to M_G^3 points (Sec. 2.1).

    Returns f with shape (3, Mx, My, Mz), axes (component, x, y, z).
    """
    Yw = wrap(Y, p.Lv)
    F = np.asarray(F, dtype=np.float64)
    M3 = p.Mv[0] * p.Mv[1] * p.Mv[2]
    f = np.zeros((3, M3))
    for lo in range(0, len(Yw), chunk):
        hi = min(lo + chunk, len(Yw))
        flat, dmod, dtor, (dx3, dy3, dz3) = _particle_weights(p, Yw[lo:hi])
        idx = flat.ravel()
        Fc = F[lo:hi]
        comps = [dmod * Fc[:, c, None, None, None] for c in range(3)]
        if T is not None:
            Tc = np.asarray(T, dtype=np.float64)[lo:hi]
            t = [Tc[:, c, None, None, None] for c in range(3)]
            # T x d
            comps[0] = comps[0] + dtor * (t[1] * dz3 - t[2] * dy3)
            comps[1] = comps[1] + dtor * (t[2] * dx3 - t[0] * dz3)
            comps[2] = comps[2] + dtor * (t[0] * dy3 - t[1] * dx3)
        for c in range(3):
            f[c] += np.bincount(idx, weights=comps[c].ravel(), minlength=M3)
    return f.reshape(3, *p.Mv)


def wavenumbers(p, axis=0):
    """Wavenumbers 2 pi j / L of numpy's FFT ordering along one axis."""
    M, L = p.Mv[axis], p.Lv[axis]
    return 2.0 * np.pi * np.fft.fftfreq(M, d=1.0 / M) / L


def stokes_solve(p, f, workers=None):
    """Inverse Stokes operator L^{-1} in Fourier space (Sec. 2.1 step 2,
    App. A): u^ = (I - k k^T / k^2) f^ / (eta k^2), u^(0) = 0.

    Input and output have shape (3, Mx, My, Mz).  Along an axis of even
    length M the modes with index M/2 are zeroed.  ``workers``: None uses
    numpy's FFT (one thread); a number uses scipy's FFT with that many threads
    (the same transform, for the largest grids).
    """
    if workers is None:
        fftn, ifftn = np.fft.fftn, np.fft.ifftn
    else:
        import scipy.fft as sfft
        fftn = lambda a, axes: sfft.fftn(a, axes=axes, workers=workers)
        ifftn = lambda a, axes: sfft.ifftn(a, axes=axes, workers=workers)
    fh = fftn(f, axes=(1, 2, 3))
    kx = wavenumbers(p, 0)[:, None, None]
    ky = wavenumbers(p, 1)[None, :, None]
    kz = wavenumbers(p, 2)[None, None, :]
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    k2s = np.where(k2 == 0.0, 1.0, k2)
    kdotf = (kx * fh[0] + ky * fh[1] + kz * fh[2]) / k2s
    uh = np.empty_like(fh)
    uh[0] = (fh[0] - kx * kdotf) / (p.eta * k2s)
    uh[1] = (fh[1] - ky * kdotf) / (p.eta * k2s)
    uh[2] = (fh[2] - kz * kdotf) / (p.eta * k2s)
    uh[:, 0, 0, 0] = 0.0
    Mx, My, Mz = p.Mv
    if Mx % 2 == 0:
        uh[:, Mx // 2, :, :] = 0.0
    if My % 2 == 0:
        uh[:, :, My // 2, :] = 0.0
    if Mz % 2 == 0:
        uh[:, :, :, Mz // 2] = 0.0
    return np.real(ifftn(uh, axes=(1, 2, 3)))


def stokes_plane_wave(p, j, A, phi, idx):
    """The inverse Stokes operator of Sec. 2.1 step 2 (App. A) applied to one
    real Fourier mode, in closed form: f(x) = A cos(k.x + phi) with
    k_d = 2 pi j_d / L_d gives u(x) = (I - k k^T / k^2) A cos(k.x + phi) /
    (eta k^2), for an integer mode j != 0 with |j_d| < M_d / 2 on every axis
    (neither the zero mode nor an index-M/2 mode is involved).

    idx: integer grid indices, shape (n, 3) as (x, y, z), the points
    idx * dx.  The phase is 2 pi sum_d ((j_d idx_d) mod M_d) / M_d + phi,
    exact in its integer part at any grid size.  Returns u at the points,
    shape (n, 3).
    """
    j = np.asarray(j, dtype=np.int64)
    Mv = np.asarray(p.Mv, dtype=np.int64)
    if not np.any(j != 0) or np.any(2 * np.abs(j) >= Mv):
        raise ValueError("mode must be nonzero with |j_d| < M_d / 2")
    k = 2.0 * np.pi * j / p.Lv
    k2 = float(k @ k)
    A = np.asarray(A, dtype=np.float64)
    amp = (A - k * (k @ A) / k2) / (p.eta * k2)
    frac = np.sum(np.mod(np.asarray(idx, dtype=np.int64) * j, Mv) / Mv, axis=1)
    return np.cos(2.0 * np.pi * frac + phi)[:, None] * amp[None, :]


def interp(p, Y, u, want_omega=True, chunk=2048):
    """J~[u] and N~[u] (Sec. 3.1 eq. avg_particle_vel_mod, Sec. 3.4
    eq. avg_particle_rot_mod) by the trapezoid rule on the M_G^3 support
    (Sec. 2.1 step 3):

    V_m     = dV sum_g u_g Delta~(x_g - Y_m; Sigma)
    Omega_m = dV sum_g Delta(x_g - Y_m; Sigma_D) (x_g - Y_m) x u_g / (2 Sigma_D^2)

    (the second is (1/2) int (curl u) Delta after integration by parts).
    """
    Yw = wrap(Y, p.Lv)
    uf = u.reshape(3, -1)
    dV = p.dx ** 3
    V = np.zeros((len(Yw), 3))
    W = np.zeros((len(Yw), 3))
    for lo in range(0, len(Yw), chunk):
        hi = min(lo + chunk, len(Yw))
        flat, dmod, dtor, (dx3, dy3, dz3) = _particle_weights(p, Yw[lo:hi])
        ug = [uf[c][flat] for c in range(3)]
        ax = (1, 2, 3)
        for c in range(3):
            V[lo:hi, c] = dV * np.sum(dmod * ug[c], axis=ax)
        if want_omega:
            W[lo:hi, 0] = dV * np.sum(dtor * (dy3 * ug[2] - dz3 * ug[1]), axis=ax)
            W[lo:hi, 1] = dV * np.sum(dtor * (dz3 * ug[0] - dx3 * ug[2]), axis=ax)
            W[lo:hi, 2] = dV * np.sum(dtor * (dx3 * ug[1] - dy3 * ug[0]), axis=ax)
    return V, W


# --- Sec. 4 step 6: pairwise correction, App. B: self correction -----------

def min_image(x, L):
    L = np.asarray(L, dtype=np.float64)
    return x - L * np.round(x / L)


def pair_correction(p, Y, F, T=None, targets=None):
    """Velocity and angular-velocity corrections (M - M~)(F; T) for pairs with
    R_mn < R_c found through the cell lists (Sec. 4, pairwise correction),
    plus the self corrections of App. B.

    targets: indices of the particles whose corrections are wanted (default
    all).  Returns dV, dW of shape (len(targets), 3).
    """
    Yw = wrap(Y, p.Lv)
    N = len(Yw)
    F = np.asarray(F, dtype=np.float64)
    Tq = np.zeros((N, 3)) if T is None else np.asarray(T, dtype=np.float64)
    if targets is None:
        targets = np.arange(N)
    dV = np.zeros((len(targets), 3))
    dW = np.zeros((len(targets), 3))
    sg, sD, Sg, SD, eta = p.sigma, p.sigma_D, p.Sigma, p.Sigma_D, p.eta
    if p.R_c > 0.0:
        m = np.broadcast_to(np.asarray(cell_counts(p.Lv, p.R_c), dtype=np.int64), (3,))
        keys = hash_particles(Yw, p.Lv, m)
        order, start = cell_lists(keys, m)
        cw = p.Lv / m
    for t, n in enumerate(targets):
        if p.R_c <= 0.0:
            dV[t] += cf.self_correction_VF(p.a, sg, Sg, eta) * F[n]
            dW[t] += cf.self_correction_OT(p.a, SD, eta) * Tq[n]
            continue
        c = np.minimum(np.floor(Yw[n] / cw).astype(np.int64), m - 1)
        cand = []
        for oz in (-1, 0, 1):
            for oy in (-1, 0, 1):
                for ox in (-1, 0, 1):
                    cx, cy, cz = (c[0] + ox) % m[0], (c[1] + oy) % m[1], (c[2] + oz) % m[2]
                    key = cx + (cy + cz * m[1]) * m[0]
                    cand.append(order[start[key]:start[key + 1]])
        cand = np.concatenate(cand)
        cand = cand[cand != n]
        x = min_image(Yw[n][None, :] - Yw[cand], p.Lv)
        r = np.sqrt(np.sum(x * x, axis=1))
        # a neighbour at the same point (r = 0 exactly): the corrections take
        # their r -> 0 limits of App. B, the self-correction values (the
        # force-torque blocks are odd in x and vanish there)
        same = cand[r == 0.0]
        dV[t] += cf.self_correction_VF(p.a, sg, Sg, eta) * F[same].sum(axis=0)
        dW[t] += cf.self_correction_OT(p.a, SD, eta) * Tq[same].sum(axis=0)
        sel = (r < p.R_c) & (r > 0.0)
        cand, x = cand[sel], x[sel]
        if len(cand):
            CVF = cf.correction_VF(x, sg, Sg, eta)
            CVT = cf.correction_VT(x, sg, sD, Sg, SD, eta)
            COF = cf.correction_OF(x, sg, sD, Sg, SD, eta)
            COT = cf.correction_OT(x, sD, SD, eta)
            dV[t] += np.einsum("pij,pj->i", CVF, F[cand]) + np.einsum("pij,pj->i", CVT, Tq[cand])
            dW[t] += np.einsum("pij,pj->i", COF, F[cand]) + np.einsum("pij,pj->i", COT, Tq[cand])
        dV[t] += cf.self_correction_VF(p.a, sg, Sg, eta) * F[n]
        dW[t] += cf.self_correction_OT(p.a, SD, eta) * Tq[n]
    return dV, dW


def mobility(p, Y, F, T=None, targets=None, with_correction=True):
    """Fast-FCM action of the mobility (Sec. 4): (V, Omega) = M~ (F, T) + (M - M~)(F, T).

    Spreading always uses every particle; interpolation and correction are
    evaluated for ``targets`` (default all), in that order.
    """
    Y = np.asarray(Y, dtype=np.float64)
    N = len(Y)
    if targets is None:
        targets = np.arange(N)
    f = spread(p, Y, F, T)
    u = stokes_solve(p, f)
    V, W = interp(p, Y[targets], u)
    if with_correction:
        dV, dW = pair_correction(p, Y, F, T, targets)
        V = V + dV
        W = W + dW
    return V, W
