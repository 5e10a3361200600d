"""Exact periodic FCM mobilities as Fourier lattice sums, plain FP64.

TEST INFRASTRUCTURE ONLY (see the package header).

App. A writes the FCM pair mobility as a Fourier integral of the inverse
Stokes operator times the squared Gaussian transform.  In the periodic box
[0, L)^3 the integral becomes a sum over k = 2 pi j / L, j in Z^3 \\ {0}
(the k = 0 mode carries no flow):

  M^{VF}_{nm}  = (1 / eta L^3) sum_k exp(-sigma^2 k^2)          (I - k^ k^^T) / k^2  cos(k.x)
  M^{OT}_{nm}  = (1 / 4 eta L^3) sum_k exp(-sigma_D^2 k^2)      (I - k^ k^^T)        cos(k.x)
  M^{OF}_{nm}  = (1 / 2 eta L^3) sum_k exp(-(sigma^2+sigma_D^2) k^2 / 2) (k x) / k^2 (-sin(k.x))
  M^{VT}_{nm}  = (M^{OF}_{mn})^T

with x = Y_n - Y_m, and (k x) the matrix of the cross product with k.  The
force-velocity weight exp(-sigma^2 k^2) is (2 pi)^6 times the squared Gaussian
transform of App. A; the torque rows follow from Omega = (1/2) curl u averaged
with the sigma_D Gaussian (Sec. 3.4), and the torque spreading (1/2) curl(T Delta).

The same sums with each Gaussian transform multiplied by the modified-kernel
factor (1 + (sigma^2 - Sigma^2) k^2 / 2)... written out in ``modified=True``
give the exact periodic version of the grid part M~ (Sec. 3.3, the transform of
Delta~ is (1 - (sigma^2 - Sigma^2) k^2 / 2) times that of Delta(.; Sigma)).
"""

import numpy as np


def _modes(L, kmax):
    jmax = int(np.ceil(kmax * L / (2.0 * np.pi)))
    j = np.arange(-jmax, jmax + 1)
    jx, jy, jz = np.meshgrid(j, j, j, indexing="ij")
    k = 2.0 * np.pi / L * np.stack([jx.ravel(), jy.ravel(), jz.ravel()], axis=1)
    k2 = np.sum(k * k, axis=1)
    keep = (k2 > 0.0) & (k2 <= kmax * kmax)
    return k[keep], k2[keep]


def mobility_matrix(Y, L, a, eta=1.0, Sigma=None, Sigma_D=None, tol=1e-17, modified=False):
    """Assemble the 6N x 6N periodic FCM mobility by direct lattice sums.

    Ordering of unknowns: (V_1..V_N, Omega_1..Omega_N) <- (F_1..F_N, T_1..T_N).
    With ``modified=True`` the grid part M~ of fast FCM with widths Sigma,
    Sigma_D is summed instead of M.
    """
    Y = np.asarray(Y, dtype=np.float64)
    N = len(Y)
    sigma = a / np.sqrt(np.pi)
    sigma_D = a / (6.0 * np.sqrt(np.pi)) ** (1.0 / 3.0)
    if modified:
        if Sigma_D is None:
            Sigma_D = Sigma
        wF, wD = Sigma, Sigma_D
        c = sigma ** 2 - Sigma ** 2
    else:
        wF, wD = sigma, sigma_D
        c = 0.0
    smin = min(wF, wD)
    kmax = np.sqrt(-np.log(tol)) / smin
    k, k2 = _modes(L, kmax)
    # transforms of the force and torque kernels (up to (2 pi)^-3)
    gF = (1.0 - 0.5 * c * k2) * np.exp(-0.5 * wF ** 2 * k2)
    gD = np.exp(-0.5 * wD ** 2 * k2)
    khat = k / np.sqrt(k2)[:, None]
    proj = np.eye(3)[None] - khat[:, :, None] * khat[:, None, :]
    kx = np.zeros((len(k), 3, 3))
    kx[:, 0, 1], kx[:, 0, 2] = -k[:, 2], k[:, 1]
    kx[:, 1, 0], kx[:, 1, 2] = k[:, 2], -k[:, 0]
    kx[:, 2, 0], kx[:, 2, 1] = -k[:, 1], k[:, 0]
    V3 = L ** 3
    Mat = np.zeros((6 * N, 6 * N))
    for n in range(N):
        for m in range(N):
            x = Y[n] - Y[m]
            kdx = k @ x
            cs, sn = np.cos(kdx), np.sin(kdx)
            VF = np.einsum("p,pij->ij", gF * gF * cs / k2, proj) / (eta * V3)
            OT = np.einsum("p,pij->ij", gD * gD * cs, proj) / (4.0 * eta * V3)
            # Omega_n from F_m: (1/2) i k x u^, u^ = P F g/(eta k^2), phase e^{ik.x}
            OF = np.einsum("p,pij->ij", -gF * gD * sn / k2, kx) / (2.0 * eta * V3)
            Mat[3 * n:3 * n + 3, 3 * m:3 * m + 3] = VF
            Mat[3 * N + 3 * n:3 * N + 3 * n + 3, 3 * N + 3 * m:3 * N + 3 * m + 3] = OT
            Mat[3 * N + 3 * n:3 * N + 3 * n + 3, 3 * m:3 * m + 3] = OF
    # M^{VT}_{nm} = (M^{OF}_{mn})^T
    for n in range(N):
        for m in range(N):
            Mat[3 * n:3 * n + 3, 3 * N + 3 * m:3 * N + 3 * m + 3] = \
                Mat[3 * N + 3 * m:3 * N + 3 * m + 3, 3 * n:3 * n + 3].T
    return Mat
