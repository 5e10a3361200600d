"""Derivations of stored parameters, using only the oracle's closed forms.

TEST INFRASTRUCTURE ONLY (see the package header).

``cutoff_for_tolerance`` finds the pair-correction cut-off radius beyond which
every entry of the correction blocks (eqs. correction_VF, correction_WF,
correction_WT), scaled by the single-particle mobilities 1/(6 pi eta a) and
1/(8 pi eta a^3), stays below a tolerance.  The corrections decay like
exp(-r^2 / 4 Sigma^2) (Sec. 3.2), so beyond their last sign change the scaled
size is monotone and bisection applies.

Run as a script to print the cut-off of the 64-sphere FP64 parity workload
(a = 1, Sigma = 2 sigma, tolerance 1e-10); ``workloads.py`` stores the value.
"""

import math

import numpy as np

from . import closed_forms as cf


def scaled_correction(r, a, Sigma, Sigma_D=None, eta=1.0):
    """Largest scaled entry of the three correction blocks at distance r,
    over the axis and body-diagonal directions."""
    if Sigma_D is None:
        Sigma_D = Sigma
    sigma = a / math.sqrt(math.pi)
    sigma_D = a / (6.0 * math.sqrt(math.pi)) ** (1.0 / 3.0)
    dirs = np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0], [1.0, 1.0, 1.0]])
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    x = r * dirs
    sv = 6.0 * math.pi * eta * a
    so = 8.0 * math.pi * eta * a ** 3
    sm = math.sqrt(sv * so)
    vf = np.abs(cf.correction_VF(x, sigma, Sigma, eta)).max() * sv
    of = np.abs(cf.correction_OF(x, sigma, sigma_D, Sigma, Sigma_D, eta)).max() * sm
    ot = np.abs(cf.correction_OT(x, sigma_D, Sigma_D, eta)).max() * so
    return max(vf, of, ot)


def cutoff_for_tolerance(a, Sigma, tol, r_hi, Sigma_D=None, eta=1.0):
    """Smallest r (to 1e-9 relative) in (0, r_hi] with scaled_correction < tol
    from r onwards, by bisection from a bracket found on a coarse scan."""
    rs = np.linspace(r_hi, 0.05 * a, 2000)
    lo = None
    for r in rs:                      # walk inwards until the bound is violated
        if scaled_correction(r, a, Sigma, Sigma_D, eta) >= tol:
            lo = r
            break
    if lo is None:
        return 0.0
    hi = lo + (rs[0] - rs[1])
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if scaled_correction(mid, a, Sigma, Sigma_D, eta) >= tol:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-9 * hi:
            break
    return hi


if __name__ == "__main__":
    a = 1.0
    sigma = a / math.sqrt(math.pi)
    print(repr(cutoff_for_tolerance(a, 2.0 * sigma, 1e-10, 19.9)))
