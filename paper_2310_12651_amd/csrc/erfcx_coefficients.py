"""Coefficients of the Chebyshev series of erfcx(x) = exp(x^2) erfc(x), x >= 0,
used by the pair correction (fcm_pair.hip, erfcx_series): the interpolant of
erfcx in u = (2 - x) / (2 + x) at the 27 Chebyshev nodes of [-1, 1], its
coefficients from the discrete Chebyshev transform in extended precision.
Run to print them and the relative error of the series (summed as the kernel
sums it, by Clenshaw's recurrence) against scipy's erfcx and erfc."""

import numpy as np
from scipy.special import erfc, erfcx

DEGREE = 26


def coefficients(deg=DEGREE):
    ld = np.longdouble
    n = deg + 1
    th = np.pi * (np.arange(n, dtype=ld) + ld(0.5)) / n
    u = np.cos(th)
    x = (2 - 2 * u) / (1 + u)          # inverse of u = (2 - x) / (2 + x)
    f = np.array([erfcx(float(v)) for v in x], dtype=ld)
    c = np.array([2 / ld(n) * np.sum(f * np.cos(j * th)) for j in range(n)], dtype=ld)
    c[0] /= 2
    return c.astype(np.float64)


def series(c, x):
    u = (2.0 - x) / (2.0 + x)
    b1 = np.zeros_like(x)
    b2 = np.zeros_like(x)
    for cj in c[:0:-1]:
        b1, b2 = 2.0 * u * b1 + (cj - b2), b1
    return u * b1 + (c[0] - b2)


if __name__ == "__main__":
    c = coefficients()
    for i in range(0, len(c), 3):
        print("        " + ", ".join(repr(float(v)) for v in c[i:i + 3]) + ",")
    x = np.concatenate([np.linspace(0.0, 10.0, 200001), np.geomspace(1e-12, 1.0, 2000)])
    r1 = np.abs(series(c, x) - erfcx(x)) / erfcx(x)
    r2 = np.abs(np.exp(-x * x) * series(c, x) - erfc(x)) / erfc(x)
    print(f"erfcx relative error max {r1.max():.2e}; erfc relative error max {r2.max():.2e}")
