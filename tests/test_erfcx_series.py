"""The Chebyshev series of erfcx(x) = exp(x^2) erfc(x) that the pair correction
sums on the GPU (fcm_pair.hip, erfcx_series): its coefficients are those its
generator derives, and the series, summed by the same recurrence, reproduces
scipy's erfc to a few units in the last place on the range the pair blocks use."""

import os
import re
import sys

import numpy as np
from scipy.special import erfc, erfcx

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2310_12651_amd", "csrc")
sys.path.insert(0, CSRC)
import erfcx_coefficients as gen  # noqa: E402


def _kernel_coefficients():
    src = open(os.path.join(CSRC, "fcm_pair.hip")).read()
    body = src[src.index("__device__ inline double erfcx_series"):]
    block = body[body.index("{", body.index("c[27]")) + 1: body.index("};")]
    return np.array([float(v) for v in re.findall(r"[-+0-9.e]+", block)])


def test_kernel_coefficients_are_the_generators():
    assert np.array_equal(_kernel_coefficients(), gen.coefficients())


def test_series_reproduces_erfc():
    c = gen.coefficients()
    x = np.concatenate([np.linspace(0.0, 10.0, 100001), np.geomspace(1e-12, 1.0, 1000)])
    assert np.max(np.abs(gen.series(c, x) - erfcx(x)) / erfcx(x)) < 3e-15
    assert np.max(np.abs(np.exp(-x * x) * gen.series(c, x) - erfc(x)) / erfc(x)) < 3e-15


def test_width_differences_stay_accurate():
    """The pair blocks take differences erfc(r e2) - erfc(r e1) of two widths."""
    c = gen.coefficients()
    r = np.linspace(1e-3, 30.0, 60001)
    for e1, e2 in ((1.2, 0.6), (0.9, 0.42), (0.9, 0.19)):
        ref = erfc(r * e2) - erfc(r * e1)
        new = np.exp(-(r * e2) ** 2) * gen.series(c, r * e2) - np.exp(-(r * e1) ** 2) * gen.series(c, r * e1)
        assert np.max(np.abs(new - ref)) < 3e-15
