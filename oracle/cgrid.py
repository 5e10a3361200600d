"""Spreading in plain C (oracle/cgrid.c) -- TEST INFRASTRUCTURE ONLY.

``spread`` has the signature and the result of ``fastfcm.spread`` (Sec. 3.1
eq. force_kernel_mod, Sec. 3.4 eq. torque_kernel_mod) and evaluates the same
kernels point by point in FP64; it exists so that the oracle can spread the
10^5-particle problems of the request stream on 288^3-432^3 grids with
M_G = 16 in seconds.  Its agreement with ``fastfcm.spread`` is pinned in
tests/test_oracle_grid.py.

The shared library is compiled with gcc into oracle/_cgrid.so by ``build``
(called from the package build), or on first use when it is missing.
"""

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cgrid.c")
LIB = os.path.join(HERE, "_cgrid.so")

_lib = None


def build():
    """Compile cgrid.c with gcc (IEEE arithmetic, no fast-math)."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-o", tmp, SRC, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"gcc failed:\n{r.stdout}{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_spread.argtypes = [ctypes.c_int64, dp, dp, dp, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        lib.oracle_spread.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def spread(p, Y, F, T=None):
    """J~^dagger[F] + N~^dagger[T] on the grid of ``p`` (a fastfcm.Params).

    Returns f with shape (3, Mx, My, Mz), axes (component, x, y, z).
    """
    lib = _load()
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    Tc = None if T is None else np.ascontiguousarray(T, dtype=np.float64)
    Mx, My, Mz = p.Mv
    f = np.zeros((3, Mx, My, Mz))
    st = lib.oracle_spread(len(Y), _ptr(Y), _ptr(F), None if Tc is None else _ptr(Tc), Mx, My, Mz,
                           float(p.Lv[0]), float(p.Lv[1]), float(p.Lv[2]), int(p.M_G), p.sigma,
                           p.Sigma, p.Sigma_D, _ptr(f))
    if st != 0:
        raise ValueError("oracle_spread: invalid arguments")
    return f
