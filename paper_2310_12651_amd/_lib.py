"""ctypes binding of the fast-FCM C ABI (include/fcm.h).

Argument marshalling only: every step of the computation runs in the HIP
library ``libfcm.so``.  PyTorch supplies device memory and streams.  If the
library has not been built, importing works but every call raises
``LibraryMissing``; there is no fallback implementation.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfcm.so")

FCM_OK, FCM_EINVAL, FCM_ENOMEM, FCM_EDEVICE, FCM_ERANGE, FCM_ENONFINITE = 0, -1, -2, -3, -4, -5
FCM_ESCRATCH = -7
FCM_FP64, FCM_FP32_BULK = 0, 1

EXPORTS = [
    "fcm_options_default", "fcm_plan", "fcm_plan_ex", "fcm_plan_box", "fcm_plan_box_info",
    "fcm_plan_destroy", "fcm_mobility",
    "fcm_mobility_repeat", "fcm_brownian", "fcm_brownian_reserve", "fcm_spread", "fcm_solve", "fcm_interp", "fcm_correct", "fcm_plan_info",
    "fcm_plan_footprint", "fcm_plan_footprint_box", "fcm_plan_last_error", "fcm_status_string", "fcm_plan_set_timing",
    "fcm_plan_stage_times", "fcm_mobility_static",
]
STAGES = ["sort", "spread", "fft_x_fwd", "fft_y_fwd", "fft_z_solve", "fft_y_inv", "fft_x_inv",
          "interp", "pair"]


class LibraryMissing(RuntimeError):
    pass


class FCMError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


class Options(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("support", ctypes.c_int),
                ("sigma_D_grid", ctypes.c_double), ("precision", ctypes.c_int),
                ("kahan", ctypes.c_int)]


_lib = None


def library():
    """The loaded libfcm.so (raises LibraryMissing if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} is not built; run python -m paper_2310_12651_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp, dp, i64, ci, cd = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    sig = {
        "fcm_options_default": ([ctypes.POINTER(Options)], ci),
        "fcm_plan": ([ctypes.POINTER(vp), i64, cd, cd, cd, ci, cd], ci),
        "fcm_plan_ex": ([ctypes.POINTER(vp), i64, cd, cd, cd, ci, cd, ctypes.POINTER(Options)], ci),
        "fcm_plan_box": ([ctypes.POINTER(vp), i64, ctypes.POINTER(cd), cd, cd, ctypes.POINTER(ci), cd,
                          ctypes.POINTER(Options)], ci),
        "fcm_plan_box_info": ([vp, ctypes.POINTER(cd), ctypes.POINTER(ci), ctypes.POINTER(ci)], ci),
        "fcm_plan_destroy": ([vp], ci),
        "fcm_mobility": ([vp, dp, dp, dp, dp, dp, vp], ci),
        "fcm_mobility_repeat": ([vp, dp, dp, dp, dp, vp], ci),
        "fcm_brownian": ([vp, dp, vp, dp, cd, cd, dp, ctypes.POINTER(ci), vp], ci),
        "fcm_brownian_reserve": ([vp, ci], ci),
        "fcm_spread": ([vp, dp, dp, dp, vp, vp], ci),
        "fcm_solve": ([vp, vp, vp], ci),
        "fcm_interp": ([vp, dp, vp, dp, dp, vp], ci),
        "fcm_correct": ([vp, dp, dp, dp, dp, dp, vp], ci),
        "fcm_plan_info": ([vp, ctypes.POINTER(i64), ctypes.POINTER(ci), ctypes.POINTER(ci),
                           ctypes.POINTER(ci), ctypes.POINTER(ci)], ci),
        "fcm_plan_footprint": ([i64, ci, ci, ctypes.POINTER(i64)], ci),
        "fcm_plan_footprint_box": ([i64, ctypes.POINTER(cd), cd, cd, ctypes.POINTER(ci), cd,
                                    ctypes.POINTER(Options), ctypes.POINTER(i64)], ci),
        "fcm_plan_last_error": ([vp], ci),
        "fcm_status_string": ([ci], ctypes.c_char_p),
        "fcm_plan_set_timing": ([vp, ci], ci),
        "fcm_plan_stage_times": ([vp, ctypes.POINTER(cd), ctypes.POINTER(ci)], ci),
        "fcm_mobility_static": ([i64, cd, cd, cd, ci, cd, ctypes.POINTER(Options), dp, dp, dp, dp, dp, vp],
                                ci),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def status_string(status):
    try:
        return library().fcm_status_string(int(status)).decode()
    except LibraryMissing:
        return f"status {status}"


def _check(status, where):
    if status != FCM_OK:
        raise FCMError(status, where)


def _ptr(t, name, n=None, dtype=None, allow_none=False):
    """Device pointer of a contiguous CUDA/HIP tensor (or None)."""
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    import torch
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if n is not None and tuple(t.shape) != (n, 3):
        raise ValueError(f"{name} must have shape ({n}, 3), got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def fcm_options_default():
    o = Options()
    _check(library().fcm_options_default(ctypes.byref(o)), "fcm_options_default")
    return o


def fcm_plan_footprint(N, grid, precision):
    b = ctypes.c_int64()
    _check(library().fcm_plan_footprint(int(N), int(grid), int(precision), ctypes.byref(b)),
           "fcm_plan_footprint")
    return b.value


def fcm_plan_footprint_box(N, L, a, Sigma, grid, r_cut, options=None):
    """Exact device bytes of the plan fcm_plan_box would build (L, grid: one
    number for a cube or three)."""
    L3 = (ctypes.c_double * 3)(*([float(L)] * 3 if isinstance(L, (int, float)) else [float(x) for x in L]))
    g3 = (ctypes.c_int * 3)(*([int(grid)] * 3 if isinstance(grid, int) else [int(x) for x in grid]))
    b = ctypes.c_int64()
    opt = None if options is None else ctypes.byref(options)
    _check(library().fcm_plan_footprint_box(int(N), L3, float(a), float(Sigma), g3, float(r_cut), opt,
                                            ctypes.byref(b)), "fcm_plan_footprint_box")
    return b.value


def mobility_static(N, L, a, Sigma, grid, r_cut, pos, F, T=None, V=None, Omega=None, eta=1.0, support=0,
                    sigma_D_grid=0.0, precision=FCM_FP32_BULK, kahan=0, stream=None, want_omega=True):
    """fcm_mobility_static: the mobility without a plan, in the library's
    static device scratch (no allocation by the library; V and Omega are
    allocated here unless given)."""
    import torch
    N = int(N)
    if V is None:
        V = torch.empty((N, 3), dtype=torch.float64, device=pos.device)
    if Omega is None and want_omega:
        Omega = torch.empty((N, 3), dtype=torch.float64, device=pos.device)
    o = fcm_options_default()
    o.eta, o.support, o.sigma_D_grid = float(eta), int(support), float(sigma_D_grid)
    o.precision, o.kahan = int(precision), int(kahan)
    f64 = torch.float64
    _check(library().fcm_mobility_static(N, float(L), float(a), float(Sigma), int(grid), float(r_cut),
                                         ctypes.byref(o), _ptr(pos, "pos", N, f64), _ptr(F, "F", N, f64),
                                         _ptr(T, "T", N, f64, True), _ptr(V, "V", N, f64),
                                         _ptr(Omega, "Omega", N, f64, True), _stream(stream)),
           "fcm_mobility_static")
    return V, Omega


class Plan:
    """A fast-FCM plan: N spheres of radius a in the periodic cube [0, L)^3,
    modified kernel width Sigma, grid^3 points, pair cut-off r_cut.  L and grid
    may also be three values (x, y, z) for a rectangular box with one grid
    spacing (fcm_plan_box)."""

    def __init__(self, N, L, a, Sigma, grid, r_cut, eta=1.0, support=0, sigma_D_grid=0.0,
                 precision=FCM_FP32_BULK, kahan=0):
        import torch
        lib = library()
        if isinstance(precision, str):
            precision = {"fp64": FCM_FP64, "fp32": FCM_FP32_BULK}[precision]
        o = fcm_options_default()
        o.eta, o.support, o.sigma_D_grid = float(eta), int(support), float(sigma_D_grid)
        o.precision, o.kahan = int(precision), int(kahan)
        h = ctypes.c_void_p()
        if hasattr(L, "__len__") or hasattr(grid, "__len__"):
            L3 = [float(x) for x in (L if hasattr(L, "__len__") else (L, L, L))]
            g3 = [int(x) for x in (grid if hasattr(grid, "__len__") else (grid, grid, grid))]
            _check(lib.fcm_plan_box(ctypes.byref(h), int(N), (ctypes.c_double * 3)(*L3), float(a),
                                    float(Sigma), (ctypes.c_int * 3)(*g3), float(r_cut),
                                    ctypes.byref(o)), "fcm_plan_box")
        else:
            L3, g3 = [float(L)] * 3, [int(grid)] * 3
            _check(lib.fcm_plan_ex(ctypes.byref(h), int(N), float(L), float(a), float(Sigma),
                                   int(grid), float(r_cut), ctypes.byref(o)), "fcm_plan_ex")
        self._h = h
        self.N, self.a, self.Sigma, self.r_cut = int(N), a, Sigma, r_cut
        self.L = L3[0] if L3[0] == L3[1] == L3[2] else tuple(L3)
        self.grid = g3[0] if g3[0] == g3[1] == g3[2] else tuple(g3)
        self.grid_shape = (3, g3[2], g3[1], g3[0])
        self.precision = int(precision)
        self.grid_dtype = torch.float64 if precision == FCM_FP64 else torch.float32
        info = self.info()
        self.support, self.cells_per_axis = info["support"], info["cells_per_axis"]

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan destroyed")
        return self._h

    def info(self):
        N, g, s, p, m = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(library().fcm_plan_info(self.handle, ctypes.byref(N), ctypes.byref(g), ctypes.byref(s),
                                       ctypes.byref(p), ctypes.byref(m)), "fcm_plan_info")
        return dict(N=N.value, grid=g.value, support=s.value, precision=p.value, cells_per_axis=m.value)

    def box_info(self):
        """Box sides, grid points and pair cells per axis (x, y, z)."""
        L, g, c = (ctypes.c_double * 3)(), (ctypes.c_int * 3)(), (ctypes.c_int * 3)()
        _check(library().fcm_plan_box_info(self.handle, L, g, c), "fcm_plan_box_info")
        return dict(L=tuple(L), grid=tuple(g), cells=tuple(c))

    def new_grid(self):
        import torch
        return torch.empty(self.grid_shape, dtype=self.grid_dtype, device="cuda")

    def mobility(self, pos, F, T=None, V=None, Omega=None, stream=None, want_omega=True):
        import torch
        N = self.N
        if V is None:
            V = torch.empty((N, 3), dtype=torch.float64, device=pos.device)
        if Omega is None and want_omega:
            Omega = torch.empty((N, 3), dtype=torch.float64, device=pos.device)
        f64 = torch.float64
        _check(library().fcm_mobility(self.handle, _ptr(pos, "pos", N, f64), _ptr(F, "F", N, f64),
                                      _ptr(T, "T", N, f64, True), _ptr(V, "V", N, f64),
                                      _ptr(Omega, "Omega", N, f64, True), _stream(stream)),
               "fcm_mobility")
        return V, Omega

    def mobility_repeat(self, F, T=None, V=None, Omega=None, stream=None, want_omega=True):
        """fcm_mobility_repeat: the mobility at the positions of the last mobility call."""
        import torch
        N = self.N
        if V is None:
            V = torch.empty((N, 3), dtype=torch.float64, device=F.device)
        if Omega is None and want_omega:
            Omega = torch.empty((N, 3), dtype=torch.float64, device=F.device)
        f64 = torch.float64
        _check(library().fcm_mobility_repeat(self.handle, _ptr(F, "F", N, f64),
                                             _ptr(T, "T", N, f64, True), _ptr(V, "V", N, f64),
                                             _ptr(Omega, "Omega", N, f64, True), _stream(stream)),
               "fcm_mobility_repeat")
        return V, Omega

    def brownian(self, pos, xi_grid, xi_pair, kT, tol=1e-8, V=None, max_iter=48, stream=None):
        """fcm_brownian: Brownian velocities from the given noise; returns (V, Lanczos steps)."""
        import torch
        N = self.N
        if V is None:
            V = torch.empty((N, 3), dtype=torch.float64, device=pos.device)
        self._check_grid(xi_grid)
        _check(library().fcm_brownian_reserve(self.handle, int(max_iter)), "fcm_brownian_reserve")
        it = ctypes.c_int()
        f64 = torch.float64
        _check(library().fcm_brownian(self.handle, _ptr(pos, "pos", N, f64), ctypes.c_void_p(xi_grid.data_ptr()),
                                      _ptr(xi_pair, "xi_pair", N, f64, True), float(kT), float(tol),
                                      _ptr(V, "V", N, f64), ctypes.byref(it), _stream(stream)),
               "fcm_brownian")
        return V, it.value

    def spread(self, pos, F, T=None, grid_out=None, stream=None):
        import torch
        N = self.N
        g = self.new_grid() if grid_out is None else grid_out
        self._check_grid(g)
        f64 = torch.float64
        _check(library().fcm_spread(self.handle, _ptr(pos, "pos", N, f64), _ptr(F, "F", N, f64),
                                    _ptr(T, "T", N, f64, True), ctypes.c_void_p(g.data_ptr()),
                                    _stream(stream)), "fcm_spread")
        return g

    def solve(self, grid, stream=None):
        self._check_grid(grid)
        _check(library().fcm_solve(self.handle, ctypes.c_void_p(grid.data_ptr()), _stream(stream)),
               "fcm_solve")
        return grid

    def interp(self, pos, grid, V=None, Omega=None, stream=None, want_omega=True):
        import torch
        N = self.N
        self._check_grid(grid)
        if V is None:
            V = torch.empty((N, 3), dtype=torch.float64, device=pos.device)
        if Omega is None and want_omega:
            Omega = torch.empty((N, 3), dtype=torch.float64, device=pos.device)
        f64 = torch.float64
        _check(library().fcm_interp(self.handle, _ptr(pos, "pos", N, f64), ctypes.c_void_p(grid.data_ptr()),
                                    _ptr(V, "V", N, f64), _ptr(Omega, "Omega", N, f64, True),
                                    _stream(stream)), "fcm_interp")
        return V, Omega

    def correct(self, pos, F, T, V, Omega=None, stream=None):
        import torch
        N = self.N
        f64 = torch.float64
        _check(library().fcm_correct(self.handle, _ptr(pos, "pos", N, f64), _ptr(F, "F", N, f64),
                                     _ptr(T, "T", N, f64, True), _ptr(V, "V", N, f64),
                                     _ptr(Omega, "Omega", N, f64, True), _stream(stream)),
               "fcm_correct")
        return V, Omega

    def set_timing(self, enable=True, stage=None):
        """Per-stage HIP-event timing of later calls: every stage, or with
        `stage` (a name of STAGES) that stage alone."""
        mode = 0 if not enable else (1 if stage is None else 2 + STAGES.index(stage))
        _check(library().fcm_plan_set_timing(self.handle, mode), "fcm_plan_set_timing")

    def stage_times(self):
        """Per-stage milliseconds summed over the calls recorded since the last read."""
        ms = (ctypes.c_double * len(STAGES))()
        n = ctypes.c_int()
        _check(library().fcm_plan_stage_times(self.handle, ms, ctypes.byref(n)), "fcm_plan_stage_times")
        return dict(zip(STAGES, list(ms))), n.value

    def last_error(self):
        return library().fcm_plan_last_error(self.handle)

    def _check_grid(self, g):
        n = self.grid_shape[1] * self.grid_shape[2] * self.grid_shape[3]
        if (not g.is_cuda or g.dtype != self.grid_dtype or not g.is_contiguous()
                or g.numel() != 3 * n):
            raise ValueError(f"grid must be a contiguous device tensor of shape {self.grid_shape}, "
                             f"{self.grid_dtype}")

    def close(self):
        if self._h is not None:
            library().fcm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
