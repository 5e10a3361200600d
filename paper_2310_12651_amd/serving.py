"""ctypes binding of the request server (include/fcm_server.h) and a driver that
replays a timed request stream through it.

Argument marshalling only: admission, plan caching, stream slots and the
evaluations themselves run in libfcm.so.
"""

import ctypes
import time

from ._lib import FCM_FP32_BULK, FCM_OK, FCMError, library

FCM_EBUSY = -6


class Request(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("L", ctypes.c_double), ("a", ctypes.c_double),
                ("sigma_delta", ctypes.c_double), ("grid", ctypes.c_int), ("r_cut", ctypes.c_double),
                ("support", ctypes.c_int), ("eta", ctypes.c_double),
                ("pos", ctypes.c_void_p), ("F", ctypes.c_void_p), ("T", ctypes.c_void_p),
                ("V", ctypes.c_void_p), ("Omega", ctypes.c_void_p), ("after_stream", ctypes.c_void_p)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("max_bytes", ctypes.c_int64), ("slots", ctypes.c_int), ("precision", ctypes.c_int),
                ("kahan", ctypes.c_int), ("max_queue", ctypes.c_int), ("max_points", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("plans_built", ctypes.c_int64), ("plans_rebound", ctypes.c_int64),
                ("plans_evicted", ctypes.c_int64), ("bytes_in_use", ctypes.c_int64),
                ("bytes_peak", ctypes.c_int64), ("inflight_peak", ctypes.c_int)]


SERVER_EXPORTS = ["fcm_server_options_default", "fcm_server_create", "fcm_server_submit",
                  "fcm_server_submit_box", "fcm_server_poll", "fcm_server_wait", "fcm_server_get_stats",
                  "fcm_server_destroy"]

_bound = False


def _lib():
    global _bound
    lib = library()
    if not _bound:
        vp, ci, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        sig = {
            "fcm_server_options_default": ([ctypes.POINTER(ServerOptions)], ci),
            "fcm_server_create": ([ctypes.POINTER(vp), ctypes.POINTER(ServerOptions)], ci),
            "fcm_server_submit": ([vp, ctypes.POINTER(Request), ctypes.POINTER(i64)], ci),
            "fcm_server_submit_box": ([vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ci), ctypes.POINTER(i64)], ci),
            "fcm_server_poll": ([vp, i64, ctypes.POINTER(ci)], ci),
            "fcm_server_wait": ([vp, i64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], ci),
            "fcm_server_get_stats": ([vp, ctypes.POINTER(ServerStats)], ci),
            "fcm_server_destroy": ([vp], ci),
        }
        for name, (args, res) in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _bound = True
    return lib


def _check(st, where):
    if st != FCM_OK:
        raise FCMError(st, where)


class Server:
    """Continuous-batching request server on the current device."""

    def __init__(self, slots=8, precision=FCM_FP32_BULK, kahan=0, max_bytes=0, max_queue=4096,
                 max_points=None):
        lib = _lib()
        o = ServerOptions()
        _check(lib.fcm_server_options_default(ctypes.byref(o)), "fcm_server_options_default")
        o.slots, o.precision, o.kahan, o.max_bytes, o.max_queue = slots, precision, kahan, max_bytes, max_queue
        if max_points is not None:
            o.max_points = int(max_points)
        h = ctypes.c_void_p()
        _check(lib.fcm_server_create(ctypes.byref(h), ctypes.byref(o)), "fcm_server_create")
        self._h = h

    def submit(self, N, L, a, Sigma, grid, r_cut, pos, F, T=None, V=None, Omega=None, support=0, eta=1.0,
               stream=None):
        """Queue one evaluation; it runs after the work queued so far on
        ``stream`` (default: the current stream, where torch wrote the inputs).
        ``L`` and ``grid`` may be three values (x, y, z) for a rectangular box
        (fcm_server_submit_box)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        box = hasattr(L, "__len__") or hasattr(grid, "__len__")
        L3 = tuple(float(v) for v in L) if hasattr(L, "__len__") else (float(L),) * 3
        g3 = tuple(int(v) for v in grid) if hasattr(grid, "__len__") else (int(grid),) * 3
        r = Request(N=int(N), L=L3[0], a=float(a), sigma_delta=float(Sigma), grid=g3[0],
                    r_cut=float(r_cut), support=int(support), eta=float(eta),
                    pos=pos.data_ptr(), F=F.data_ptr(), T=None if T is None else T.data_ptr(),
                    V=V.data_ptr(), Omega=None if Omega is None else Omega.data_ptr(),
                    after_stream=stream.cuda_stream)
        t = ctypes.c_int64()
        if box:
            st = _lib().fcm_server_submit_box(self._h, ctypes.byref(r), (ctypes.c_double * 3)(*L3),
                                              (ctypes.c_int * 3)(*g3), ctypes.byref(t))
            _check(st, "fcm_server_submit_box")
        else:
            st = _lib().fcm_server_submit(self._h, ctypes.byref(r), ctypes.byref(t))
            _check(st, "fcm_server_submit")
        return t.value

    def poll(self, ticket):
        s = ctypes.c_int()
        st = _lib().fcm_server_poll(self._h, int(ticket), ctypes.byref(s))
        return s.value, st

    def wait(self, ticket):
        q, r = ctypes.c_double(), ctypes.c_double()
        st = _lib().fcm_server_wait(self._h, int(ticket), ctypes.byref(q), ctypes.byref(r))
        return st, q.value, r.value

    def stats(self):
        s = ServerStats()
        _check(_lib().fcm_server_get_stats(self._h, ctypes.byref(s)), "fcm_server_get_stats")
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self._h is not None:
            _lib().fcm_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def replay(server, reqs, tensors, arrivals=None):
    """Submit requests at their arrival offsets (seconds, host clock; None =
    all at once), wait for all, and return per-request latencies (submit to
    completion, ms) and the makespan (s)."""
    t0 = time.perf_counter()
    tickets = []
    for i, r in enumerate(reqs):
        if arrivals is not None:
            delay = arrivals[i] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
        Y, F, T, V, W = tensors[i]
        tickets.append(server.submit(r["N"], r["L"], r["a"], r["Sigma"], r["grid"], r["R_c"], Y, F, T, V, W,
                                     support=r.get("M_G", 0), eta=r.get("eta", 1.0)))
    lat = []
    for t in tickets:
        st, q, run = server.wait(t)
        if st != FCM_OK:
            raise FCMError(st, "request")
        lat.append(q + run)
    return lat, time.perf_counter() - t0


def run_sequential(server, reqs, tensors):
    """One request at a time: submit, wait, next (closed loop)."""
    t0 = time.perf_counter()
    lat = []
    for i, r in enumerate(reqs):
        Y, F, T, V, W = tensors[i]
        t = server.submit(r["N"], r["L"], r["a"], r["Sigma"], r["grid"], r["R_c"], Y, F, T, V, W,
                          support=r.get("M_G", 0), eta=r.get("eta", 1.0))
        st, q, run = server.wait(t)
        if st != FCM_OK:
            raise FCMError(st, "request")
        lat.append(q + run)
    return lat, time.perf_counter() - t0
