"""Python binding of the continuous-batching server (fe_server_* in
include/fe.h). Marshalling only: admission, copies, batching and timing run
in libfe's scheduler thread."""
from __future__ import annotations

import ctypes

from . import fe

GPU, FAKE = 0, 1


class ServerConfig(ctypes.Structure):
    _fields_ = [("kinds", ctypes.POINTER(fe.BatchKind)), ("n_kinds", ctypes.c_int32),
                ("max_slots", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_int64),
                ("max_chunks", ctypes.c_int32), ("blocks_per_kind", ctypes.c_int32),
                ("chunk_elems", ctypes.c_int64), ("backend", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("fake_ns_per_elem", ctypes.c_double),
                ("fake_h2d_bytes_per_s", ctypes.c_double), ("fake_tick_overhead_s", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("inputs_on_device", ctypes.c_int32),
                ("n_elem", ctypes.c_int64), ("coords", ctypes.c_void_p), ("coeffs", ctypes.c_void_p),
                ("ld_in", ctypes.c_int64), ("tag", ctypes.c_uint64)]


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("kind", ctypes.c_int32), ("n_elem", ctypes.c_int64), ("out_K", ctypes.c_void_p),
                ("out_F", ctypes.c_void_p), ("ld_out", ctypes.c_int64), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_ready", ctypes.c_double), ("t_done", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "admitted", "completed", "failed",
                                              "in_queue", "in_flight", "bytes_in_use", "bytes_peak",
                                              "elements_done", "ticks")] + \
               [(n, ctypes.c_double) for n in ("p50_s", "p99_s", "mean_s", "mean_queue_s",
                                               "mean_h2d_s", "mean_device_s")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _sigs(L):
    if getattr(L, "_server_sigs", False):
        return
    vp = ctypes.c_void_p
    L.fe_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    L.fe_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.fe_server_poll.argtypes = [vp, ctypes.POINTER(Completion), ctypes.c_int, ctypes.c_double]
    L.fe_server_release.argtypes = [vp, ctypes.c_uint64]
    L.fe_server_stats_get.argtypes = [vp, ctypes.POINTER(Stats)]
    L.fe_server_reset_stats.argtypes = [vp]
    L.fe_server_destroy.argtypes = [vp]
    L.fe_server_now.restype = ctypes.c_double
    L._server_sigs = True


def now() -> float:
    L = fe.lib()
    _sigs(L)
    return float(L.fe_server_now())


class Server:
    def __init__(self, kinds, max_slots=64, hbm_budget_bytes=64 << 30, max_chunks=2048,
                 chunk_elems=4096, blocks_per_kind=0, backend=GPU, fake_ns_per_elem=0.1,
                 fake_h2d_bytes_per_s=50e9, fake_tick_overhead_s=20e-6):
        """kinds: list of (Problem, elem, Rule)."""
        L = fe.lib()
        fe._batch_sigs(L)
        _sigs(L)
        self.kinds = list(kinds)
        arr = (fe.BatchKind * len(kinds))()
        for i, (p, elem, rule) in enumerate(kinds):
            arr[i].problem = p
            arr[i].elem_type = fe.ELEM.get(elem, elem)
            arr[i].n_q = rule.n_q
            arr[i].xi = rule.c.xi
            arr[i].w = rule.c.w
        cfg = ServerConfig(arr, len(kinds), max_slots, hbm_budget_bytes, max_chunks, blocks_per_kind,
                           chunk_elems, backend, 0, fake_ns_per_elem, fake_h2d_bytes_per_s,
                           fake_tick_overhead_s)
        self._h = ctypes.c_void_p()
        fe._check(L.fe_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))
        self._keep = {}

    def submit(self, kind, n_elem, coords_ptr, coeffs_ptr=None, on_device=False, ld_in=0, tag=0,
               keep=None) -> int:
        """Queue one request. coords_ptr / coeffs_ptr are addresses (host or
        device) of arrays with leading dimension ld_in (default n_elem);
        `keep` is held until the request is released (the buffers must
        outlive the request)."""
        r = Request(kind, 1 if on_device else 0, n_elem, coords_ptr, coeffs_ptr,
                    ld_in if ld_in else n_elem, tag)
        rid = ctypes.c_uint64()
        fe._check(fe.lib().fe_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)))
        if keep is not None:
            self._keep[rid.value] = keep
        return rid.value

    def poll(self, max_n=256, timeout_s=0.0):
        buf = (Completion * max_n)()
        n = fe.lib().fe_server_poll(self._h, buf, max_n, timeout_s)
        if n < 0:
            raise fe.FeError(-n, "poll failed")
        return [buf[i] for i in range(n)]

    def release(self, rid: int) -> None:
        fe._check(fe.lib().fe_server_release(self._h, rid))
        self._keep.pop(rid, None)

    def stats(self) -> dict:
        st = Stats()
        fe._check(fe.lib().fe_server_stats_get(self._h, ctypes.byref(st)))
        return st.as_dict()

    def reset_stats(self) -> None:
        fe._check(fe.lib().fe_server_reset_stats(self._h))

    def close(self) -> None:
        if self._h:
            fe.lib().fe_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
