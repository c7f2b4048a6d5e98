"""Registration serving loop (ls_server_*) from Python.

A `Server` owns one ls_server: requests are queued with `submit`, admitted
against the device-byte budget, batched with every other active request at
iteration granularity, and collected with `poll` / `wait`.  The arrays a
request references are kept alive here until its result has been polled.
"""

from __future__ import annotations

import ctypes as C
import time

import numpy as np
import torch

from . import lib as L
from .register import default_params, make_pair


class Server:
    def __init__(self, budget_bytes: int = 200 << 30, max_slots: int = 64, chunk_iters: int = 16,
                 instance_headroom: float = 1.5, use_graphs: bool = True, max_active_pixels: int = 0):
        L.load()
        prm = L.ls_server_params(int(budget_bytes), int(max_slots), int(chunk_iters), float(instance_headroom),
                                 1 if use_graphs else 0, int(max_active_pixels))
        h = C.c_void_p()
        L.check(L.load().ls_server_create(C.byref(prm), C.byref(h)))
        self.h = h
        self._keep = {}

    def submit(self, P, Q, cam, c2w_p, c2w_q, rgbP, depthP, rgbQ, depthQ, params: L.ls_reg_params | None = None):
        params = params or default_params()
        pair, keep = make_pair(P, Q, cam, c2w_p, c2w_q, rgbP, depthP, rgbQ, depthQ)
        t = C.c_uint64()
        # the server reads the buffers after the work queued so far on the current stream
        producer = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        L.check(L.load().ls_register_submit(self.h, C.byref(pair), C.byref(params), producer, C.byref(t)))
        self._keep[t.value] = (keep, P, Q, pair.vP + pair.vQ, bool(params.exposure))
        return t.value

    def poll(self, ticket: int):
        """None while running; else dict(T, per_view, residual, status, iters,
        times, exposure) (exposure: per-view (a, b) when requested, else None)."""
        keep = self._keep.get(ticket)
        nv = keep[3] if keep else 1
        per_view = np.zeros((nv, 12), np.float32)
        resid = np.zeros(nv, np.float32)
        expo = np.zeros((nv, 2), np.float32)
        res = L.ls_reg_result()
        res.per_view_T = per_view.ctypes.data_as(C.c_void_p)
        res.residual = resid.ctypes.data_as(C.c_void_p)
        res.exposure = expo.ctypes.data_as(C.c_void_p)
        times = np.zeros(3, np.float64)
        st = L.load().ls_register_poll(self.h, ticket, C.byref(res), times.ctypes.data_as(C.c_void_p))
        if st == L.LS_NOT_READY:
            return None
        self._keep.pop(ticket, None)
        T = np.eye(4)
        T[:3, :] = np.asarray(res.T_PQ, np.float64).reshape(3, 4)
        pv = np.tile(np.eye(4), (nv, 1, 1))
        pv[:, :3, :] = per_view.reshape(nv, 3, 4)
        return dict(T=T, per_view=pv, residual=resid.astype(np.float64), status=int(st), iters=res.iters_done,
                    times=dict(queue=times[0], run=times[1], total=times[2]),
                    exposure=expo.astype(np.float64) if keep and keep[4] else None)

    def wait(self, ticket: int, timeout: float = 600.0, interval: float = 0.002):
        t0 = time.time()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.time() - t0 > timeout:
                raise TimeoutError(f"ticket {ticket} not done after {timeout} s")
            time.sleep(interval)

    def stats(self) -> dict:
        st = L.ls_server_stats()
        L.check(L.load().ls_server_get_stats(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in L.ls_server_stats._fields_ if k != "pad"}

    def close(self):
        if getattr(self, "h", None) is not None:
            L.load().ls_server_destroy(self.h)
            self.h = None
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
