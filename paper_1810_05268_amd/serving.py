"""Continuous-batching shot-gradient server on one GPU (binding of the C engine).

The engine (``wv_engine_*`` in include/wv.h) admits queued requests first fit in
arrival order whenever a worker stream and a contiguous slice of the device pool
(workspace plus checkpoint arena) are free, and runs the admitted shots
concurrently on their own HIP streams; with batching on, 2-D requests that share a
grid and schedule run together in one persistent launch.  This module owns the pool
tensor, keeps each request's device buffers alive until it completes, and replays
timed request streams.  No solver arithmetic happens here.
"""
from __future__ import annotations

import ctypes as C
import time

import torch

from . import _binding as B


class Engine:
    def __init__(self, pool_bytes: int, max_active: int = 4, device: str = "cuda", max_batch: int = 0):
        self.device = torch.device(device)
        self._pool = torch.empty(int(pool_bytes) + 256, dtype=torch.uint8, device=self.device)
        off = (-self._pool.data_ptr()) % 256
        self._h = C.c_void_p()
        torch.cuda.synchronize(self.device)
        B._check(B.lib().wv_engine_create(self._pool.data_ptr() + off, int(pool_bytes), int(max_active),
                                          C.byref(self._h)), "wv_engine_create")
        if max_batch > 1:
            B._check(B.lib().wv_engine_set_batching(self._h, int(max_batch)), "wv_engine_set_batching")
        self._live = {}

    def submit(self, shot, d_obs, mem_budget: int, tol: float = 0.0, ratio_hint: float = 0.0,
               grad=None) -> int:
        """shot: a DeviceShot (its velocity, wavelet and geometry); d_obs: device data."""
        g = grad if grad is not None else torch.empty(shot.shape, dtype=torch.float64, device=self.device)
        # inputs are produced on torch's stream; the engine's streams do not wait for it
        torch.cuda.current_stream(self.device).synchronize()
        rid = B.lib().wv_engine_submit(self._h, C.byref(shot.pb.model), C.byref(shot.pb.geom), B._ptr(d_obs),
                                       int(mem_budget), float(tol), float(ratio_hint), B._ptr(g), None)
        if rid < 0:
            raise B.WvError(rid, "wv_engine_submit")
        self._live[rid] = (shot, d_obs, g)
        return rid

    def wait(self, rid: int, timeout_ms: float = -1.0):
        res = B.WvResult()
        rc = B.lib().wv_engine_wait(self._h, int(rid), float(timeout_ms), C.byref(res))
        if rc == B.WV_ETIMEOUT:
            return None
        B._check(rc, "wv_engine_wait")
        shot, d_obs, g = self._live.pop(rid)
        out = {"status": res.status, "misfit": res.misfit, "t_submit_ms": res.t_submit_ms,
               "t_start_ms": res.t_start_ms, "t_end_ms": res.t_end_ms, "stats": res.stats.as_dict(), "grad": g}
        return out

    def pending(self):
        q, a = C.c_int(0), C.c_int(0)
        B._check(B.lib().wv_engine_pending(self._h, C.byref(q), C.byref(a)), "wv_engine_pending")
        return q.value, a.value

    def close(self):
        if self._h:
            B.lib().wv_engine_destroy(self._h)
            self._h = C.c_void_p()
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:        # noqa: BLE001 - interpreter shutdown
            pass


def replay(engine: Engine, items, time_scale: float = 1.0, timeout_s: float | None = None):
    """Submit (arrival_s, shot, d_obs, mem_budget, tol, hint) items at their arrival times
    (scaled by time_scale) and wait for all.  Returns per-request results with latency
    measured from arrival (submission) to completion.  With timeout_s, a request not done
    that many seconds after the last submission raises TimeoutError."""
    t0 = time.perf_counter()
    ids = []
    for arrival, shot, d_obs, budget, tol, hint in items:
        dt = arrival * time_scale - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        ids.append(engine.submit(shot, d_obs, budget, tol, hint))
    deadline = None if timeout_s is None else time.perf_counter() + timeout_s
    out = []
    for rid in ids:
        left = -1.0 if deadline is None else max(0.0, deadline - time.perf_counter()) * 1e3
        r = engine.wait(rid, left)
        if r is None:
            raise TimeoutError(f"serving request {rid} not done {timeout_s} s after the last arrival")
        r["latency_ms"] = r["t_end_ms"] - r["t_submit_ms"]
        r["queue_ms"] = r["t_start_ms"] - r["t_submit_ms"]
        out.append(r)
    wall = time.perf_counter() - t0
    return out, wall
