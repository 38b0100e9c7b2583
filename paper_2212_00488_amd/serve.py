"""ctypes front end of the serving runtime (include/stereo.h, stereo_server_*)
and a driver that replays a timed stream of frame requests against it.

The runtime itself (admission, slots, resident graphs, completion) is the
library's C++ worker thread; this module only submits frames at their
arrival times and collects the results.
"""

from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass

import numpy as np

from .binding import ServerConfig, ServerResult, StereoError, lib


class Server:
    """A serving runtime on one HIP device."""

    def __init__(self, device: int = 0, slots: int = 4, mem_budget: int = 0, params=None,
                 max_batch: int = 8):
        cfg = ServerConfig()
        lib().stereo_server_default_config(ctypes.byref(cfg))
        cfg.device, cfg.slots, cfg.mem_budget = device, slots, mem_budget
        cfg.max_batch = max_batch
        if params is not None:
            cfg.params = params
        h = ctypes.c_void_p()
        rc = lib().stereo_server_create(ctypes.byref(h), ctypes.byref(cfg))
        if rc:
            raise StereoError(rc, "stereo_server_create failed")
        self._h = h
        self._keep = {}

    def submit(self, left: np.ndarray, right: np.ndarray, dmax: int, out: np.ndarray, tag: int):
        """Queue one frame: left/right uint8 [H][W][3] host arrays (kept alive
        by the server object until the result is polled), out int16 [H][W]."""
        H, W, _ = left.shape
        for a, dt in ((left, np.uint8), (right, np.uint8), (out, np.int16)):
            if a.dtype != dt or not a.flags["C_CONTIGUOUS"]:
                raise TypeError("frames must be contiguous uint8 images and an int16 map")
        if right.shape != left.shape or out.shape != (H, W):
            raise ValueError("shape mismatch")
        self._keep[tag] = (left, right, out)
        rc = lib().stereo_server_submit(self._h, left.ctypes.data, right.ctypes.data, W, H,
                                        int(dmax), out.ctypes.data, ctypes.c_uint64(tag))
        if rc:
            del self._keep[tag]
            raise StereoError(rc, "stereo_server_submit failed")

    def poll(self, max_results: int = 64, timeout_ms: int = 0):
        buf = (ServerResult * max_results)()
        n = lib().stereo_server_poll(self._h, buf, max_results, int(timeout_ms))
        if n < 0:
            raise StereoError(n, "stereo_server_poll failed")
        out = []
        for i in range(n):
            r = buf[i]
            out.append(dict(tag=int(r.tag), status=int(r.status), slot=int(r.slot),
                            t_submit_ms=r.t_submit_ms, t_admit_ms=r.t_admit_ms,
                            t_done_ms=r.t_done_ms, batch=int(r.batch)))
            self._keep.pop(int(r.tag), None)
        return out

    def last_error(self) -> str:
        return lib().stereo_server_last_error(self._h).decode()

    def close(self):
        if getattr(self, "_h", None):
            lib().stereo_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class StreamReport:
    results: list
    latency_ms: np.ndarray      # t_done - t_submit per request, in request order
    wall_s: float               # first submit to last completion
    throughput: float           # requests per second over wall_s


def replay(server: Server, frames, arrivals_s, dmaxes, outs=None, poll_ms: int = 1):
    """Submit frame i = (left, right) at arrivals_s[i] seconds after the start
    (host clock), collect every result, and report latencies.

    frames: list of (left, right) uint8 host images; dmaxes: per request.
    outs: optional list of int16 output arrays (allocated when None).
    """
    n = len(frames)
    if outs is None:
        outs = [np.empty(f[0].shape[:2], np.int16) for f in frames]
    results = {}
    start = time.perf_counter()
    i = 0
    while len(results) < n:
        now = time.perf_counter() - start
        while i < n and arrivals_s[i] <= now:
            server.submit(frames[i][0], frames[i][1], dmaxes[i], outs[i], i)
            i += 1
        wait = 0
        if i < n:
            wait = max(0, min(poll_ms, int((arrivals_s[i] - now) * 1000)))
        for r in server.poll(256, wait if i < n else poll_ms):
            results[r["tag"]] = r
    res = [results[k] for k in range(n)]
    bad = [r for r in res if r["status"] != 0]
    if bad:
        raise StereoError(bad[0]["status"], f"{len(bad)} frames failed: {server.last_error()}")
    lat = np.array([r["t_done_ms"] - r["t_submit_ms"] for r in res])
    wall = (max(r["t_done_ms"] for r in res) - min(r["t_submit_ms"] for r in res)) / 1000.0
    return StreamReport(res, lat, wall, n / wall), outs
