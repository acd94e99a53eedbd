"""Continuous-batching labeling server: Python face of the library's native
server (ccl_server_* in include/ccl.h).

Requests (a device-resident uint8 image, a connectivity, optionally a
threshold level) arrive at any time.  The scheduler runs in the library, on
its own thread, without the interpreter lock: it keeps up to `n_streams`
batches in flight on their own HIP streams and, whenever one completes,
launches the requests waiting at that moment as the next batch, so requests
that arrive while others are on the GPU join the next batch and batches on
different streams overlap on the device.  Admission is by HBM footprint: the
server owns `hbm_budget` bytes of workspace split evenly over its streams, a
request joins a batch only if its workspace region fits, and one that could
never fit is rejected at submission.  Latency is measured by the library
from submission to the moment the scheduler sees the batch complete.

Each result is the same whether the image is labeled alone or in a mix:
labels are canonical (components ranked by smallest raster index) and do
not depend on tiling, batching or scheduling.
"""
from __future__ import annotations

import collections
import ctypes

import torch

from . import ccl


class Request:
    """One submitted image.  `labels` is valid once `wait()` returned (or
    `done` is true); `latency` is in seconds."""

    __slots__ = ("server", "rid", "img", "conn", "labels", "_status", "_lat")

    def __init__(self, server, rid, img, conn, labels, status):
        self.server, self.rid, self.img, self.conn, self.labels = server, rid, img, conn, labels
        self._status = status
        self._lat = None

    def _poll(self, block: bool):
        if self._status != "queued":
            return
        lat = ctypes.c_double()
        fn = ccl._lib.ccl_server_wait if block else ccl._lib.ccl_server_poll
        st = fn(self.server._h, self.rid, ctypes.byref(lat))
        if block:
            ccl._check(st)
            st = 1
        elif st < 0:
            ccl._check(st)
        if st == 1:
            self._status = "done"
            self._lat = lat.value * 1e-3

    def wait(self) -> bool:
        self._poll(True)
        return self._status == "done"

    @property
    def done(self) -> bool:
        self._poll(False)
        return self._status == "done"

    @property
    def status(self) -> str:
        self._poll(False)
        return self._status

    @property
    def latency(self):
        self._poll(False)
        return self._lat


class Server:
    def __init__(self, hbm_budget: int = 8 << 30, n_streams: int = 3, max_batch: int = 64,
                 max_batch_pixels: int = 96 << 20, tile: int = 0, device="cuda:0"):
        self.device = torch.device(device)
        cfg = ccl.ServerConfig(n_streams=n_streams, max_batch=max_batch, max_batch_pixels=max_batch_pixels,
                               hbm_budget=int(hbm_budget), tile=tile)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            ccl._check(ccl._lib.ccl_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._final = None
        # label buffers of requests not yet seen complete: kept referenced so
        # that the allocator cannot hand their memory out while the GPU writes
        self._inflight = collections.deque()

    def submit(self, img: torch.Tensor, conn: int = 8, out: torch.Tensor | None = None, level: int = 0,
               scan: int = ccl.SCAN_PAIR, gray: bool = False, ready=True, order: int = ccl.CANONICAL,
               tile: int = 0) -> Request:
        """Queue one image.  ready: True = the image and `out` are ready once
        the current stream's work so far is (the library waits for it on the
        device), a torch stream = once that stream's work is, False = now."""
        H, W, stride = ccl._img_geometry(img)
        if out is None:
            out = torch.empty((H, W), dtype=torch.int32, device=img.device)
        ccl._check_out(out, img)
        d = ccl.ImageDescEx(img=img.data_ptr(), H=H, W=W, stride=stride, conn=int(conn), labels=out.data_ptr(),
                            num_components=None, level=int(level), scan=int(scan), gray=int(bool(gray)),
                            order=int(order), tile=int(tile))
        t = ctypes.c_uint64()
        rs = None if ready is False else ccl._stream_handle(None if ready is True else ready)
        st = ccl._lib.ccl_server_submit(self._h, ctypes.byref(d), rs, ctypes.byref(t))
        if st == ccl.STATUS["CCL_ERR_BUDGET"]:
            return Request(self, 0, img, conn, None, "rejected")
        ccl._check(st)
        r = Request(self, t.value, img, conn, out, "queued")
        self._inflight.append(r)
        while self._inflight and self._inflight[0].done:
            self._inflight.popleft()
        return r

    def drain(self):
        ccl._check(ccl._lib.ccl_server_drain(self._h))
        for r in self._inflight:   # all complete now: record their latencies
            r._poll(False)
        self._inflight.clear()

    def close(self, drain: bool = True):
        if self._h:
            if drain:
                self.drain()
            self._final = self._stats()
            st = ccl._lib.ccl_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._inflight.clear()
            ccl._check(st)

    def _stats(self):
        s = ccl.ServerStats()
        ccl._check(ccl._lib.ccl_server_stats_get(self._h, ctypes.byref(s)))
        return s

    def stats(self, t0: float | None = None, t1: float | None = None) -> dict:
        """Counters and latency percentiles (ms) since creation (a closed
        server reports its final ones); gpx_per_s over [t0, t1] seconds."""
        s = self._stats() if self._h else self._final
        out = {
            "submitted": s.submitted, "completed": s.completed, "rejected": s.rejected, "batches": s.batches,
            "max_batches_in_flight": s.in_flight_max, "p50_ms": s.p50_ms, "p99_ms": s.p99_ms,
            "mean_ms": s.mean_ms, "pixels_completed": s.pixels_completed,
        }
        if t0 is not None and t1 is not None:
            out["gpx_per_s"] = s.pixels_completed / max(t1 - t0, 1e-9) / 1e9
        return out

    def latency_stats(self, first: int, last: int) -> dict:
        """p50 / p99 / mean latency (ms) of the completed requests with
        tickets first..last (the library keeps each request's latency)."""
        lat = []
        for t in range(first, last + 1):
            v = ctypes.c_double()
            if ccl._lib.ccl_server_poll(self._h, t, ctypes.byref(v)) == 1:
                lat.append(v.value)
        lat.sort()
        n = len(lat)
        if not n:
            return {"p50_ms": None, "p99_ms": None, "mean_ms": None, "n": 0}
        return {"p50_ms": lat[min(n - 1, int(0.5 * n))], "p99_ms": lat[min(n - 1, int(0.99 * n))],
                "mean_ms": sum(lat) / n, "n": n}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
