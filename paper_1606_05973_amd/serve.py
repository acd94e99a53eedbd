"""Continuous-batching labeling server.

Requests (a device-resident uint8 image and a connectivity) arrive at any
time.  A scheduler thread keeps up to `n_streams` batches in flight on their
own HIP streams: whenever a stream is free and HBM allows, it admits the
waiting requests into a new batch (one ccl_label_batch call), so requests
that arrive while others are on the GPU join the next batch instead of
waiting for the queue to drain, and batches on different streams overlap on
the device.  Admission is by HBM footprint: each request needs its label
buffer (4 B/px) and its share of the batch workspace
(ccl_batch_workspace_bytes); the footprint of everything in flight stays
under `hbm_budget` bytes, and a request that could never fit is rejected at
submission.  Completion is detected with events; latency is measured from
submission to the moment the scheduler sees the batch's event complete.

Each result is the same whether the image is labeled alone or in a mix:
labels are canonical (components ranked by smallest raster index) and do
not depend on tiling, batching or scheduling.
"""
from __future__ import annotations

import collections
import statistics
import threading
import time

import torch

from . import ccl


class Request:
    __slots__ = ("rid", "img", "conn", "t_submit", "t_launch", "t_done", "labels", "status", "footprint", "_done")

    def __init__(self, rid, img, conn):
        self.rid = rid
        self.img = img
        self.conn = conn
        self.t_submit = time.perf_counter()
        self.t_launch = None
        self.t_done = None
        self.labels = None
        self.status = "queued"
        self.footprint = 0
        self._done = threading.Event()

    def wait(self, timeout=None) -> bool:
        return self._done.wait(timeout)

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_submit


class Server:
    def __init__(self, hbm_budget: int = 8 << 30, n_streams: int = 3, max_batch: int = 64,
                 max_batch_pixels: int = 96 << 20, tile: int = 0, device="cuda:0", on_done=None):
        self.budget = int(hbm_budget)
        self.on_done = on_done      # called with each finished Request, on the scheduler thread
        self.max_batch = max_batch
        self.max_batch_pixels = max_batch_pixels
        self.tile = tile
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]
        # Grow each stream's library workspace once, up front, to what a full
        # batch needs, so that serving never waits on a reallocation.
        side = int(max_batch_pixels ** 0.5) + 1
        ws = ccl.batch_workspace_bytes([(side, side)] * 2, 4, tile) + max_batch * (1 << 20)
        with torch.cuda.device(self.device):
            for st in self.streams:
                ccl.reserve(ws, st)
        self.free_streams = list(range(n_streams))
        self.pending = collections.deque()
        self.inflight = []          # (stream index, event, [requests], footprint)
        self.used = 0               # bytes held by in-flight batches
        self.lock = threading.Lock()
        self.wake = threading.Event()
        self.stop_flag = False
        self.done = []
        self.rejected = 0
        self.batches = 0
        self.max_inflight = 0
        self._next_id = 0
        self.thread = threading.Thread(target=self._loop, name="ccl-serve", daemon=True)
        self.thread.start()

    # ------------------------------------------------------------------ API
    def request_footprint(self, H: int, W: int, conn: int) -> int:
        return H * W * 4 + ccl.workspace_bytes(H, W, conn, self.tile)

    def submit(self, img: torch.Tensor, conn: int = 8) -> Request:
        with self.lock:
            r = Request(self._next_id, img, conn)
            self._next_id += 1
        H, W = img.shape
        r.footprint = self.request_footprint(H, W, conn)
        if r.footprint > self.budget:
            r.status = "rejected"
            r.t_done = time.perf_counter()
            with self.lock:
                self.rejected += 1
            r._done.set()
            return r
        with self.lock:
            self.pending.append(r)
        self.wake.set()
        return r

    def close(self, drain: bool = True):
        if drain:
            while True:
                with self.lock:
                    if not self.pending and not self.inflight:
                        break
                time.sleep(1e-4)
        self.stop_flag = True
        self.wake.set()
        self.thread.join()

    def stats(self, t0: float, t1: float):
        lat = sorted(r.latency for r in self.done if r.status == "done")
        px = sum(r.img.numel() for r in self.done if r.status == "done")

        def pct(q):
            return lat[min(len(lat) - 1, int(q * len(lat)))] * 1e3 if lat else None
        return {
            "completed": len(lat), "rejected": self.rejected, "batches": self.batches,
            "max_batches_in_flight": self.max_inflight,
            "p50_ms": pct(0.50), "p99_ms": pct(0.99), "mean_ms": statistics.mean(lat) * 1e3 if lat else None,
            "gpx_per_s": px / max(t1 - t0, 1e-9) / 1e9,
        }

    # ------------------------------------------------------------ scheduler
    def _retire(self):
        still = []
        for si, ev, reqs, fp in self.inflight:
            if ev.query():
                now = time.perf_counter()
                for r in reqs:
                    r.t_done = now
                    r.status = "done"
                    r._done.set()
                    if self.on_done is not None:
                        self.on_done(r)
                self.done.extend(reqs)
                self.used -= fp
                self.free_streams.append(si)
            else:
                still.append((si, ev, reqs, fp))
        self.inflight = still

    def _admit(self) -> bool:
        launched = False
        while self.free_streams:
            batch, fp, px = [], 0, 0
            with self.lock:
                while self.pending and len(batch) < self.max_batch:
                    r = self.pending[0]
                    n = r.img.numel()
                    if batch and px + n > self.max_batch_pixels:
                        break
                    if self.used + fp + r.footprint > self.budget:
                        break
                    self.pending.popleft()
                    batch.append(r)
                    fp += r.footprint
                    px += n
            if not batch:
                return launched
            si = self.free_streams.pop()
            s = self.streams[si]
            with torch.cuda.stream(s):
                outs = [torch.empty(tuple(r.img.shape), dtype=torch.int32, device=self.device) for r in batch]
                now = time.perf_counter()
                for r, o in zip(batch, outs):
                    r.labels = o
                    r.t_launch = now
                    r.status = "running"
                ccl.label_batch([r.img for r in batch], [r.conn for r in batch], outs=outs, tile=self.tile, stream=s)
                ev = torch.cuda.Event()
                ev.record(s)
            self.used += fp
            self.batches += 1
            self.inflight.append((si, ev, batch, fp))
            self.max_inflight = max(self.max_inflight, len(self.inflight))
            launched = True
        return launched

    def _loop(self):
        torch.cuda.set_device(self.device)
        while True:
            self._retire()
            launched = self._admit()
            with self.lock:
                idle = not self.pending and not self.inflight
            if self.stop_flag and idle:
                return
            if idle:
                self.wake.wait(0.001)
                self.wake.clear()
            elif not launched:
                time.sleep(20e-6)
