"""Tile-shape autotuner for the labeling library.

The library exposes a few tile configurations (ccl.tile_configs()).  Which
one is fastest depends on the image size (how many tiles fill the GPU, how
much edge merging a tile shape causes) and on connectivity.  The tuner times
every configuration on a representative image of a size bucket and keeps the
winner in a JSON cache keyed by GPU architecture, connectivity and bucket, so
later calls pick a tile without timing.

Buckets: log2 of the pixel count rounded to the nearest integer, and the
aspect class (wide / square / tall).  Batches are tuned as a whole
(tune_batch): every configuration labels the batch once, the fastest wins.

plan_batch tunes a batch's schedule as well: each size bucket of the batch
gets the tile that labels that bucket's images fastest, and the whole batch
is then timed both ways -- one tile for every image (one launch group per
kind of image) and the per-bucket tiles (one launch group per distinct tile,
so more launches, each group's latency-bound phases one after another) --
and the faster assignment is kept.
"""
from __future__ import annotations

import json
import math
import os
import threading

import torch

from . import ccl, inputs

_DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_1606_05973_amd", "tiles.json")


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def bucket(H: int, W: int, conn: int) -> str:
    area = max(1, H * W)
    a = W / max(H, 1)
    shape = "wide" if a > 2 else ("tall" if a < 0.5 else "square")
    return f"c{conn}_a{int(round(math.log2(area)))}_{shape}"


def _time(fn, reps: int = 3) -> float:
    fn()  # warm
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        fn()
        e.record()
        torch.cuda.synchronize()
        best = min(best, s.elapsed_time(e))
    return best


class Autotuner:
    def __init__(self, cache_path: str | None = None):
        self.path = cache_path or os.environ.get("CCL_TUNE_CACHE", _DEFAULT_CACHE)
        self._lock = threading.Lock()
        self.cache = {}
        if os.path.exists(self.path):
            try:
                with open(self.path) as f:
                    self.cache = json.load(f)
            except (OSError, ValueError):
                self.cache = {}

    def _key(self, k: str) -> str:
        return f"{_arch()}/{k}"

    def save(self):
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(self.cache, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def timings(self, H: int, W: int, conn: int, img: torch.Tensor | None = None, reps: int = 3):
        """{tile id: ms} for every configuration on img (or a Bernoulli 0.5 image)."""
        if img is None:
            img = inputs.bernoulli(H, W, 0.5, seed=1234, device="cuda")
        out = torch.empty((H, W), dtype=torch.int32, device=img.device)
        res = {}
        for tid in range(1, len(ccl.tile_configs()) + 1):
            ccl.reserve(ccl.workspace_bytes(H, W, conn, tid))
            res[tid] = _time(lambda: ccl.label(img, conn, out=out, tile=tid), reps)
        return res

    def best_tile(self, H: int, W: int, conn: int, img: torch.Tensor | None = None) -> int:
        k = self._key(bucket(H, W, conn))
        with self._lock:
            if k in self.cache:
                return int(self.cache[k]["tile"])
        t = self.timings(H, W, conn, img)
        best = min(t, key=t.get)
        with self._lock:
            self.cache[k] = {"tile": best, "ms": {str(a): round(b, 4) for a, b in t.items()}}
            self.save()
        return best

    def tune_batch(self, imgs, conns, key: str | None = None, reps: int = 2) -> int:
        """Fastest tile configuration for labeling this batch as one call."""
        if key is not None:
            with self._lock:
                kk = self._key("batch/" + key)
                if kk in self.cache:
                    return int(self.cache[kk]["tile"])
        outs = [torch.empty(tuple(im.shape), dtype=torch.int32, device=im.device) for im in imgs]
        shapes = [tuple(im.shape) for im in imgs]
        res = {}
        for tid in range(1, len(ccl.tile_configs()) + 1):
            ccl.reserve(ccl.batch_workspace_bytes(shapes, conns, tid))
            res[tid] = _time(lambda: ccl.label_batch(imgs, conns, outs=outs, tile=tid), reps)
        best = min(res, key=res.get)
        if key is not None:
            with self._lock:
                self.cache[self._key("batch/" + key)] = {"tile": best, "ms": {str(a): round(b, 4) for a, b in res.items()}}
                self.save()
        return best

    def plan_batch(self, imgs, conns, key: str | None = None, reps: int = 3) -> dict:
        """Per-image tile ids for labeling this batch as one call, and the
        schedule they come from: {"tiles": [...], "schedule": "one tile" or
        "per bucket", "one_tile": id, "ms": {"one tile": t1, "per bucket":
        t2}, "buckets": {bucket: id}}."""
        if key is not None:
            with self._lock:
                kk = self._key("plan/" + key)
                if kk in self.cache and len(self.cache[kk]["tiles"]) == len(imgs):
                    return dict(self.cache[kk])
        n = len(imgs)
        conns = list(conns) if isinstance(conns, (list, tuple)) else [conns] * n
        outs = [torch.empty(tuple(im.shape), dtype=torch.int32, device=im.device) for im in imgs]
        shapes = [tuple(im.shape) for im in imgs]
        ntiles = len(ccl.tile_configs())
        ccl.reserve(max(ccl.batch_workspace_bytes(shapes, conns, t) for t in range(1, ntiles + 1)))
        whole = {t: _time(lambda: ccl.label_batch(imgs, conns, outs=outs, tile=t), reps)
                 for t in range(1, ntiles + 1)}
        one = min(whole, key=whole.get)
        groups = {}
        for i, (H, W) in enumerate(shapes):
            groups.setdefault(bucket(H, W, conns[i]), []).append(i)
        per = {}
        for b, idx in groups.items():
            sub, so, sc = [imgs[i] for i in idx], [outs[i] for i in idx], [conns[i] for i in idx]
            tt = {t: _time(lambda: ccl.label_batch(sub, sc, outs=so, tile=t), reps) for t in range(1, ntiles + 1)}
            per[b] = min(tt, key=tt.get)
        tiles = [per[bucket(H, W, conns[i])] for i, (H, W) in enumerate(shapes)]
        t_per = _time(lambda: ccl.label_batch(imgs, conns, outs=outs, tiles=tiles), reps)
        plan = {"one_tile": one, "buckets": per,
                "ms": {"one tile": round(whole[one], 4), "per bucket": round(t_per, 4)}}
        if t_per < whole[one]:
            plan.update(tiles=tiles, schedule="per bucket")
        else:
            plan.update(tiles=[one] * n, schedule="one tile")
        if key is not None:
            with self._lock:
                self.cache[self._key("plan/" + key)] = plan
                self.save()
        return plan


_default = None


def default() -> Autotuner:
    global _default
    if _default is None:
        _default = Autotuner()
    return _default
