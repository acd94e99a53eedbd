"""Seeded synthetic input images (binary uint8) for tests and benchmarks.

This module holds none of the labeling arithmetic: it only makes images.  It is
the one piece shared by the CPU oracle side and the GPU side, so both label
the very same bytes.  Every generator is deterministic in its arguments and
runs on any torch device; the integer generators produce identical bytes on
every device.

Workloads standing in for the paper's images (Section V: USC-SIPI Texture /
Aerial / Misc and NLCD 2006 land cover, binarized at luminance 0.5; the
largest is 465.20 MB, Table III).  Those images are not available here:

* ``bernoulli``  -- i.i.d. foreground with probability p.  Pixel (r, c) is
  foreground iff the upper 32 bits of the (r*W + c)-th SplitMix64 output for
  ``seed`` are below floor(p * 2**32).  Exact integer thresholding.
* ``grf``        -- thresholded Gaussian random field: i.i.d. N(0,1) noise
  (Box-Muller on two SplitMix64 streams), smoothed with a periodic Gaussian
  of standard deviation ``sigma`` px (FFT), foreground iff the value exceeds
  its q-quantile (estimated on a strided subsample of at most 2**22 values),
  so about (1-q) of the pixels are foreground.  Blobby, land-cover-like.
* ``adversarial`` -- structured images that stress union-find depth and the
  component count: spiral, checkerboard, all-ones, all-zeros, horizontal /
  vertical / diagonal stripes, comb.
* ``batch_specs`` -- the uneven batch mix: side H log-uniform in [64, 4096],
  aspect log-uniform in [0.25, 4], W = clamp(round(H*aspect), 64, 4096);
  content Bernoulli p ~ U[0.2, 0.8] or GRF sigma ~ U[1, 16] at q = 0.5.
* ``gray``       -- a grayscale image (bytes 0..255) for the fused
  threshold and, quantized to a few levels (``gray(...) // k``), for
  gray-level labeling: a Gaussian random field as in ``grf``, standardized
  and mapped to 128 + 40 * z, rounded and clipped.
* ``serve_specs`` -- a request stream for the server: Poisson arrival times
  at a given rate, 95% of sizes as in ``batch_specs`` and 5% with sides
  log-uniform up to 8192, connectivity 4 or 8 with equal probability.
"""
from __future__ import annotations

import math

import numpy as np
import torch

GOLDEN_GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1


def _s64(v: int) -> int:
    """Two's-complement int64 value with the same bits as the uint64 v."""
    v &= MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def _srl(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of int64 bit patterns."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def splitmix64(index: torch.Tensor, seed: int) -> torch.Tensor:
    """The index-th output (0-based) of SplitMix64 started from state ``seed``.

    Works on int64 tensors holding uint64 bit patterns (wrapping arithmetic).
    """
    z = index.to(torch.int64) + 1
    z = z * _s64(GOLDEN_GAMMA) + _s64(seed)
    z = (z ^ _srl(z, 30)) * _s64(MIX1)
    z = (z ^ _srl(z, 27)) * _s64(MIX2)
    return z ^ _srl(z, 31)


def splitmix64_py(index: int, seed: int) -> int:
    """Pure-Python SplitMix64 (reference for the tensor version)."""
    z = (seed + (index + 1) * GOLDEN_GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * MIX1) & MASK64
    z = ((z ^ (z >> 27)) * MIX2) & MASK64
    return z ^ (z >> 31)


def _alloc(H: int, W: int, stride: int | None, device) -> torch.Tensor:
    if stride is None:
        stride = W
    if stride < W:
        raise ValueError("stride must be >= W")
    buf = torch.zeros((H, stride), dtype=torch.uint8, device=device)
    return buf[:, :W]


def bernoulli(H: int, W: int, p: float, seed: int = 0, device="cpu", stride: int | None = None,
              rows_per_chunk: int | None = None) -> torch.Tensor:
    """H x W uint8 image, pixel = 1 with probability p (exact integer test)."""
    out = _alloc(H, W, stride, device)
    thr = int(math.floor(p * 2**32))
    if rows_per_chunk is None:
        rows_per_chunk = max(1, (1 << 25) // max(W, 1))
    col = torch.arange(W, dtype=torch.int64, device=device)
    for r0 in range(0, H, rows_per_chunk):
        r1 = min(H, r0 + rows_per_chunk)
        rows = torch.arange(r0, r1, dtype=torch.int64, device=device)
        idx = rows[:, None] * W + col[None, :]
        hi = _srl(splitmix64(idx, seed), 32)
        out[r0:r1] = (hi < thr).to(torch.uint8)
    return out


def _uniform01(H: int, W: int, seed: int, device) -> torch.Tensor:
    """Uniform (0, 1] doubles from the top 53 bits of SplitMix64."""
    idx = torch.arange(H * W, dtype=torch.int64, device=device).reshape(H, W)
    bits = _srl(splitmix64(idx, seed), 11)
    return (bits.to(torch.float64) + 1.0) * (1.0 / 9007199254740992.0)


def grf(H: int, W: int, sigma: float, q: float = 0.5, seed: int = 0, device="cpu",
        stride: int | None = None) -> torch.Tensor:
    """Thresholded periodic Gaussian random field (foreground fraction ~ 1-q).

    The smoothing of fields up to 2**24 pixels runs on the CPU: a GPU FFT
    compiles kernels for every new size, which would dominate the cost of
    building an uneven batch.  Larger fields are smoothed on `device`.
    (Float rounding may differ between the two, so the bytes of one spec can
    differ by device; consumers label the same bytes on both sides.)"""
    dst = device
    u1 = _uniform01(H, W, seed, device)
    u2 = _uniform01(H, W, seed ^ 0x5DEECE66D, device)
    noise = (torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * math.pi * u2)).to(torch.float32)
    del u1, u2
    if H * W <= (1 << 24):
        device = "cpu"
        noise = noise.to(device)
    fy = torch.fft.fftfreq(H, device=device, dtype=torch.float32)
    fx = torch.fft.rfftfreq(W, device=device, dtype=torch.float32)
    s2 = 2.0 * (math.pi * sigma) ** 2
    gain = torch.exp(-s2 * (fy[:, None] ** 2 + fx[None, :] ** 2))
    field = torch.fft.irfft2(torch.fft.rfft2(noise) * gain, s=(H, W))
    del noise, gain
    flat = field.reshape(-1)
    step = max(1, flat.numel() // (1 << 22))
    thr = torch.quantile(flat[::step].to(torch.float64), q).to(torch.float32)
    out = _alloc(H, W, stride, dst)
    out.copy_((field > thr).to(torch.uint8))
    return out


def gray(H: int, W: int, sigma: float = 4.0, seed: int = 0, device="cpu", stride: int | None = None) -> torch.Tensor:
    """Smooth grayscale bytes: 128 + 40 * (standardized Gaussian field)."""
    dst = device
    u1 = _uniform01(H, W, seed, device)
    u2 = _uniform01(H, W, seed ^ 0x5DEECE66D, device)
    noise = (torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * math.pi * u2)).to(torch.float32)
    del u1, u2
    if H * W <= (1 << 24):
        device = "cpu"
        noise = noise.to(device)
    fy = torch.fft.fftfreq(H, device=device, dtype=torch.float32)
    fx = torch.fft.rfftfreq(W, device=device, dtype=torch.float32)
    gain = torch.exp(-2.0 * (math.pi * sigma) ** 2 * (fy[:, None] ** 2 + fx[None, :] ** 2))
    field = torch.fft.irfft2(torch.fft.rfft2(noise) * gain, s=(H, W))
    z = (field - field.mean()) / field.std(correction=0).clamp_min(1e-12)
    out = _alloc(H, W, stride, dst)
    out.copy_(torch.clamp(torch.round(128.0 + 40.0 * z), 0, 255).to(torch.uint8))
    return out


ADVERSARIAL = ("spiral", "checkerboard", "ones", "zeros", "hstripes", "vstripes", "diagonal", "comb")


def adversarial(name: str, H: int, W: int, device="cpu", stride: int | None = None,
                k: int = 4) -> torch.Tensor:
    """Structured images (closed-form component counts, see the test-suite).

    spiral       concentric one-pixel rings at even ring depth d (ring depth of
                 (r, c) is min(r, c, H-1-r, W-1-c)); every ring of size at
                 least 3x3 is cut open at (d+1, d), and a connector pixel at
                 (d+1, d+2) joins ring d to ring d+2: one winding component.
    checkerboard (r + c) even
    ones, zeros  constant images
    hstripes     r even;  vstripes  c even
    diagonal     (r + c) % k == 0
    comb         teeth on even columns, joined by the full bottom row
    """
    r = torch.arange(H, device=device)[:, None]
    c = torch.arange(W, device=device)[None, :]
    if name == "checkerboard":
        img = ((r + c) % 2 == 0)
    elif name == "ones":
        img = torch.ones((H, W), dtype=torch.bool, device=device)
    elif name == "zeros":
        img = torch.zeros((H, W), dtype=torch.bool, device=device)
    elif name == "hstripes":
        img = (r % 2 == 0).expand(H, W)
    elif name == "vstripes":
        img = (c % 2 == 0).expand(H, W)
    elif name == "diagonal":
        img = ((r + c) % k == 0)
    elif name == "comb":
        img = (c % 2 == 0) | (r == H - 1)
    elif name == "spiral":
        depth = torch.minimum(torch.minimum(r, c), torch.minimum(H - 1 - r, W - 1 - c))
        img = (depth % 2 == 0).clone()
        dmax = (min(H, W) - 1) // 2
        d = torch.arange(0, dmax + 1, 2, device=device)
        # cut each ring that is at least 3 x 3 at (d+1, d)
        cut = d[(H - 1 - d >= d + 2) & (W - 1 - d >= d + 2)]
        img[cut + 1, cut] = False
        # connect ring d to ring d+2 through (d+1, d+2) when ring d+2 has a corner there
        con = d[(H - 1 - (d + 2) >= d + 2) & (W - 1 - (d + 2) >= d + 2)]
        img[con + 1, con + 2] = True
    else:
        raise ValueError(f"unknown adversarial pattern {name!r}")
    out = _alloc(H, W, stride, device)
    out.copy_(img.to(torch.uint8))
    return out


def batch_specs(n: int, seed: int = 0, min_side: int = 64, max_side: int = 4096):
    """Shapes and contents of an uneven batch: list of dicts (H, W, kind, param, seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for i in range(n):
        H = int(round(math.exp(rng.uniform(math.log(min_side), math.log(max_side)))))
        a = math.exp(rng.uniform(math.log(0.25), math.log(4.0)))
        W = int(min(max(round(H * a), min_side), max_side))
        if rng.uniform() < 0.5:
            specs.append(dict(H=H, W=W, kind="bernoulli", param=float(rng.uniform(0.2, 0.8)),
                              seed=seed * 100003 + i))
        else:
            specs.append(dict(H=H, W=W, kind="grf", param=float(rng.uniform(1.0, 16.0)),
                              seed=seed * 100003 + i))
    return specs


def serve_specs(n: int, rate: float, seed: int = 0, pool: int = 0, large_frac: float = 0.05,
                large_max: int = 8192):
    """A seeded request stream: list of dicts (t, img index or spec, conn).

    Arrival times t (seconds from 0) are a Poisson process of intensity
    ``rate``.  With ``pool`` > 0 the requests pick images from a pool of
    that many specs (returned separately) instead of carrying one each, so a
    long stream needs only a bounded set of device images.  Returns
    (requests, specs)."""
    rng = np.random.Generator(np.random.PCG64(seed ^ 0x5EED))
    m = pool if pool > 0 else n
    specs = batch_specs(m, seed=seed)
    for i in range(m):
        if rng.uniform() < large_frac:
            H = int(round(math.exp(rng.uniform(math.log(64), math.log(large_max)))))
            a = math.exp(rng.uniform(math.log(0.25), math.log(4.0)))
            specs[i] = dict(specs[i], H=H, W=int(min(max(round(H * a), 64), large_max)))
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    which = rng.integers(0, m, size=n) if pool > 0 else np.arange(n)
    conns = np.where(rng.uniform(size=n) < 0.5, 4, 8)
    reqs = [dict(t=float(t[i]), img=int(which[i]), conn=int(conns[i])) for i in range(n)]
    return reqs, specs


def make(spec: dict, device="cpu", stride: int | None = None) -> torch.Tensor:
    """Build the image a ``batch_specs`` entry describes."""
    if spec["kind"] == "bernoulli":
        return bernoulli(spec["H"], spec["W"], spec["param"], spec["seed"], device, stride)
    if spec["kind"] == "grf":
        return grf(spec["H"], spec["W"], spec["param"], 0.5, spec["seed"], device, stride)
    return adversarial(spec["kind"], spec["H"], spec["W"], device, stride)
