"""Independent references used to pin the oracle (no code shared with it).

* ``min_propagation`` -- vectorised fixed-point iteration: every foreground
  pixel repeatedly takes the smallest raster index found among itself and its
  foreground neighbours.  At the fixed point each pixel holds the smallest
  raster index of its component; ranking those minima gives the canonical
  labels.  Works on a stack of images at once.
* ``bfs_labels`` -- textbook breadth-first flood fill started at every
  unvisited foreground pixel in raster order (canonical by construction).
* ``read_golden`` -- parser for the hand-derived fixtures in tests/golden.
"""
from collections import deque

import numpy as np

OFFS8 = [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 1), (1, -1), (1, 0), (1, 1)]
OFFS4 = [(-1, 0), (0, -1), (0, 1), (1, 0)]


def min_propagation(imgs, conn):
    """imgs: (N, H, W) array-like of 0/1 -> (N, H, W) int32 canonical labels."""
    imgs = np.asarray(imgs) != 0
    N, H, W = imgs.shape
    BIG = np.int64(H * W + 1)
    idx = np.arange(H * W, dtype=np.int64).reshape(1, H, W)
    lab = np.where(imgs, idx, BIG)
    offs = OFFS8 if conn == 8 else OFFS4
    while True:
        pad = np.full((N, H + 2, W + 2), BIG, dtype=np.int64)
        pad[:, 1:-1, 1:-1] = lab
        new = lab.copy()
        for dr, dc in offs:
            new = np.minimum(new, pad[:, 1 + dr:1 + dr + H, 1 + dc:1 + dc + W])
        new = np.where(imgs, new, BIG)
        if np.array_equal(new, lab):
            break
        lab = new
    flat = lab.reshape(N, H * W)
    isroot = (flat == np.arange(H * W)[None, :])
    rank = np.cumsum(isroot, axis=1)  # rank[i] = 1-based rank of root i
    safe = np.where(flat == BIG, 0, flat)
    out = np.take_along_axis(rank, safe, axis=1)
    out = np.where(flat == BIG, 0, out)
    return out.reshape(N, H, W).astype(np.int32)


def bfs_labels(img, conn):
    img = np.asarray(img) != 0
    H, W = img.shape
    out = np.zeros((H, W), dtype=np.int32)
    offs = OFFS8 if conn == 8 else OFFS4
    k = 0
    for r in range(H):
        for c in range(W):
            if img[r, c] and out[r, c] == 0:
                k += 1
                out[r, c] = k
                q = deque([(r, c)])
                while q:
                    y, x = q.popleft()
                    for dy, dx in offs:
                        yy, xx = y + dy, x + dx
                        if 0 <= yy < H and 0 <= xx < W and img[yy, xx] and out[yy, xx] == 0:
                            out[yy, xx] = k
                            q.append((yy, xx))
    return out


def all_images(H, W):
    """Every H x W binary image (H*W <= 16) as an (2**(H*W), H, W) uint8 stack."""
    n = H * W
    codes = np.arange(1 << n, dtype=np.int64)
    bits = (codes[:, None] >> np.arange(n)[None, :]) & 1
    return bits.reshape(-1, H, W).astype(np.uint8)


def read_golden(path):
    """Returns (image uint8, {conn: (labels int32, K)})."""
    lines = [l.strip() for l in open(path) if l.strip() and not l.lstrip().startswith("#")]
    sections, cur = {}, None
    for l in lines:
        head = l.split()
        if head[0] in ("image", "labels8", "labels4"):
            cur = head[0]
            sections[cur] = {"K": int(head[1]) if len(head) > 1 else None, "rows": []}
        else:
            sections[cur]["rows"].append([int(v) for v in head])
    img = np.array(sections["image"]["rows"], dtype=np.uint8)
    out = {}
    for conn in (8, 4):
        s = sections.get(f"labels{conn}")
        if s:
            out[conn] = (np.array(s["rows"], dtype=np.int32), s["K"])
    return img, out


def bfs_gray_labels(img, conn):
    """Textbook flood fill for the gray-level extension: object pixels are
    nonzero, neighbours connect when their values are equal; components
    numbered by first pixel in raster order."""
    img = np.asarray(img)
    H, W = img.shape
    out = np.zeros((H, W), dtype=np.int32)
    offs = OFFS8 if conn == 8 else OFFS4
    k = 0
    for r in range(H):
        for c in range(W):
            v = img[r, c]
            if v and out[r, c] == 0:
                k += 1
                out[r, c] = k
                q = deque([(r, c)])
                while q:
                    y, x = q.popleft()
                    for dy, dx in offs:
                        yy, xx = y + dy, x + dx
                        if 0 <= yy < H and 0 <= xx < W and img[yy, xx] == v and out[yy, xx] == 0:
                            out[yy, xx] = k
                            q.append((yy, xx))
    return out


def all_gray_images(H, W, levels):
    """Every H x W image with pixel values in range(levels)."""
    n = H * W
    codes = np.arange(levels ** n, dtype=np.int64)
    digits = (codes[:, None] // (levels ** np.arange(n))[None, :]) % levels
    return digits.reshape(-1, H, W).astype(np.uint8)
