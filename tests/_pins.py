"""Independent references used to pin the oracle (no code shared with it).

* ``min_propagation`` -- vectorised fixed-point iteration: every foreground
  pixel repeatedly takes the smallest raster index found among itself and its
  foreground neighbours.  At the fixed point each pixel holds the smallest
  raster index of its component; ranking those minima gives the canonical
  labels.  Works on a stack of images at once.
* ``bfs_labels`` -- textbook breadth-first flood fill started at every
  unvisited foreground pixel in raster order (canonical by construction).
* ``read_golden`` -- parser for the hand-derived fixtures in tests/golden.
* ``provisional_by_steps`` -- the provisional (flatten) numbering computed the
  way the paper's steps produce it: per-tile components, disjoint label
  ranges per tile, unions across tile edges, then Algorithm 3's consecutive
  numbering in label order.
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


def provisional_by_steps(img, conn, th, tw, block=1, gray=False):
    """Tile-major two-pass labeling, step by step, on a small image.

    1. Tiles in raster order; inside a tile, nodes are the runs of `block`
       rows (gray: runs of equal values in one row) in (block row, start)
       order; the tile's components (flood fill inside the tile) take labels
       in the order of their first node, after the labels of earlier tiles.
    2. Every pair of neighbouring object pixels in different tiles unites
       their labels (a plain union-find whose root is the smaller label).
    3. Flatten: walking labels in increasing order, a root takes the next
       consecutive number and every other label its root's number."""
    img = np.asarray(img)
    H, W = img.shape
    fg = (img != 0)
    same = (lambda a, b: img[a] == img[b]) if gray else (lambda a, b: True)
    offs = OFFS8 if conn == 8 else OFFS4
    prov = np.zeros((H, W), dtype=np.int64)
    nxt = 1
    for ty in range(0, H, th):
        for tx in range(0, W, tw):
            y1, x1 = min(H, ty + th), min(W, tx + tw)
            # node of each pixel: (block row, start column of its run)
            node = {}
            for y in range(ty, y1):
                br = (y - ty) // block
                for x in range(tx, x1):
                    if not fg[y, x]:
                        continue
                    rows = range(ty + br * block, min(y1, ty + br * block + block))
                    s = x
                    while s - 1 >= tx and (any(fg[yy, s - 1] for yy in rows) if not gray
                                           else (fg[y, s - 1] and img[y, s - 1] == img[y, x])):
                        s -= 1
                    node[(y, x)] = (br, s - tx)
            comp = {}
            comps = []
            for y in range(ty, y1):
                for x in range(tx, x1):
                    if fg[y, x] and (y, x) not in comp:
                        k = len(comps)
                        members = [(y, x)]
                        comp[(y, x)] = k
                        q = deque([(y, x)])
                        while q:
                            a = q.popleft()
                            for dy, dx in offs:
                                b = (a[0] + dy, a[1] + dx)
                                if ty <= b[0] < y1 and tx <= b[1] < x1 and fg[b] and b not in comp and same(a, b):
                                    comp[b] = k
                                    members.append(b)
                                    q.append(b)
                        comps.append(members)
            order = sorted(range(len(comps)), key=lambda k: min(node[p] for p in comps[k]))
            for rank, k in enumerate(order):
                for p in comps[k]:
                    prov[p] = nxt + rank
            nxt += len(comps)
    parent = list(range(nxt))

    def root(a):
        while parent[a] != a:
            a = parent[a]
        return a
    for y in range(H):
        for x in range(W):
            if not fg[y, x]:
                continue
            for dy, dx in offs:
                yy, xx = y + dy, x + dx
                if 0 <= yy < H and 0 <= xx < W and fg[yy, xx] and same((y, x), (yy, xx)) \
                        and (yy // th, xx // tw) != (y // th, x // tw):
                    a, b = root(prov[y, x]), root(prov[yy, xx])
                    if a != b:
                        parent[max(a, b)] = min(a, b)
    number = [0] * nxt
    k = 0
    for i in range(1, nxt):
        if root(i) == i:
            k += 1
            number[i] = k
        else:
            number[i] = number[root(i)]
    out = np.zeros((H, W), dtype=np.int32)
    for y in range(H):
        for x in range(W):
            if fg[y, x]:
                out[y, x] = number[prov[y, x]]
    return out, k
