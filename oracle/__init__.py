"""CPU oracle for two-pass connected component labeling (arXiv 1606.05973).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1606_05973_amd``) and the library never falls
back to it.

The arithmetic lives in ``ccl_oracle.c`` (plain single-threaded C following
Algorithms 1-8 of the paper); this module only compiles it with gcc and
marshals numpy arrays through ctypes.

Functions
---------
cclremsp(img, conn)          -> (labels int32 HxW, K)   Algorithms 1-4
aremsp(img, conn, raw=False) -> (labels, K)             Algorithms 2, 3, 5, 6
paremsp(img, conn, nchunks)  -> (labels, K)             Algorithms 6, 7, 8 (chunks in turn)
paremsp_threads(img, conn, n)-> (labels, K)             the same, one thread per chunk
canonical(labels)            -> (labels, K)             rank by first raster index
merge_pairs(p, pairs)        -> p                       Algorithm 2 on a parent array
merger_pairs(p, pairs)       -> p                       Algorithm 8 (sequential schedule)
flatten(p, count)            -> (p, K)                  Algorithm 3
label(img, conn, level)      -> labels                  the reference labeling (CCLRemSP)
binarize(img, level)         -> uint8 0/1               Section V thresholding
gray(img, conn)              -> (labels, K)             gray-level extension (Section V):
                                                        equal nonzero neighbours connect
provisional(img, conn, tile_h, tile_w, block, gray)
                             -> (labels, K)             the flatten's numbering (Algorithm 3)
                                                        over tile-major provisional labels

All labelings returned by ``cclremsp``, ``aremsp`` and ``paremsp`` use the
canonical numbering: 0 is background and component k (1-based) is the k-th
component met in raster order, i.e. ranked by its smallest raster index.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ccl_oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile ccl_oracle.c into _liboracle.so with gcc (host code only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-pthread", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            u8p = ctypes.POINTER(ctypes.c_uint8)
            i32p = ctypes.POINTER(ctypes.c_int32)
            i64 = ctypes.c_int64
            lib.oracle_cclremsp.argtypes = [u8p, i64, i64, i64, ctypes.c_int, i32p]
            lib.oracle_cclremsp.restype = i64
            lib.oracle_aremsp.argtypes = [u8p, i64, i64, i64, ctypes.c_int, i32p, ctypes.c_int]
            lib.oracle_aremsp.restype = i64
            lib.oracle_paremsp.argtypes = [u8p, i64, i64, i64, ctypes.c_int, i32p, ctypes.c_int]
            lib.oracle_paremsp.restype = i64
            lib.oracle_paremsp_threads.argtypes = [u8p, i64, i64, i64, ctypes.c_int, i32p, ctypes.c_int]
            lib.oracle_paremsp_threads.restype = i64
            lib.oracle_gray.argtypes = [u8p, i64, i64, i64, ctypes.c_int, i32p]
            lib.oracle_gray.restype = i64
            lib.oracle_canonical.argtypes = [i32p, i64, i64]
            lib.oracle_canonical.restype = i64
            lib.oracle_merge_pairs.argtypes = [i32p, i32p, i64]
            lib.oracle_merge_pairs.restype = None
            lib.oracle_merger_pairs.argtypes = [i32p, i32p, i64]
            lib.oracle_merger_pairs.restype = None
            lib.oracle_flatten.argtypes = [i32p, ctypes.c_int32]
            lib.oracle_flatten.restype = ctypes.c_int32
            lib.oracle_provisional.argtypes = [i32p, i64, i64, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int]
            lib.oracle_provisional.restype = i64
            _lib = lib
    return _lib


def _img_args(img):
    img = np.asarray(img)
    if img.ndim != 2:
        raise ValueError("image must be 2-D")
    if img.dtype != np.uint8:
        img = (img != 0).astype(np.uint8)
    if img.strides[1] != 1 or img.strides[0] < img.shape[1]:
        img = np.ascontiguousarray(img)
    H, W = img.shape
    stride = img.strides[0]
    ptr = img.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    return img, ptr, H, W, stride


def _i32ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _check(k):
    if k < 0:
        raise ValueError("oracle rejected its arguments (or ran out of memory)")
    return int(k)


def cclremsp(img, conn: int = 8):
    """CCLRemSP (Algorithm 1): decision-tree scan + RemSP, flatten, labeling."""
    lib = _load()
    img, ptr, H, W, stride = _img_args(img)
    out = np.empty((H, W), dtype=np.int32)
    k = lib.oracle_cclremsp(ptr, H, W, stride, conn, _i32ptr(out))
    return out, _check(k)


def aremsp(img, conn: int = 8, raw: bool = False):
    """ARemSP (Algorithm 5); canonical numbering unless raw=True."""
    lib = _load()
    img, ptr, H, W, stride = _img_args(img)
    out = np.empty((H, W), dtype=np.int32)
    k = lib.oracle_aremsp(ptr, H, W, stride, conn, _i32ptr(out), int(raw))
    return out, _check(k)


def paremsp(img, conn: int = 8, nchunks: int = 4):
    """PARemSP (Algorithm 7) with nchunks row chunks, canonical numbering."""
    lib = _load()
    img, ptr, H, W, stride = _img_args(img)
    out = np.empty((H, W), dtype=np.int32)
    k = lib.oracle_paremsp(ptr, H, W, stride, conn, _i32ptr(out), int(nchunks))
    return out, _check(k)


def paremsp_threads(img, conn: int = 8, nthreads: int = 4):
    """PARemSP (Algorithm 7) with one POSIX thread per row chunk: the chunk
    scans run at once, then the boundary unions run concurrently with
    Algorithm 8's locked root links; canonical numbering."""
    lib = _load()
    img, ptr, H, W, stride = _img_args(img)
    out = np.empty((H, W), dtype=np.int32)
    k = lib.oracle_paremsp_threads(ptr, H, W, stride, conn, _i32ptr(out), int(nthreads))
    return out, _check(k)


def canonical(labels):
    """Renumber an arbitrary labeling canonically (first raster occurrence)."""
    lib = _load()
    out = np.ascontiguousarray(labels, dtype=np.int32).copy()
    H, W = out.shape
    k = lib.oracle_canonical(_i32ptr(out), H, W)
    return out, _check(k)


def merge_pairs(p, pairs):
    """Apply Algorithm 2 to the parent array p for each (x, y) in pairs."""
    lib = _load()
    p = np.ascontiguousarray(p, dtype=np.int32).copy()
    pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    lib.oracle_merge_pairs(_i32ptr(p), _i32ptr(pr), pr.shape[0])
    return p


def merger_pairs(p, pairs):
    """Apply Algorithm 8 (run sequentially) for each (x, y) in pairs."""
    lib = _load()
    p = np.ascontiguousarray(p, dtype=np.int32).copy()
    pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    lib.oracle_merger_pairs(_i32ptr(p), _i32ptr(pr), pr.shape[0])
    return p


def flatten(p, count: int):
    """Algorithm 3 on a copy of p; returns (flattened p, number of roots)."""
    lib = _load()
    p = np.ascontiguousarray(p, dtype=np.int32).copy()
    k = lib.oracle_flatten(_i32ptr(p), int(count))
    return p, int(k)


def gray(img, conn: int = 8):
    """Gray-level labeling (the extension Section V mentions): object pixels
    are nonzero bytes, neighbouring object pixels connect when their bytes
    are equal; canonical numbering."""
    lib = _load()
    img = np.asarray(img)
    if img.dtype != np.uint8:
        raise ValueError("gray labeling takes uint8 images")
    img, ptr, H, W, stride = _img_args(img)
    out = np.empty((H, W), dtype=np.int32)
    k = lib.oracle_gray(ptr, H, W, stride, conn, _i32ptr(out))
    return out, _check(k)


def binarize(img, level: int):
    """Section V: every test image is turned into a binary image by a
    luminance threshold before labeling.  On bytes: foreground (1) iff the
    byte is greater than ``level``."""
    return (np.asarray(img).astype(np.int32) > int(level)).astype(np.uint8)


def label(img, conn: int = 8, level: int | None = None):
    """The reference labeling used for parity: CCLRemSP output (of the
    binarized image when ``level`` is given)."""
    if level is not None:
        img = binarize(img, level)
    return cclremsp(img, conn)[0]


def provisional(img, conn: int, tile_h: int, tile_w: int, block: int = 1, gray_levels: bool = False):
    """Labels numbered in provisional order, the numbering of the flatten
    (Algorithm 3, Section III): label k goes to the set whose smallest
    provisional label is the k-th smallest among the sets' smallest labels.

    The provisional labels are those of a tiled two-pass scan: the image is
    cut into tile_h x tile_w tiles, taken in raster order, each handing out
    its labels after those of the tiles before it (the disjoint per-thread
    label ranges of Algorithm 7, Section IV, with tiles for row chunks).
    Inside a tile the labels follow the scan's nodes: runs of `block` image
    rows (2: the two-row mask of Fig. 1b; 1: single rows; single rows of
    equal bytes with ``gray_levels``), ordered by (block row, first column);
    a tile-local component is labeled by its first node.  So the smallest
    provisional label of a set is the minimum over its pixels of
    (tile index, block row inside the tile, column inside the tile), which
    is what is ranked here; the partition itself is the oracle's
    (``cclremsp`` or ``gray``)."""
    glab, K = (gray if gray_levels else cclremsp)(img, conn)
    H, W = glab.shape
    k = _load().oracle_provisional(_i32ptr(glab), H, W, K, int(tile_h), int(tile_w), int(block))
    return glab, _check(k)
