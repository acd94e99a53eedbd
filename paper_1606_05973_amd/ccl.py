"""Python binding of libccl.so (include/ccl.h): argument marshalling only.

Every step of the labeling runs in the library's HIP kernels.  If the
library is not built this module raises on import: there is no fallback.
torch is used for device memory and streams.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

from .build import LIB

if not os.path.exists(LIB):
    raise ImportError(f"{LIB} is missing: build it with `python -m paper_1606_05973_amd.build` "
                      "(or __graft_entry__.build())")

_lib = ctypes.CDLL(LIB)

_u8p = ctypes.c_void_p
_i32p = ctypes.c_void_p
_i64 = ctypes.c_int64
_stream = ctypes.c_void_p


class ImageDesc(ctypes.Structure):
    """ccl_image_desc of include/ccl.h (the plain batch call)."""
    _fields_ = [("img", ctypes.c_void_p), ("H", _i64), ("W", _i64), ("stride", _i64),
                ("conn", ctypes.c_int), ("labels", ctypes.c_void_p), ("num_components", ctypes.c_void_p)]


class ImageDescEx(ctypes.Structure):
    """ccl_image_desc_ex of include/ccl.h (the extended calls)."""
    _fields_ = [("img", ctypes.c_void_p), ("H", _i64), ("W", _i64), ("stride", _i64),
                ("conn", ctypes.c_int), ("labels", ctypes.c_void_p), ("num_components", ctypes.c_void_p),
                ("level", ctypes.c_int), ("scan", ctypes.c_int), ("gray", ctypes.c_int),
                ("order", ctypes.c_int), ("tile", ctypes.c_int)]


_lib.ccl_label.argtypes = [_u8p, _i64, _i64, _i64, ctypes.c_int, _i32p, _stream]
_lib.ccl_label.restype = ctypes.c_int
_lib.ccl_label_ex.argtypes = [_u8p, _i64, _i64, _i64, ctypes.c_int, _i32p, _i32p, ctypes.c_int, _stream]
_lib.ccl_label_ex.restype = ctypes.c_int
_lib.ccl_label_level.argtypes = [_u8p, _i64, _i64, _i64, ctypes.c_int, ctypes.c_int, _i32p, _i32p, ctypes.c_int,
                                 _stream]
_lib.ccl_label_level.restype = ctypes.c_int
_lib.ccl_label_gray.argtypes = [_u8p, _i64, _i64, _i64, ctypes.c_int, ctypes.c_int, _i32p, _i32p, ctypes.c_int,
                                _stream]
_lib.ccl_label_gray.restype = ctypes.c_int
_lib.ccl_label_provisional.argtypes = [_u8p, _i64, _i64, _i64, ctypes.c_int, _i32p, _i32p, ctypes.c_int, _stream]
_lib.ccl_label_provisional.restype = ctypes.c_int
_lib.ccl_label_noalloc.argtypes = [_u8p, _i64, _i64, _i64, ctypes.c_int, _i32p, _i32p, _stream]
_lib.ccl_label_noalloc.restype = ctypes.c_int
_lib.ccl_label_batch.argtypes = [ctypes.POINTER(ImageDesc), ctypes.c_int, _stream]
_lib.ccl_label_batch.restype = ctypes.c_int
_lib.ccl_label_batch_ex.argtypes = [ctypes.POINTER(ImageDescEx), ctypes.c_int, ctypes.c_int, _stream]
_lib.ccl_label_batch_ex.restype = ctypes.c_int
_lib.ccl_workspace_bytes.argtypes = [_i64, _i64, ctypes.c_int]
_lib.ccl_workspace_bytes.restype = ctypes.c_size_t
_lib.ccl_batch_workspace_bytes.argtypes = [ctypes.POINTER(ImageDescEx), ctypes.c_int, ctypes.c_int]
_lib.ccl_batch_workspace_bytes.restype = ctypes.c_size_t
_lib.ccl_reserve.argtypes = [ctypes.c_size_t, _stream]
_lib.ccl_reserve.restype = ctypes.c_int
_lib.ccl_release.argtypes = []
_lib.ccl_release.restype = ctypes.c_int
_lib.ccl_tile_config.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
_lib.ccl_tile_config.restype = ctypes.c_int
_lib.ccl_tile_count.argtypes = []
_lib.ccl_tile_count.restype = ctypes.c_int
_lib.ccl_tile_default.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
_lib.ccl_tile_default.restype = ctypes.c_int
_lib.ccl_batch_graph_create.argtypes = [ctypes.POINTER(ImageDescEx), ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_void_p)]
_lib.ccl_batch_graph_create.restype = ctypes.c_int
_lib.ccl_graph_launch.argtypes = [ctypes.c_void_p, _stream]
_lib.ccl_graph_launch.restype = ctypes.c_int
_lib.ccl_graph_destroy.argtypes = [ctypes.c_void_p]
_lib.ccl_graph_destroy.restype = ctypes.c_int
_lib.ccl_profile.argtypes = [ctypes.c_int]
_lib.ccl_profile.restype = ctypes.c_int
_lib.ccl_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
_lib.ccl_profile_read.restype = ctypes.c_int
class ServerConfig(ctypes.Structure):
    """ccl_server_config of include/ccl.h."""
    _fields_ = [("n_streams", ctypes.c_int), ("max_batch", ctypes.c_int), ("max_batch_pixels", _i64),
                ("hbm_budget", ctypes.c_size_t), ("tile", ctypes.c_int)]


class ServerStats(ctypes.Structure):
    """ccl_server_stats of include/ccl.h."""
    _fields_ = [("submitted", _i64), ("completed", _i64), ("rejected", _i64), ("batches", _i64),
                ("in_flight_max", _i64), ("pixels_completed", ctypes.c_double), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double)]


_lib.ccl_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(ctypes.c_void_p)]
_lib.ccl_server_create.restype = ctypes.c_int
_lib.ccl_server_submit.argtypes = [ctypes.c_void_p, ctypes.POINTER(ImageDescEx), _stream,
                                   ctypes.POINTER(ctypes.c_uint64)]
_lib.ccl_server_submit.restype = ctypes.c_int
_lib.ccl_server_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
_lib.ccl_server_poll.restype = ctypes.c_int
_lib.ccl_server_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
_lib.ccl_server_wait.restype = ctypes.c_int
_lib.ccl_server_drain.argtypes = [ctypes.c_void_p]
_lib.ccl_server_drain.restype = ctypes.c_int
_lib.ccl_server_stats_get.argtypes = [ctypes.c_void_p, ctypes.POINTER(ServerStats)]
_lib.ccl_server_stats_get.restype = ctypes.c_int
_lib.ccl_server_destroy.argtypes = [ctypes.c_void_p]
_lib.ccl_server_destroy.restype = ctypes.c_int
_lib.ccl_strerror.argtypes = [ctypes.c_int]
_lib.ccl_strerror.restype = ctypes.c_char_p

CCL_OK = 0
STATUS = {
    "CCL_ERR_NULL": -1, "CCL_ERR_SHAPE": -2, "CCL_ERR_STRIDE": -3, "CCL_ERR_CONN": -4,
    "CCL_ERR_TOO_LARGE": -5, "CCL_ERR_NOMEM": -6, "CCL_ERR_HIP": -7, "CCL_ERR_TILE": -8,
    "CCL_ERR_CAPTURE": -9, "CCL_ERR_BATCH": -10, "CCL_ERR_LEVEL": -11, "CCL_ERR_SCAN": -12,
    "CCL_ERR_BUDGET": -13, "CCL_ERR_TICKET": -14, "CCL_ERR_GRAY": -15, "CCL_ERR_ORDER": -16,
    "CCL_ERR_SCRATCH": -17,
}
NOALLOC_SCRATCH_BYTES = 96 << 20   # CCL_NOALLOC_SCRATCH_BYTES: static workspace of ccl_label_noalloc
SCAN_PAIR, SCAN_ROW = 0, 1   # ccl_scan: two-row (default) / one-row tile-local scan
CANONICAL, PROVISIONAL = 0, 1   # ccl_order: smallest raster index (default) / the flatten's provisional order


class CCLError(RuntimeError):
    def __init__(self, status: int):
        self.status = status
        super().__init__(f"ccl status {status}: {strerror(status)}")


def strerror(status: int) -> str:
    return _lib.ccl_strerror(int(status)).decode()


def _check(status: int):
    if status != CCL_OK:
        raise CCLError(status)


def _stream_handle(stream) -> int | None:
    """torch stream, raw hipStream_t as int (0 = default stream), or None for
    torch's current stream."""
    if isinstance(stream, int):
        return stream or None
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


def _img_geometry(img: torch.Tensor):
    if img.dim() != 2 or img.dtype != torch.uint8:
        raise ValueError("image must be a 2-D uint8 tensor")
    if not img.is_cuda:
        raise ValueError("image must be on the GPU")
    if img.stride(1) != 1:
        raise ValueError("image rows must be contiguous (stride(1) == 1)")
    H, W = img.shape
    stride = img.stride(0) if H > 1 else W
    return H, W, max(stride, W)


def tile_configs():
    """[(block_rows, tile_w)] for ids 1..n; id 0 means each kind's default
    (tile_default).  Tile height is block_rows * 2 under 8-connectivity,
    block_rows under 4."""
    out = []
    for i in range(1, _lib.ccl_tile_count() + 1):
        h, w = ctypes.c_int(), ctypes.c_int()
        _check(_lib.ccl_tile_config(i, ctypes.byref(h), ctypes.byref(w)))
        out.append((h.value, w.value))
    return out


def level_of(fraction: float) -> int:
    """Byte level of a fractional threshold of the full range: v > fraction*255
    iff v > level_of(fraction) for every byte v (0.5 -> 127)."""
    import math
    return min(255, max(0, int(math.floor(fraction * 255))))


def _check_out(out: torch.Tensor, img: torch.Tensor):
    """The label buffer the library writes H*W int32 into."""
    if not isinstance(out, torch.Tensor) or tuple(out.shape) != tuple(img.shape) or out.dtype != torch.int32 \
            or not out.is_contiguous() or out.device != img.device:
        raise ValueError("out must be a contiguous int32 tensor of the image's shape on the image's device")


def _check_counts(num_components, n: int, device) -> None:
    """The K output: a contiguous device int32 tensor with at least n slots."""
    if num_components is None:
        return
    if not isinstance(num_components, torch.Tensor) or num_components.dtype != torch.int32 \
            or not num_components.is_contiguous() or num_components.numel() < n \
            or num_components.device != torch.device(device):
        raise ValueError(f"num_components must be a contiguous int32 tensor with at least {n} slots "
                         "on the images' device")


def label(img: torch.Tensor, conn: int = 8, out: torch.Tensor | None = None, tile: int = 0,
          num_components: torch.Tensor | None = None, stream=None, level: int = 0,
          scan: int = SCAN_PAIR) -> torch.Tensor:
    """Canonical int32 labels of a 2-D uint8 device image; foreground iff the
    byte exceeds `level` (0 = nonzero).  `scan` picks the tile-local scan
    strategy (SCAN_PAIR or SCAN_ROW); the labels do not depend on it."""
    H, W, stride = _img_geometry(img)
    if out is None:
        out = torch.empty((H, W), dtype=torch.int32, device=img.device)
    _check_out(out, img)
    _check_counts(num_components, 1, img.device)
    if scan != SCAN_PAIR:
        return label_batch([img], conn, outs=[out], tile=tile, num_components=num_components, stream=stream,
                           level=level, scan=scan)[0]
    nc = num_components.data_ptr() if num_components is not None else None
    st = _lib.ccl_label_level(img.data_ptr(), H, W, stride, int(level), int(conn), out.data_ptr(), nc,
                              int(tile), _stream_handle(stream))
    _check(st)
    return out


def label_provisional(img: torch.Tensor, conn: int = 8, out: torch.Tensor | None = None, tile: int = 0,
                      num_components: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Labels numbered 1..K in provisional order (ccl_label_provisional): the
    same components as label(), numbered as the paper's flatten numbers them
    (by each set's smallest provisional label: tile, then component)."""
    H, W, stride = _img_geometry(img)
    if out is None:
        out = torch.empty((H, W), dtype=torch.int32, device=img.device)
    _check_out(out, img)
    _check_counts(num_components, 1, img.device)
    nc = num_components.data_ptr() if num_components is not None else None
    _check(_lib.ccl_label_provisional(img.data_ptr(), H, W, stride, int(conn), out.data_ptr(), nc, int(tile),
                                      _stream_handle(stream)))
    return out


def label_gray(img: torch.Tensor, conn: int = 8, out: torch.Tensor | None = None, tile: int = 0,
               num_components: torch.Tensor | None = None, stream=None, level: int = 0) -> torch.Tensor:
    """Gray-level labeling: object pixels are bytes > `level`; neighbouring
    object pixels connect when their bytes are equal."""
    H, W, stride = _img_geometry(img)
    if out is None:
        out = torch.empty((H, W), dtype=torch.int32, device=img.device)
    _check_out(out, img)
    _check_counts(num_components, 1, img.device)
    nc = num_components.data_ptr() if num_components is not None else None
    _check(_lib.ccl_label_gray(img.data_ptr(), H, W, stride, int(level), int(conn), out.data_ptr(), nc,
                               int(tile), _stream_handle(stream)))
    return out


def label_noalloc(img: torch.Tensor, conn: int, out: torch.Tensor, num_components: torch.Tensor | None = None,
                  stream=None) -> torch.Tensor:
    """ccl_label_noalloc: label() with the library's static scratch as its
    workspace; allocates nothing, so `out` must be given.  Images that need
    more than NOALLOC_SCRATCH_BYTES of workspace raise CCLError
    (CCL_ERR_SCRATCH)."""
    H, W, stride = _img_geometry(img)
    _check_out(out, img)
    _check_counts(num_components, 1, img.device)
    nc = num_components.data_ptr() if num_components is not None else None
    _check(_lib.ccl_label_noalloc(img.data_ptr(), H, W, stride, int(conn), out.data_ptr(), nc,
                                  _stream_handle(stream)))
    return out


def label_raw(img_ptr: int, H: int, W: int, stride: int, conn: int, labels_ptr: int, stream=None) -> int:
    """Direct ccl_label call with raw device pointers; returns the status."""
    return _lib.ccl_label(img_ptr or None, H, W, stride, conn, labels_ptr or None, _stream_handle(stream))


_DESC_FIELDS = ("img", "H", "W", "stride", "conn", "labels", "num_components", "level", "scan", "gray", "order",
                "tile")
# numpy view of ccl_image_desc_ex (same offsets and size as the ctypes
# structure): a batch's descriptors are written column by column
_DESC_DTYPE = np.dtype({
    "names": list(_DESC_FIELDS),
    "formats": [np.uint64, np.int64, np.int64, np.int64, np.int32, np.uint64, np.uint64, np.int32, np.int32,
                np.int32, np.int32, np.int32],
    "offsets": [getattr(ImageDescEx, f).offset for f in _DESC_FIELDS],
    "itemsize": ctypes.sizeof(ImageDescEx)})


class _DescArray:
    """A batch's ccl_image_desc_ex array (numpy-backed); .ptr is what the
    library calls take, valid while this object lives."""

    def __init__(self, rows: np.ndarray):
        self.rows = rows
        self.ptr = rows.ctypes.data_as(ctypes.POINTER(ImageDescEx))

    def __len__(self):
        return len(self.rows)


def _descs(imgs, conns, outs, num_components, levels=None, scans=None, grays=None, orders=None, tiles=None):
    """Extended descriptors of a batch, after checking every buffer the
    library will write: outs[i] for image i, slot i of num_components.
    (One pass with few tensor attribute reads per image, then the fields
    written column by column; anything unusual goes through the full checks,
    which raise the detailed errors.)"""
    n = len(imgs)
    if len(outs) != n:
        raise ValueError("one label buffer per image")
    rows = np.zeros(max(n, 1), dtype=_DESC_DTYPE)
    if not n:
        return _DescArray(rows)
    _check_counts(num_components, n, imgs[0].device)
    dev = imgs[0].get_device()
    u8, i32 = torch.uint8, torch.int32
    ptr, hs, ws, strides, lab = [0] * n, [0] * n, [0] * n, [0] * n, [0] * n
    for i in range(n):
        img, out = imgs[i], outs[i]
        shp = img.shape
        st = img.stride() if len(shp) == 2 else None
        if (st is None or img.dtype is not u8 or st[1] != 1 or img.get_device() != dev or dev < 0
                or not isinstance(out, torch.Tensor) or out.shape != shp or out.dtype is not i32
                or not out.is_contiguous() or out.get_device() != dev):
            # the full checks name what is wrong (and accept what they accept)
            _img_geometry(img)
            _check_out(out, img)
            if img.get_device() != dev:
                raise ValueError("all images of a batch must be on one device")
        H, W = shp
        stride = st[0] if H > 1 else W
        ptr[i], hs[i], ws[i], strides[i], lab[i] = img.data_ptr(), H, W, max(stride, W), out.data_ptr()
    rows = rows[:n]
    rows["img"], rows["H"], rows["W"], rows["stride"], rows["labels"] = ptr, hs, ws, strides, lab
    rows["conn"] = [int(c) for c in conns]
    if num_components is not None:
        rows["num_components"] = num_components.data_ptr() + 4 * np.arange(n, dtype=np.uint64)
    for name, vals in (("level", levels), ("scan", scans), ("order", orders), ("tile", tiles)):
        if vals is not None:
            rows[name] = [int(v) for v in vals]
    if grays is not None:
        rows["gray"] = [int(bool(v)) for v in grays]
    return _DescArray(rows)


def _per_image(v, n):
    out = list(v) if isinstance(v, (list, tuple)) else [v] * n
    if len(out) != n:
        raise ValueError("a per-image option list must have one entry per image")
    return out


def label_batch(imgs, conn=8, outs=None, tile: int = 0, num_components: torch.Tensor | None = None,
                stream=None, level=0, scan=SCAN_PAIR, gray=False, order=CANONICAL, tiles=0):
    """Label a list of images with one launch per phase and launch group
    (ccl_label_batch_ex).

    conn, level, scan, gray, order: one value or a per-image list.  tiles:
    per-image tile ids (0 = `tile`, whose 0 means each kind's default).
    num_components: optional contiguous device int32 tensor with one slot per
    image."""
    n = len(imgs)
    conns, levels = _per_image(conn, n), _per_image(level, n)
    scans, grays = _per_image(scan, n), _per_image(gray, n)
    orders, tl = _per_image(order, n), _per_image(tiles, n)
    if outs is None:
        outs = [torch.empty(tuple(im.shape), dtype=torch.int32, device=im.device) for im in imgs]
    arr = _descs(imgs, conns, outs, num_components, levels, scans, grays, orders, tl)
    _check(_lib.ccl_label_batch_ex(arr.ptr, n, int(tile), _stream_handle(stream)))
    return outs


def tile_default(conn: int, scan: int = SCAN_PAIR, gray: bool = False) -> int:
    """Configuration id that tile 0 selects for this kind of image."""
    t = _lib.ccl_tile_default(int(conn), int(scan), int(bool(gray)))
    if t <= 0:
        raise ValueError("invalid conn / scan / gray")
    return t


def tile_shape(tile: int, conn: int, scan: int = SCAN_PAIR, gray: bool = False):
    """(tile height, tile width) in pixels of configuration `tile` for `conn`
    (gray-level tiles have half the block rows, one image row each)."""
    nsr, tw = tile_configs()[(tile if tile > 0 else tile_default(conn, scan, gray)) - 1]
    if gray:
        return nsr // 2, tw
    return nsr * (2 if conn == 8 and scan == SCAN_PAIR else 1), tw


class BatchGraph:
    """A batch captured once into a HIP graph (ccl_batch_graph_create) and
    replayed with one launch.  The image and label tensors are kept alive and
    reused on every replay."""

    def __init__(self, imgs, conn=8, outs=None, tile: int = 0, num_components: torch.Tensor | None = None,
                 level=0, scan=SCAN_PAIR, gray=False, order=CANONICAL, tiles=0):
        n = len(imgs)
        conns, levels, scans = _per_image(conn, n), _per_image(level, n), _per_image(scan, n)
        grays, orders, tl = _per_image(gray, n), _per_image(order, n), _per_image(tiles, n)
        if outs is None:
            outs = [torch.empty(tuple(im.shape), dtype=torch.int32, device=im.device) for im in imgs]
        self.imgs, self.outs, self.counts = list(imgs), outs, num_components
        arr = _descs(imgs, conns, outs, num_components, levels, scans, grays, orders, tl)
        h = ctypes.c_void_p()
        _check(_lib.ccl_batch_graph_create(arr.ptr, n, int(tile), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(_lib.ccl_graph_launch(self._h, _stream_handle(stream)))
        return self.outs

    def close(self):
        if self._h:
            _check(_lib.ccl_graph_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_bytes(H: int, W: int, conn: int = 8, tile: int = 0, scan: int = SCAN_PAIR) -> int:
    """Workspace bytes of one labeling call (ccl_workspace_bytes for the
    defaults, else the extended batch form)."""
    if scan != SCAN_PAIR or tile != 0:
        return batch_workspace_bytes([(H, W)], conn, tile, scan)
    return int(_lib.ccl_workspace_bytes(H, W, conn))


def batch_workspace_bytes(shapes, conn=8, tile: int = 0, scan=SCAN_PAIR, gray=False, order=CANONICAL,
                          tiles=0) -> int:
    n = len(shapes)
    conns, scans, grays = _per_image(conn, n), _per_image(scan, n), _per_image(gray, n)
    orders, tl = _per_image(order, n), _per_image(tiles, n)
    arr = (ImageDescEx * max(n, 1))()
    for i, (H, W) in enumerate(shapes):
        arr[i].img = 1
        arr[i].labels = 1
        arr[i].H, arr[i].W, arr[i].stride = H, W, W
        arr[i].conn = int(conns[i])
        arr[i].scan = int(scans[i])
        arr[i].gray = int(bool(grays[i]))
        arr[i].order = int(orders[i])
        arr[i].tile = int(tl[i])
    return int(_lib.ccl_batch_workspace_bytes(arr, n, int(tile)))


def reserve(nbytes: int, stream=None):
    _check(_lib.ccl_reserve(int(nbytes), _stream_handle(stream)))


def release():
    _check(_lib.ccl_release())


PHASES = ("tile_scan", "boundary_merge", "flatten", "scan_blocks", "scan_totals", "component_labels", "labeling_pass")


def profile(enable: bool):
    """Record per-phase HIP events in every later call (see ccl_profile)."""
    _check(_lib.ccl_profile(int(bool(enable))))


def profile_read():
    """({phase: summed ms}, number of calls) since the previous read."""
    ms = (ctypes.c_double * len(PHASES))()
    n = ctypes.c_int(0)
    _check(_lib.ccl_profile_read(ms, len(PHASES), ctypes.byref(n)))
    return {p: ms[i] for i, p in enumerate(PHASES)}, n.value


def library_path() -> str:
    return LIB
