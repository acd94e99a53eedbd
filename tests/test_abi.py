"""The C ABI without a GPU: the library loads, exports every function that
include/ccl.h declares, and rejects bad arguments on the host with the
documented status codes before touching the device."""
import ctypes
import os
import re

import pytest

from paper_1606_05973_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccl.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(ccl_[a-z_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_api():
    names = _declared_functions()
    for expected in ("ccl_label", "ccl_label_ex", "ccl_label_batch", "ccl_workspace_bytes",
                     "ccl_batch_workspace_bytes", "ccl_reserve", "ccl_release", "ccl_tile_config",
                     "ccl_tile_count", "ccl_tile_default", "ccl_strerror", "ccl_batch_graph_create", "ccl_graph_launch",
                     "ccl_graph_destroy", "ccl_profile", "ccl_profile_read"):
        assert expected in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(build.LIB), "libccl.so not built"
    lib = ctypes.CDLL(build.LIB)
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_status_codes_on_host():
    from paper_1606_05973_amd import ccl
    S = ccl.STATUS
    dummy = 4096  # never dereferenced: the checks fail first
    assert ccl.label_raw(0, 10, 10, 10, 8, dummy, stream=0) == S["CCL_ERR_NULL"]
    assert ccl.label_raw(dummy, 10, 10, 10, 8, 0, stream=0) == S["CCL_ERR_NULL"]
    assert ccl.label_raw(dummy, 0, 10, 10, 8, dummy, stream=0) == S["CCL_ERR_SHAPE"]
    assert ccl.label_raw(dummy, 10, -1, 10, 8, dummy, stream=0) == S["CCL_ERR_SHAPE"]
    assert ccl.label_raw(dummy, 10, 10, 9, 8, dummy, stream=0) == S["CCL_ERR_STRIDE"]
    assert ccl.label_raw(dummy, 10, 10, 10, 6, dummy, stream=0) == S["CCL_ERR_CONN"]
    assert ccl.label_raw(dummy, 1 << 16, 1 << 15, 1 << 15, 8, dummy, stream=0) == S["CCL_ERR_TOO_LARGE"]
    lib = ccl._lib
    assert lib.ccl_label_ex(dummy, 10, 10, 10, 8, dummy, None, 99, None) == S["CCL_ERR_TILE"]
    assert lib.ccl_label_batch(None, -1, 0, None) == S["CCL_ERR_BATCH"]
    assert lib.ccl_label_batch(None, 3, 0, None) == S["CCL_ERR_BATCH"]
    assert lib.ccl_label_batch(None, 0, 0, None) == 0
    # a bad descriptor anywhere in the batch rejects the whole call
    arr = (ccl.ImageDesc * 2)()
    for i in range(2):
        arr[i].img, arr[i].labels = dummy, dummy
        arr[i].H = arr[i].W = arr[i].stride = 8
        arr[i].conn = 8
    arr[1].conn = 5
    assert lib.ccl_label_batch(arr, 2, 0, None) == S["CCL_ERR_CONN"]
    arr[1].conn = 4
    arr[0].level = 256
    assert lib.ccl_label_batch(arr, 2, 0, None) == S["CCL_ERR_LEVEL"]
    arr[0].level = -1
    assert lib.ccl_label_batch(arr, 2, 0, None) == S["CCL_ERR_LEVEL"]
    assert lib.ccl_label_level(dummy, 10, 10, 10, 256, 8, dummy, None, 0, None) == S["CCL_ERR_LEVEL"]
    assert lib.ccl_label_level(dummy, 10, 10, 10, -3, 8, dummy, None, 0, None) == S["CCL_ERR_LEVEL"]
    arr[0].level = 0
    arr[1].scan = 2
    assert lib.ccl_label_batch(arr, 2, 0, None) == S["CCL_ERR_SCAN"]
    arr[1].scan = 0
    arr[1].gray = 3
    assert lib.ccl_label_batch(arr, 2, 0, None) == S["CCL_ERR_GRAY"]
    arr[1].gray = 0
    assert lib.ccl_label_gray(dummy, 10, 10, 10, 300, 8, dummy, None, 0, None) == S["CCL_ERR_LEVEL"]
    assert lib.ccl_label_gray(dummy, 10, 10, 10, 0, 5, dummy, None, 0, None) == S["CCL_ERR_CONN"]
    arr[1].conn = 5
    # graph creation validates the same way before allocating anything
    h = ctypes.c_void_p()
    assert lib.ccl_batch_graph_create(arr, 2, 0, ctypes.byref(h)) == S["CCL_ERR_CONN"] and not h.value
    assert lib.ccl_batch_graph_create(arr, 0, 0, ctypes.byref(h)) == S["CCL_ERR_BATCH"]
    assert lib.ccl_graph_launch(None, None) == S["CCL_ERR_NULL"]
    assert lib.ccl_graph_destroy(None) == 0


def test_strerror_and_tiles():
    from paper_1606_05973_amd import ccl
    for code in [0, *ccl.STATUS.values()]:
        assert ccl.strerror(code) and ccl.strerror(code) != "unknown status"
    assert ccl.strerror(12345) == "unknown status"
    tiles = ccl.tile_configs()
    assert tiles[0] == (32, 256) and len(tiles) == ccl._lib.ccl_tile_count()
    for nsr, tw in tiles:
        assert tw % 64 == 0 and 2 * nsr * tw < 65536
    # id 0: each kind takes its own default
    assert ccl.tile_default(8) == 1 and ccl.tile_default(4) == 4 and ccl.tile_default(8, ccl.SCAN_ROW) == 4
    assert ccl.tile_default(8, gray=True) == 7 and ccl.tile_default(4, gray=True) == 7
    assert ccl.tile_shape(0, 8) == (64, 256) and ccl.tile_shape(0, 4) == (64, 128)
    assert ccl.tile_shape(0, 8, gray=True) == (32, 256)
    for bad in ((6, 0, 0), (8, 2, 0), (8, 0, 2)):
        assert ccl._lib.ccl_tile_default(*bad) == 0


def test_workspace_bytes():
    from paper_1606_05973_amd import ccl
    assert ccl.workspace_bytes(0, 10) == 0
    assert ccl.workspace_bytes(10, 10, conn=3) == 0
    a = ccl.workspace_bytes(1000, 1000)
    b = ccl.workspace_bytes(2000, 2000)
    assert 0 < a < b
    # worst-case per-tile capacities (every pixel its own component under
    # 4-conn): a few bytes per pixel, reported for admission by HBM footprint
    assert ccl.workspace_bytes(21568, 21568) < 4 * 21568 * 21568
    assert ccl.workspace_bytes(21568, 21568, conn=4) < 5 * 21568 * 21568
    both = ccl.batch_workspace_bytes([(1000, 1000), (2000, 2000)])
    assert both >= a + b - 1024
    # the one-row scan under 8-connectivity tiles like 4-connectivity
    assert ccl.workspace_bytes(1000, 1000, 8, scan=ccl.SCAN_ROW) == ccl.workspace_bytes(1000, 1000, 4)
    assert ccl.workspace_bytes(1000, 1000, 8, scan=7) == 0


def test_product_path_is_independent_of_the_oracle():
    """The package and its sources neither import nor include the oracle."""
    pkg = os.path.join(ROOT, "paper_1606_05973_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, flags=re.M), f
                assert "ccl_oracle" not in text, f


def test_level_of_matches_the_fractional_threshold():
    """level_of(f) must reproduce "v > f * 255" exactly for every byte v
    (exact rational arithmetic), e.g. f = 0.5 -> foreground iff v >= 128."""
    from fractions import Fraction

    from paper_1606_05973_amd import ccl
    for num in range(0, 1001):
        f = Fraction(num, 1000)
        lv = ccl.level_of(float(f))
        for v in range(256):
            assert (v > lv) == (v > f * 255), (num, v, lv)
    assert ccl.level_of(0.5) == 127
