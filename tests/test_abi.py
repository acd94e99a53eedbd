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
    for expected in ("ccl_label", "ccl_label_ex", "ccl_label_batch", "ccl_label_batch_ex", "ccl_workspace_bytes",
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
    # sides that would overflow int32 once rounded up to tiles and edge lines
    assert ccl.label_raw(dummy, 1, (1 << 31) - 200, (1 << 31) - 200, 8, dummy, stream=0) == S["CCL_ERR_TOO_LARGE"]
    assert ccl.label_raw(dummy, (1 << 31) - 200, 1, 1, 8, dummy, stream=0) == S["CCL_ERR_TOO_LARGE"]
    # H*W below 2^31, but 2^22 tiles of one row: more boundary slots than 32-bit ids address
    assert ccl.label_raw(dummy, 1, 1 << 30, 1 << 30, 8, dummy, stream=0) == S["CCL_ERR_TOO_LARGE"]
    lib = ccl._lib
    assert lib.ccl_label_ex(dummy, 10, 10, 10, 8, dummy, None, 99, None) == S["CCL_ERR_TILE"]
    # the plain batch call (descriptor of seven fields, no options)
    assert lib.ccl_label_batch(None, -1, None) == S["CCL_ERR_BATCH"]
    assert lib.ccl_label_batch(None, 3, None) == S["CCL_ERR_BATCH"]
    assert lib.ccl_label_batch(None, 0, None) == 0
    plain = (ccl.ImageDesc * 2)()
    for i in range(2):
        plain[i].img, plain[i].labels = dummy, dummy
        plain[i].H = plain[i].W = plain[i].stride = 8
        plain[i].conn = 8
    plain[1].stride = 7
    assert lib.ccl_label_batch(plain, 2, None) == S["CCL_ERR_STRIDE"]
    plain[1].stride = 8
    plain[0].labels = None
    assert lib.ccl_label_batch(plain, 2, None) == S["CCL_ERR_NULL"]
    # the extended batch call
    assert lib.ccl_label_batch_ex(None, -1, 0, None) == S["CCL_ERR_BATCH"]
    assert lib.ccl_label_batch_ex(None, 0, 0, None) == 0
    # a bad descriptor anywhere in the batch rejects the whole call
    arr = (ccl.ImageDescEx * 2)()
    for i in range(2):
        arr[i].img, arr[i].labels = dummy, dummy
        arr[i].H = arr[i].W = arr[i].stride = 8
        arr[i].conn = 8
    assert lib.ccl_label_batch_ex(arr, 2, 99, None) == S["CCL_ERR_TILE"]
    arr[1].conn = 5
    assert lib.ccl_label_batch_ex(arr, 2, 0, None) == S["CCL_ERR_CONN"]
    arr[1].conn = 4
    arr[0].level = 256
    assert lib.ccl_label_batch_ex(arr, 2, 0, None) == S["CCL_ERR_LEVEL"]
    arr[0].level = -1
    assert lib.ccl_label_batch_ex(arr, 2, 0, None) == S["CCL_ERR_LEVEL"]
    assert lib.ccl_label_level(dummy, 10, 10, 10, 256, 8, dummy, None, 0, None) == S["CCL_ERR_LEVEL"]
    assert lib.ccl_label_level(dummy, 10, 10, 10, -3, 8, dummy, None, 0, None) == S["CCL_ERR_LEVEL"]
    arr[0].level = 0
    arr[1].scan = 2
    assert lib.ccl_label_batch_ex(arr, 2, 0, None) == S["CCL_ERR_SCAN"]
    arr[1].scan = 0
    arr[1].gray = 3
    assert lib.ccl_label_batch_ex(arr, 2, 0, None) == S["CCL_ERR_GRAY"]
    arr[1].gray = 0
    arr[1].order = 2
    assert lib.ccl_label_batch_ex(arr, 2, 0, None) == S["CCL_ERR_ORDER"]
    arr[1].order = 0
    arr[0].tile = 8
    assert lib.ccl_label_batch_ex(arr, 2, 0, None) == S["CCL_ERR_TILE"]
    arr[0].tile = -1
    assert lib.ccl_label_batch_ex(arr, 2, 0, None) == S["CCL_ERR_TILE"]
    arr[0].tile = 0
    assert lib.ccl_label_provisional(dummy, 10, 10, 10, 8, dummy, None, 9, None) == S["CCL_ERR_TILE"]
    assert lib.ccl_label_provisional(dummy, 10, 10, 10, 3, dummy, None, 0, None) == S["CCL_ERR_CONN"]
    assert lib.ccl_label_gray(dummy, 10, 10, 10, 300, 8, dummy, None, 0, None) == S["CCL_ERR_LEVEL"]
    assert lib.ccl_label_gray(dummy, 10, 10, 10, 0, 5, dummy, None, 0, None) == S["CCL_ERR_CONN"]
    arr[1].conn = 5
    # graph creation validates the same way before allocating anything
    h = ctypes.c_void_p()
    assert lib.ccl_batch_graph_create(arr, 2, 0, ctypes.byref(h)) == S["CCL_ERR_CONN"] and not h.value
    assert lib.ccl_batch_graph_create(arr, 0, 0, ctypes.byref(h)) == S["CCL_ERR_BATCH"]
    assert lib.ccl_graph_launch(None, None) == S["CCL_ERR_NULL"]
    assert lib.ccl_graph_destroy(None) == 0


def test_descriptor_layouts_match_the_header(tmp_path):
    """The ctypes descriptors have the size and field offsets that a C
    compiler gives the structs of include/ccl.h."""
    import subprocess

    from paper_1606_05973_amd import ccl
    fields = {"ccl_image_desc": (ccl.ImageDesc, ["img", "H", "W", "stride", "conn", "labels", "num_components"]),
              "ccl_image_desc_ex": (ccl.ImageDescEx, ["img", "H", "W", "stride", "conn", "labels", "num_components",
                                                      "level", "scan", "gray", "order", "tile"]),
              "ccl_server_config": (ccl.ServerConfig, ["n_streams", "max_batch", "max_batch_pixels", "hbm_budget",
                                                       "tile"]),
              "ccl_server_stats": (ccl.ServerStats, ["submitted", "completed", "rejected", "batches",
                                                     "in_flight_max", "pixels_completed", "p50_ms", "p99_ms",
                                                     "mean_ms"])}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ccl.h"', 'int main(void) {']
    for st, (_, names) in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in names:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    for st, (cls, names) in fields.items():
        assert int(got[st]) == ctypes.sizeof(cls), st
        for f in names:
            assert int(got[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)


def test_noalloc_checks_on_host():
    """ccl_label_noalloc rejects bad arguments and images beyond its static
    scratch before any device call; the limit is the header's."""
    from paper_1606_05973_amd import ccl
    S = ccl.STATUS
    lib = ccl._lib
    dummy = 4096  # never dereferenced: the checks fail first
    assert lib.ccl_label_noalloc(None, 10, 10, 10, 8, dummy, None, None) == S["CCL_ERR_NULL"]
    assert lib.ccl_label_noalloc(dummy, 10, 0, 10, 8, dummy, None, None) == S["CCL_ERR_SHAPE"]
    assert lib.ccl_label_noalloc(dummy, 10, 10, 10, 5, dummy, None, None) == S["CCL_ERR_CONN"]
    assert lib.ccl_label_noalloc(dummy, 8192, 8192, 8192, 8, dummy, None, None) == S["CCL_ERR_SCRATCH"]
    assert lib.ccl_label_noalloc(dummy, 1, 20000000, 20000000, 8, dummy, None, None) == S["CCL_ERR_SCRATCH"]
    m = re.search(r"#define CCL_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", open(HEADER).read())
    assert m and int(m.group(1)) << int(m.group(2)) == ccl.NOALLOC_SCRATCH_BYTES
    for conn in (4, 8):
        assert 0 < lib.ccl_workspace_bytes(4096, 4096, conn) <= ccl.NOALLOC_SCRATCH_BYTES
    assert lib.ccl_workspace_bytes(8192, 8192, 8) > ccl.NOALLOC_SCRATCH_BYTES


def test_batch_descriptor_rows_match_the_struct():
    """The numpy rows a batch call fills have the ccl_image_desc_ex layout."""
    import numpy as np
    from paper_1606_05973_amd import ccl
    dt = ccl._DESC_DTYPE
    assert dt.itemsize == ctypes.sizeof(ccl.ImageDescEx)
    for name, ctype in ccl.ImageDescEx._fields_:
        assert dt.fields[name][1] == getattr(ccl.ImageDescEx, name).offset, name
        assert dt.fields[name][0].itemsize == ctypes.sizeof(ctype), name
    rows = np.zeros(2, dtype=dt)
    rows["H"], rows["tile"], rows["labels"] = [7, 9], [3, 4], [1 << 40, 5]
    arr = ctypes.cast(rows.ctypes.data, ctypes.POINTER(ccl.ImageDescEx))
    assert (arr[1].H, arr[1].tile, arr[0].labels, arr[1].labels) == (9, 4, 1 << 40, 5)


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


def test_header_boundary_signatures():
    """The six calls of the contract, with exactly its argument lists."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    src = re.sub(r"\s+", " ", src)
    for decl in ("int ccl_label(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn, "
                 "int32_t *labels, hipStream_t stream);",
                 "int ccl_label_batch(const ccl_image_desc *descs, int n, hipStream_t stream);",
                 "size_t ccl_workspace_bytes(int64_t H, int64_t W, int conn);",
                 "int ccl_reserve(size_t bytes, hipStream_t stream);",
                 "const char *ccl_strerror(int status);",
                 "typedef struct { const uint8_t *img; int64_t H, W, stride; int conn; int32_t *labels; "
                 "int32_t *num_components; } ccl_image_desc;"):
        assert decl in src, decl


def test_workspace_bytes():
    from paper_1606_05973_amd import ccl
    assert ccl._lib.ccl_workspace_bytes(1000, 1000, 8) == ccl.workspace_bytes(1000, 1000)
    assert ccl._lib.ccl_workspace_bytes(1000, 1000, 5) == 0
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
    # provisional order scans one count per tile instead of one per (row, tile column)
    assert 0 < ccl.batch_workspace_bytes([(1000, 1000)], order=ccl.PROVISIONAL) < a
    # images of different tiles or orders form separate launch groups (a table each)
    mixed = ccl.batch_workspace_bytes([(300, 300)] * 4, tiles=[1, 2, 1, 2])
    same = ccl.batch_workspace_bytes([(300, 300)] * 4, tiles=[1, 1, 1, 1])
    assert mixed > 0 and same > 0 and mixed != same


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
