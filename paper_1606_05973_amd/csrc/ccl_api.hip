// Host side of the gfx950 connected component labeling library: argument
// checks, workspace cache, launch sequence.  See include/ccl.h for the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "ccl.h"
#include "ccl_kernels.hpp"

namespace ccl {
namespace {

// ---------------------------------------------------------------- tiles
struct TileCfg {
    int th, tw;
};
// id 1 is the default.
constexpr TileCfg kTiles[] = {{32, 256}, {64, 256}, {16, 512}, {64, 128}, {32, 128}, {16, 256}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

inline int cap_of(const TileCfg &c) { return 2 * (c.th + c.tw); }

size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// Workspace layout of one image (byte offsets from the image's base).
struct Layout {
    int32_t NTY, NTX, NT, nblk, nedge;
    size_t he, ve, bl_idx, bl_val, bl_cnt, seg, blk, bytes;
};

Layout layout_of(int64_t H, int64_t W, const TileCfg &c) {
    Layout L{};
    L.NTY = (int32_t)((H + c.th - 1) / c.th);
    L.NTX = (int32_t)((W + c.tw - 1) / c.tw);
    L.NT = L.NTY * L.NTX;
    int64_t nseg = H * (int64_t)L.NTX;
    L.nblk = (int32_t)((nseg + kScanChunk - 1) / kScanChunk);
    L.nedge = (int32_t)((L.NTY - 1) * W + (L.NTX - 1) * H);
    size_t off = 0;
    L.he = off;
    off = align_up(off + (size_t)L.NTY * 2 * W * sizeof(uint16_t));
    L.ve = off;
    off = align_up(off + (size_t)L.NTX * 2 * H * sizeof(uint16_t));
    L.bl_idx = off;
    off = align_up(off + (size_t)L.NT * cap_of(c) * sizeof(int32_t));
    L.bl_val = off;
    off = align_up(off + (size_t)L.NT * cap_of(c) * sizeof(int32_t));
    L.bl_cnt = off;
    off = align_up(off + (size_t)L.NT * sizeof(int32_t));
    L.seg = off;
    off = align_up(off + (size_t)nseg * sizeof(int32_t));
    L.blk = off;
    off = align_up(off + (size_t)L.nblk * sizeof(int32_t));
    L.bytes = off;
    return L;
}

int check_image(const void *img, int64_t H, int64_t W, int64_t stride, int conn, const void *labels) {
    if (!img || !labels)
        return CCL_ERR_NULL;
    if (H <= 0 || W <= 0)
        return CCL_ERR_SHAPE;
    if (stride < W)
        return CCL_ERR_STRIDE;
    if (conn != 4 && conn != 8)
        return CCL_ERR_CONN;
    if (H > INT32_MAX || W > INT32_MAX || H * W >= (int64_t)INT32_MAX)
        return CCL_ERR_TOO_LARGE;
    return CCL_OK;
}

int resolve_tile(int tile, TileCfg *out) {
    if (tile == 0)
        tile = 1;
    if (tile < 1 || tile > kNumTiles)
        return CCL_ERR_TILE;
    *out = kTiles[tile - 1];
    return CCL_OK;
}

// ------------------------------------------------------------- workspace
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

// Workspace of (current device, stream) with at least `need` bytes.
int get_workspace(hipStream_t stream, size_t need, void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return CCL_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace &w = g_ws[{dev, stream}];
    if (w.bytes < need) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(stream, &cs) != hipSuccess)
            return CCL_ERR_HIP;
        if (cs != hipStreamCaptureStatusNone)
            return CCL_ERR_CAPTURE;
        if (w.ptr) {
            if (hipStreamSynchronize(stream) != hipSuccess)
                return CCL_ERR_HIP;
            (void)hipFree(w.ptr);
            w.ptr = nullptr;
            w.bytes = 0;
        }
        size_t grow = std::max(need, (size_t)1 << 20);
        if (hipMalloc(&w.ptr, grow) != hipSuccess) {
            (void)hipGetLastError();
            w.ptr = nullptr;
            return CCL_ERR_NOMEM;
        }
        w.bytes = grow;
    }
    *out = w.ptr;
    return CCL_OK;
}

// Fill an Img from a descriptor, its layout and its workspace base.
Img make_img(const ccl_image_desc &d, const Layout &L, char *base) {
    Img im{};
    im.img = d.img;
    im.labels = d.labels;
    im.ncomp = d.num_components;
    im.he = reinterpret_cast<uint16_t *>(base + L.he);
    im.ve = reinterpret_cast<uint16_t *>(base + L.ve);
    im.bl_idx = reinterpret_cast<int32_t *>(base + L.bl_idx);
    im.bl_val = reinterpret_cast<int32_t *>(base + L.bl_val);
    im.bl_cnt = reinterpret_cast<int32_t *>(base + L.bl_cnt);
    im.seg = reinterpret_cast<int32_t *>(base + L.seg);
    im.blk = reinterpret_cast<int32_t *>(base + L.blk);
    im.stride = d.stride;
    im.H = (int32_t)d.H;
    im.W = (int32_t)d.W;
    im.NTY = L.NTY;
    im.NTX = L.NTX;
    im.conn = d.conn;
    im.nblk = L.nblk;
    return im;
}

template <int TH, int TW>
int launch_all(const Batch &b, int64_t tiles, int64_t edges, int64_t blocks, int nimg, hipStream_t s) {
    if (tiles > INT32_MAX || edges > INT32_MAX || blocks > INT32_MAX)
        return CCL_ERR_TOO_LARGE;
    const dim3 blk(kThreads);
    hipLaunchKernelGGL((k_tile_scan<TH, TW>), dim3((uint32_t)tiles), blk, 0, s, b);
    if (edges > 0)
        hipLaunchKernelGGL((k_merge<TH, TW>), dim3((uint32_t)((edges + kThreads - 1) / kThreads)), blk, 0, s, b);
    hipLaunchKernelGGL((k_flatten<TH, TW>), dim3((uint32_t)tiles), blk, 0, s, b);
    hipLaunchKernelGGL(k_scan_blocks, dim3((uint32_t)blocks), blk, 0, s, b);
    hipLaunchKernelGGL(k_scan_top, dim3((uint32_t)nimg), blk, 0, s, b);
    hipLaunchKernelGGL((k_publish<TH, TW>), dim3((uint32_t)tiles), blk, 0, s, b);
    hipLaunchKernelGGL((k_relabel<TH, TW>), dim3((uint32_t)tiles), blk, 0, s, b);
    return hipGetLastError() == hipSuccess ? CCL_OK : CCL_ERR_HIP;
}

int dispatch(const TileCfg &c, const Batch &b, int64_t tiles, int64_t edges, int64_t blocks, int nimg,
             hipStream_t s) {
#define CCL_TILE_CASE(H_, W_) \
    if (c.th == H_ && c.tw == W_) \
        return launch_all<H_, W_>(b, tiles, edges, blocks, nimg, s);
    CCL_TILE_CASE(32, 256)
    CCL_TILE_CASE(64, 256)
    CCL_TILE_CASE(16, 512)
    CCL_TILE_CASE(64, 128)
    CCL_TILE_CASE(32, 128)
    CCL_TILE_CASE(16, 256)
#undef CCL_TILE_CASE
    return CCL_ERR_TILE;
}

// Device table of a batch: kept per (device, stream) like the workspace.
int run_batch(const ccl_image_desc *descs, int n, const TileCfg &c, hipStream_t stream) {
    std::vector<Layout> lays(n);
    size_t total = align_up((size_t)n * sizeof(Img));
    for (int i = 0; i < n; i++) {
        lays[i] = layout_of(descs[i].H, descs[i].W, c);
        total += lays[i].bytes;
    }
    void *ws = nullptr;
    int st = get_workspace(stream, total, &ws);
    if (st != CCL_OK)
        return st;
    char *base = static_cast<char *>(ws);
    std::vector<Img> tab(n);
    size_t off = align_up((size_t)n * sizeof(Img));
    int64_t tiles = 0, edges = 0, blocks = 0;
    for (int i = 0; i < n; i++) {
        tab[i] = make_img(descs[i], lays[i], base + off);
        tab[i].tile0 = (int32_t)tiles;
        tab[i].edge0 = (int32_t)edges;
        tab[i].scan0 = (int32_t)blocks;
        off += lays[i].bytes;
        tiles += lays[i].NT;
        edges += lays[i].nedge;
        blocks += lays[i].nblk;
        if (tiles > INT32_MAX || edges > INT32_MAX || blocks > INT32_MAX)
            return CCL_ERR_TOO_LARGE;
    }
    Batch b{};
    b.n = n;
    if (n == 1) {
        b.one = tab[0];
        b.tab = nullptr;
    } else {
        if (hipMemcpyAsync(base, tab.data(), (size_t)n * sizeof(Img), hipMemcpyHostToDevice, stream) != hipSuccess)
            return CCL_ERR_HIP;
        b.tab = reinterpret_cast<const Img *>(base);
    }
    return dispatch(c, b, tiles, edges, blocks, n, stream);
}

}  // namespace
}  // namespace ccl

using namespace ccl;

extern "C" {

int ccl_label_ex(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn, int32_t *labels,
                 int32_t *num_components, int tile, hipStream_t stream) {
    int st = check_image(img, H, W, stride, conn, labels);
    if (st != CCL_OK)
        return st;
    TileCfg c;
    if ((st = resolve_tile(tile, &c)) != CCL_OK)
        return st;
    ccl_image_desc d{img, H, W, stride, conn, labels, num_components};
    return run_batch(&d, 1, c, stream);
}

int ccl_label(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn, int32_t *labels,
              hipStream_t stream) {
    return ccl_label_ex(img, H, W, stride, conn, labels, nullptr, 0, stream);
}

int ccl_label_batch(const ccl_image_desc *descs, int n, int tile, hipStream_t stream) {
    if (n < 0 || (n > 0 && !descs))
        return CCL_ERR_BATCH;
    TileCfg c;
    int st = resolve_tile(tile, &c);
    if (st != CCL_OK)
        return st;
    if (n == 0)
        return CCL_OK;
    for (int i = 0; i < n; i++) {
        st = check_image(descs[i].img, descs[i].H, descs[i].W, descs[i].stride, descs[i].conn, descs[i].labels);
        if (st != CCL_OK)
            return st;
    }
    return run_batch(descs, n, c, stream);
}

size_t ccl_workspace_bytes(int64_t H, int64_t W, int conn, int tile) {
    TileCfg c;
    if (resolve_tile(tile, &c) != CCL_OK)
        return 0;
    int8_t dummy;
    if (check_image(&dummy, H, W, W, conn, &dummy) != CCL_OK)
        return 0;
    return align_up(sizeof(Img)) + layout_of(H, W, c).bytes;
}

size_t ccl_batch_workspace_bytes(const ccl_image_desc *descs, int n, int tile) {
    TileCfg c;
    if (resolve_tile(tile, &c) != CCL_OK || n < 0 || (n > 0 && !descs))
        return 0;
    size_t total = align_up((size_t)n * sizeof(Img));
    for (int i = 0; i < n; i++) {
        int8_t dummy;
        if (check_image(&dummy, descs[i].H, descs[i].W, descs[i].stride, descs[i].conn, &dummy) != CCL_OK)
            return 0;
        total += layout_of(descs[i].H, descs[i].W, c).bytes;
    }
    return total;
}

int ccl_reserve(size_t bytes, hipStream_t stream) {
    void *p = nullptr;
    return get_workspace(stream, bytes, &p);
}

int ccl_release(void) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return CCL_ERR_HIP;
    if (hipDeviceSynchronize() != hipSuccess)
        return CCL_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto it = g_ws.begin(); it != g_ws.end();) {
        if (it->first.first == dev) {
            (void)hipFree(it->second.ptr);
            it = g_ws.erase(it);
        } else {
            ++it;
        }
    }
    return CCL_OK;
}

int ccl_tile_count(void) { return kNumTiles; }

int ccl_tile_config(int id, int *tile_h, int *tile_w) {
    TileCfg c;
    int st = resolve_tile(id, &c);
    if (st != CCL_OK)
        return st;
    if (tile_h)
        *tile_h = c.th;
    if (tile_w)
        *tile_w = c.tw;
    return CCL_OK;
}

const char *ccl_strerror(int status) {
    switch (status) {
    case CCL_OK: return "success";
    case CCL_ERR_NULL: return "a required pointer is NULL";
    case CCL_ERR_SHAPE: return "H and W must be positive";
    case CCL_ERR_STRIDE: return "stride must be >= W";
    case CCL_ERR_CONN: return "conn must be 4 or 8";
    case CCL_ERR_TOO_LARGE: return "H*W must be below 2^31-1";
    case CCL_ERR_NOMEM: return "workspace allocation failed";
    case CCL_ERR_HIP: return "HIP runtime call or kernel launch failed";
    case CCL_ERR_TILE: return "unknown tile configuration";
    case CCL_ERR_CAPTURE: return "workspace cannot grow while the stream is being captured (call ccl_reserve first)";
    case CCL_ERR_BATCH: return "invalid batch (n < 0 or descs NULL)";
    default: return "unknown status";
    }
}

}  // extern "C"
