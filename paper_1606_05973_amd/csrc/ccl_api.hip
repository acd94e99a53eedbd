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
// A tile configuration is (block rows, width).  The tile height is block
// rows x 2 under 8-connectivity (two image rows per block row) and block
// rows x 1 under 4-connectivity.  id 1 is the default.
struct TileCfg {
    int nsr, tw;
};
constexpr TileCfg kTiles[] = {{32, 256}, {16, 256}, {16, 512}, {64, 128}, {32, 128}, {8, 512}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

// Image rows per block row: two under 8-connectivity with the pair-row scan
// (the default), one otherwise.
inline int bh_of(int conn, int scan) { return (conn == 8 && scan == CCL_SCAN_PAIR) ? 2 : 1; }
inline int bh_of(const ccl_image_desc &d) { return bh_of(d.conn, d.scan); }

size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// Workspace layout of one image (byte offsets from the image's base).
struct Layout {
    int32_t th, NTY, NTX, NT, nblk, nedge, nm, rcap, rw, cap;
    size_t masks, rt, cb, cf, tcnt, he, ve, uf, bval, bkey, broot, seg, blk, bytes;
};

Layout layout_of(int64_t H, int64_t W, int bh, const TileCfg &c) {
    Layout L{};
    L.th = c.nsr * bh;
    L.NTY = (int32_t)((H + L.th - 1) / L.th);
    L.NTX = (int32_t)((W + c.tw - 1) / c.tw);
    L.NT = L.NTY * L.NTX;
    L.nm = L.th * (c.tw / 32);
    L.rcap = c.nsr * (c.tw / 2);
    L.rw = L.rcap / 32;
    L.cap = 2 * (L.th + c.tw);
    const int64_t nseg = H * (int64_t)L.NTX;
    L.nblk = (int32_t)((nseg + kScanChunk - 1) / kScanChunk);
    L.nedge = (int32_t)((L.NTY - 1) * ((W + 31) / 32) + (L.NTX - 1) * ((H + 31) / 32));
    const size_t NT = (size_t)L.NT;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.masks = take(NT * L.nm * sizeof(uint32_t));
    L.rt = take(NT * L.rcap * sizeof(uint16_t));
    L.cb = take(NT * L.rw * sizeof(uint32_t));
    L.cf = take(NT * L.rcap * sizeof(int32_t));
    L.tcnt = take(NT * 4 * sizeof(int32_t));
    L.he = take((size_t)L.NTY * 2 * W * sizeof(uint16_t));
    L.ve = take((size_t)L.NTX * 2 * H * sizeof(uint16_t));
    L.uf = take(NT * L.cap * sizeof(uint64_t));
    L.bval = take(NT * L.cap * sizeof(int32_t));
    L.bkey = take(NT * L.cap * sizeof(uint16_t));
    L.broot = take(NT * L.cap * sizeof(uint8_t));
    L.seg = take((size_t)nseg * sizeof(int32_t));
    L.blk = take((size_t)L.nblk * sizeof(int32_t));
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

int check_level(int level) { return (level < 0 || level > 255) ? CCL_ERR_LEVEL : CCL_OK; }

int check_opts(const ccl_image_desc &d) {
    if (d.scan != CCL_SCAN_PAIR && d.scan != CCL_SCAN_ROW)
        return CCL_ERR_SCAN;
    return check_level(d.level);
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
    im.masks = reinterpret_cast<uint32_t *>(base + L.masks);
    im.rt = reinterpret_cast<uint16_t *>(base + L.rt);
    im.cb = reinterpret_cast<uint32_t *>(base + L.cb);
    im.cf = reinterpret_cast<int32_t *>(base + L.cf);
    im.tcnt = reinterpret_cast<int32_t *>(base + L.tcnt);
    im.he = reinterpret_cast<uint16_t *>(base + L.he);
    im.ve = reinterpret_cast<uint16_t *>(base + L.ve);
    im.uf = reinterpret_cast<uint64_t *>(base + L.uf);
    im.bval = reinterpret_cast<int32_t *>(base + L.bval);
    im.bkey = reinterpret_cast<uint16_t *>(base + L.bkey);
    im.broot = reinterpret_cast<uint8_t *>(base + L.broot);
    im.seg = reinterpret_cast<int32_t *>(base + L.seg);
    im.blk = reinterpret_cast<int32_t *>(base + L.blk);
    im.stride = d.stride;
    im.H = (int32_t)d.H;
    im.W = (int32_t)d.W;
    im.NTY = L.NTY;
    im.NTX = L.NTX;
    im.conn = d.conn;
    im.level = d.level;
    im.nblk = L.nblk;
    return im;
}

// ------------------------------------------------------------- profiling
// When enabled, every call records one HIP event before each phase and one
// after the last, on the call's own stream; ccl_profile_read turns them into
// per-phase milliseconds.
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<std::vector<hipEvent_t>> g_prof_pending;  // one vector per call
std::vector<hipEvent_t> g_prof_free;

hipEvent_t prof_event() {
    hipEvent_t e = nullptr;
    if (!g_prof_free.empty()) {
        e = g_prof_free.back();
        g_prof_free.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
    }
    return e;
}

struct PhaseMarks {
    std::vector<hipEvent_t> ev;
    hipStream_t s;
    bool on;
    explicit PhaseMarks(hipStream_t st) : s(st) {
        {
            std::lock_guard<std::mutex> lk(g_prof_mu);
            on = g_prof_on;
        }
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (on && (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone))
            on = false;  // no event nodes inside captured graphs
    }
    void mark() {
        if (!on)
            return;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        hipEvent_t e = prof_event();
        if (e && hipEventRecord(e, s) == hipSuccess)
            ev.push_back(e);
        else
            on = false;
    }
    ~PhaseMarks() {
        if (!ev.empty()) {
            std::lock_guard<std::mutex> lk(g_prof_mu);
            g_prof_pending.push_back(ev);
        }
    }
};

// Workgroups of a persistent launch of `kernel`: as many as can be resident
// at once (occupancy x CUs), computed once per kernel instantiation.
template <auto kernel>
int persistent_groups(int threads) {
    static int n = 0;
    if (n == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu <= 0)
            per_cu = 1;
        n = cus * per_cu;
    }
    return n;
}

template <int NSR, int TW, int BH>
int launch_all(const Batch &b, int64_t tiles, int64_t edges, int64_t blocks, int nimg, hipStream_t s) {
    if (tiles > INT32_MAX || edges > INT32_MAX || blocks > INT32_MAX)
        return CCL_ERR_TOO_LARGE;
    const dim3 blk(kThreads);
    PhaseMarks pm(s);
    pm.mark();
    hipLaunchKernelGGL((k_tile_scan<NSR, TW, BH>), dim3((uint32_t)tiles), dim3(kTileThreads), 0, s, b);
    pm.mark();
    if (edges > 0)
        hipLaunchKernelGGL((k_merge<NSR, TW, BH>), dim3((uint32_t)((edges + kThreads - 1) / kThreads)), blk, 0, s, b);
    pm.mark();
    hipLaunchKernelGGL((k_flatten<NSR, TW, BH>), dim3((uint32_t)tiles), blk, 0, s, b);
    pm.mark();
    hipLaunchKernelGGL(k_scan_blocks, dim3((uint32_t)blocks), blk, 0, s, b);
    pm.mark();
    hipLaunchKernelGGL(k_scan_top, dim3((uint32_t)nimg), blk, 0, s, b);
    pm.mark();
    hipLaunchKernelGGL((k_comp_labels<NSR, TW, BH>), dim3((uint32_t)tiles), blk, 0, s, b);
    pm.mark();
    hipLaunchKernelGGL((k_relabel<NSR, TW, BH>),
                       dim3((uint32_t)std::min<int64_t>(tiles, persistent_groups<k_relabel<NSR, TW, BH>>(kTileThreads))),
                       dim3(kTileThreads), 0, s, b, (int32_t)tiles);
    pm.mark();
    return hipGetLastError() == hipSuccess ? CCL_OK : CCL_ERR_HIP;
}

int dispatch(const TileCfg &c, int bh, const Batch &b, int64_t tiles, int64_t edges, int64_t blocks, int nimg,
             hipStream_t s) {
#define CCL_TILE_CASE(N_, W_)                                                   \
    if (c.nsr == N_ && c.tw == W_)                                              \
        return bh == 2 ? launch_all<N_, W_, 2>(b, tiles, edges, blocks, nimg, s) \
                       : launch_all<N_, W_, 1>(b, tiles, edges, blocks, nimg, s);
    CCL_TILE_CASE(32, 256)
    CCL_TILE_CASE(16, 256)
    CCL_TILE_CASE(16, 512)
    CCL_TILE_CASE(64, 128)
    CCL_TILE_CASE(32, 128)
    CCL_TILE_CASE(8, 512)
#undef CCL_TILE_CASE
    return CCL_ERR_TILE;
}

// Images of one connectivity share every launch; a batch mixing 4- and
// 8-connectivity runs as two such groups, one after the other on the stream.
// Workspace: [tables of both groups][per-image regions].
int run_group(const ccl_image_desc *descs, const std::vector<int> &idx, const std::vector<Layout> &lays,
              const std::vector<size_t> &offs, char *base, Img *dtab, int bh, const TileCfg &c,
              hipStream_t stream, bool table_ready = false) {
    const int n = (int)idx.size();
    if (n == 0)
        return CCL_OK;
    std::vector<Img> tab(n);
    int64_t tiles = 0, edges = 0, blocks = 0;
    for (int k = 0; k < n; k++) {
        const int i = idx[k];
        tab[k] = make_img(descs[i], lays[i], base + offs[i]);
        tab[k].tile0 = (int32_t)tiles;
        tab[k].edge0 = (int32_t)edges;
        tab[k].scan0 = (int32_t)blocks;
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
        if (!table_ready &&
            hipMemcpyAsync(dtab, tab.data(), (size_t)n * sizeof(Img), hipMemcpyHostToDevice, stream) != hipSuccess)
            return CCL_ERR_HIP;
        b.tab = dtab;
    }
    return dispatch(c, bh, b, tiles, edges, blocks, n, stream);
}

size_t batch_bytes(const ccl_image_desc *descs, int n, const TileCfg &c, std::vector<Layout> *lays,
                   std::vector<size_t> *offs) {
    size_t off = align_up((size_t)n * sizeof(Img));
    for (int i = 0; i < n; i++) {
        Layout L = layout_of(descs[i].H, descs[i].W, bh_of(descs[i]), c);
        if (lays)
            lays->push_back(L);
        if (offs)
            offs->push_back(off);
        off += L.bytes;
    }
    return off;
}

int run_batch(const ccl_image_desc *descs, int n, const TileCfg &c, hipStream_t stream) {
    std::vector<Layout> lays;
    std::vector<size_t> offs;
    const size_t total = batch_bytes(descs, n, c, &lays, &offs);
    void *ws = nullptr;
    int st = get_workspace(stream, total, &ws);
    if (st != CCL_OK)
        return st;
    char *base = static_cast<char *>(ws);
    std::vector<int> g2, g1;  // by image rows per block row
    for (int i = 0; i < n; i++)
        (bh_of(descs[i]) == 2 ? g2 : g1).push_back(i);
    Img *dtab = reinterpret_cast<Img *>(base);
    st = run_group(descs, g2, lays, offs, base, dtab, 2, c, stream);
    if (st != CCL_OK)
        return st;
    return run_group(descs, g1, lays, offs, base, dtab + g2.size(), 1, c, stream);
}

// Device table of one group, uploaded synchronously (used before capture).
int upload_group_table(const ccl_image_desc *descs, const std::vector<int> &idx, const std::vector<Layout> &lays,
                       const std::vector<size_t> &offs, char *base, Img *dtab) {
    const int n = (int)idx.size();
    if (n <= 1)
        return CCL_OK;
    std::vector<Img> tab(n);
    int64_t tiles = 0, edges = 0, blocks = 0;
    for (int k = 0; k < n; k++) {
        const int i = idx[k];
        tab[k] = make_img(descs[i], lays[i], base + offs[i]);
        tab[k].tile0 = (int32_t)tiles;
        tab[k].edge0 = (int32_t)edges;
        tab[k].scan0 = (int32_t)blocks;
        tiles += lays[i].NT;
        edges += lays[i].nedge;
        blocks += lays[i].nblk;
    }
    return hipMemcpy(dtab, tab.data(), (size_t)n * sizeof(Img), hipMemcpyHostToDevice) == hipSuccess ? CCL_OK
                                                                                                     : CCL_ERR_HIP;
}

}  // namespace
}  // namespace ccl

struct ccl_graph {
    void *ws = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

using namespace ccl;

extern "C" {

int ccl_label_level(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int level, int conn,
                    int32_t *labels, int32_t *num_components, int tile, hipStream_t stream) {
    int st = check_image(img, H, W, stride, conn, labels);
    if (st != CCL_OK)
        return st;
    if ((st = check_level(level)) != CCL_OK)
        return st;
    TileCfg c;
    if ((st = resolve_tile(tile, &c)) != CCL_OK)
        return st;
    ccl_image_desc d{img, H, W, stride, conn, labels, num_components, level, CCL_SCAN_PAIR};
    return run_batch(&d, 1, c, stream);
}

int ccl_label_ex(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn, int32_t *labels,
                 int32_t *num_components, int tile, hipStream_t stream) {
    return ccl_label_level(img, H, W, stride, 0, conn, labels, num_components, tile, stream);
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
        if (st == CCL_OK)
            st = check_opts(descs[i]);
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
    ccl_image_desc d{reinterpret_cast<const uint8_t *>(&dummy), H, W, W, conn, reinterpret_cast<int32_t *>(&dummy),
                     nullptr, 0, CCL_SCAN_PAIR};
    return batch_bytes(&d, 1, c, nullptr, nullptr);
}

size_t ccl_batch_workspace_bytes(const ccl_image_desc *descs, int n, int tile) {
    TileCfg c;
    if (resolve_tile(tile, &c) != CCL_OK || n < 0 || (n > 0 && !descs))
        return 0;
    for (int i = 0; i < n; i++) {
        int8_t dummy;
        if (check_image(&dummy, descs[i].H, descs[i].W, descs[i].stride, descs[i].conn, &dummy) != CCL_OK ||
            check_opts(descs[i]) != CCL_OK)
            return 0;
    }
    return batch_bytes(descs, n, c, nullptr, nullptr);
}

int ccl_batch_graph_create(const ccl_image_desc *descs, int n, int tile, ccl_graph **out) {
    if (!out)
        return CCL_ERR_NULL;
    *out = nullptr;
    if (n <= 0 || !descs)
        return CCL_ERR_BATCH;
    TileCfg c;
    int st = resolve_tile(tile, &c);
    if (st != CCL_OK)
        return st;
    for (int i = 0; i < n; i++) {
        st = check_image(descs[i].img, descs[i].H, descs[i].W, descs[i].stride, descs[i].conn, descs[i].labels);
        if (st == CCL_OK)
            st = check_opts(descs[i]);
        if (st != CCL_OK)
            return st;
    }
    std::vector<Layout> lays;
    std::vector<size_t> offs;
    const size_t total = batch_bytes(descs, n, c, &lays, &offs);
    ccl_graph *g = new ccl_graph();
    if (hipMalloc(&g->ws, total) != hipSuccess) {
        (void)hipGetLastError();
        delete g;
        return CCL_ERR_NOMEM;
    }
    char *base = static_cast<char *>(g->ws);
    std::vector<int> g8, g4;  // by image rows per block row (2, 1)
    for (int i = 0; i < n; i++)
        (bh_of(descs[i]) == 2 ? g8 : g4).push_back(i);
    Img *dtab = reinterpret_cast<Img *>(base);
    st = upload_group_table(descs, g8, lays, offs, base, dtab);
    if (st == CCL_OK)
        st = upload_group_table(descs, g4, lays, offs, base, dtab + g8.size());
    hipStream_t cs = nullptr;
    if (st == CCL_OK && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
        st = CCL_ERR_HIP;
    if (st == CCL_OK) {
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            st = CCL_ERR_HIP;
        } else {
            int s1 = run_group(descs, g8, lays, offs, base, dtab, 2, c, cs, true);
            int s2 = s1 == CCL_OK ? run_group(descs, g4, lays, offs, base, dtab + g8.size(), 1, c, cs, true) : s1;
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(cs, &graph);
            st = s2 != CCL_OK ? s2 : (e == hipSuccess ? CCL_OK : CCL_ERR_HIP);
            g->graph = graph;
            if (st == CCL_OK && hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess)
                st = CCL_ERR_HIP;
        }
    }
    if (cs)
        (void)hipStreamDestroy(cs);
    if (st != CCL_OK) {
        ccl_graph_destroy(g);
        return st;
    }
    *out = g;
    return CCL_OK;
}

int ccl_graph_launch(ccl_graph *g, hipStream_t stream) {
    if (!g || !g->exec)
        return CCL_ERR_NULL;
    return hipGraphLaunch(g->exec, stream) == hipSuccess ? CCL_OK : CCL_ERR_HIP;
}

int ccl_graph_destroy(ccl_graph *g) {
    if (!g)
        return CCL_OK;
    int st = CCL_OK;
    if (g->exec && hipGraphExecDestroy(g->exec) != hipSuccess)
        st = CCL_ERR_HIP;
    if (g->graph && hipGraphDestroy(g->graph) != hipSuccess)
        st = CCL_ERR_HIP;
    if (g->ws) {
        if (hipDeviceSynchronize() != hipSuccess || hipFree(g->ws) != hipSuccess)
            st = CCL_ERR_HIP;
    }
    delete g;
    return st;
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

int ccl_profile(int enable) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = enable != 0;
    return CCL_OK;
}

int ccl_profile_read(double *ms, int nphase, int *ncalls) {
    if (!ms || nphase < 0)
        return CCL_ERR_NULL;
    std::vector<std::vector<hipEvent_t>> pend;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        pend.swap(g_prof_pending);
    }
    for (int i = 0; i < nphase; i++)
        ms[i] = 0.0;
    int st = CCL_OK, calls = 0;
    for (auto &ev : pend) {
        if (hipEventSynchronize(ev.back()) != hipSuccess)
            st = CCL_ERR_HIP;
        for (size_t i = 0; i + 1 < ev.size() && (int)i < nphase; i++) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) == hipSuccess)
                ms[i] += t;
            else
                st = CCL_ERR_HIP;
        }
        calls++;
    }
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        for (auto &ev : pend)
            for (hipEvent_t e : ev)
                g_prof_free.push_back(e);
    }
    if (ncalls)
        *ncalls = calls;
    return st;
}

int ccl_tile_count(void) { return kNumTiles; }

int ccl_tile_config(int id, int *tile_h, int *tile_w) {
    TileCfg c;
    int st = resolve_tile(id, &c);
    if (st != CCL_OK)
        return st;
    if (tile_h)
        *tile_h = c.nsr;
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
    case CCL_ERR_LEVEL: return "level must be in 0..255";
    case CCL_ERR_SCAN: return "unknown scan strategy";
    default: return "unknown status";
    }
}

}  // extern "C"
