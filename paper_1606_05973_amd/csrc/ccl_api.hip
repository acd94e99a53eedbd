// Host side of the gfx950 connected component labeling library: argument
// checks, workspace cache, launch sequence.  See include/ccl.h for the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_set>
#include <utility>
#include <vector>

#include "ccl.h"
#include "ccl_kernels.hpp"

namespace ccl {
namespace {

// Every path works on extended descriptors; ccl_label_batch widens its
// plain ones.
typedef ccl_image_desc_ex Desc;

// ---------------------------------------------------------------- tiles
// A tile configuration is (block rows, width).  The tile height is block
// rows x 2 under 8-connectivity with the row-pair scan (two image rows per
// block row), block rows x 1 with single rows, block rows / 2 for gray
// levels.
struct TileCfg {
    int nsr, tw;
};
constexpr TileCfg kTiles[] = {{32, 256}, {16, 256}, {16, 512}, {64, 128}, {32, 128}, {8, 512}, {64, 256}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

// Image rows per block row: two under 8-connectivity with the pair-row scan
// (the default), one otherwise.
inline int bh_of(int conn, int scan) { return (conn == 8 && scan == CCL_SCAN_PAIR) ? 2 : 1; }

// Kinds of image, each with kernels of its own: row-pair runs, single-row
// runs, gray levels.
enum Kind { kPair = 0, kRow = 1, kGray = 2, kKinds = 3 };
inline int kind_of(int conn, int scan, int gray) { return gray ? kGray : (bh_of(conn, scan) == 2 ? kPair : kRow); }
inline int kind_of(const Desc &d) { return kind_of(d.conn, d.scan, d.gray); }

// Default tile id per kind (fastest in a sweep of the configurations on
// 21568^2 images): row pairs 64x256 pixels, single rows 64x128, gray levels
// 32x256.
constexpr int kDefaultTile[kKinds] = {1, 4, 7};

// Tile configuration id (1-based) an image runs with: its descriptor's, else
// the call's, else its kind's default.
inline int tile_id_of(const Desc &d, int call_tile) {
    const int t = d.tile ? d.tile : call_tile;
    return t ? t : kDefaultTile[kind_of(d)];
}

// Labeling-pass store form an image allows: 16-byte stores need W % 4 == 0
// and 16-byte aligned labels; very wide rows need the any-width form.  A
// group takes the most general form any of its images needs.
int store_form(const Desc &d) {
    static_assert(kStoreAny < kStore4 && kStore4 < kStore16, "store forms ordered from the most general");
    if (d.W > kVecMaxW)
        return kStoreAny;
    if (d.W % 4 != 0 || (reinterpret_cast<uintptr_t>(d.labels) & 15u) != 0)
        return kStore4;
    return kStore16;
}

// Images of one kind, output order and tile configuration share every
// launch of a batch (one launch group).
struct GroupKey {
    int kind, order, tile;
    bool operator<(const GroupKey &o) const {
        return kind != o.kind ? kind < o.kind : (order != o.order ? order < o.order : tile < o.tile);
    }
};
inline GroupKey key_of(const Desc &d, int call_tile) { return {kind_of(d), d.order, tile_id_of(d, call_tile)}; }

// Inside a launch group the images are ordered by labeling-pass store form
// (16-byte, 4-byte, plain), so that each form's tiles form one range that a
// labeling-pass launch of that form covers.
constexpr int kForms = 3;
constexpr int kFormOrder[kForms] = {kStore16, kStore4, kStoreAny};
inline int form_rank(int form) { return form == kStore16 ? 0 : (form == kStore4 ? 1 : 2); }

size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// Workspace layout of one image (byte offsets from the image's base).
struct Layout {
    int32_t th, NTY, NTX, NT, nblk, nseg, nedge, nreg, nm, rcap, rw, cap, hep, vep;
    size_t masks, rt, cb, cf, tcnt, he, ve, uf, bval, bkey, seg, blk, bytes;
};

Layout layout_of(const Desc &d, const GroupKey &g) {
    const TileCfg &c = kTiles[g.tile - 1];
    const int64_t H = d.H, W = d.W;
    const bool gray = g.kind == kGray;
    Layout L{};
    // gray-level tiles hold half the rows (one per block row) so that every
    // pixel can be a node
    L.th = gray ? c.nsr / 2 : c.nsr * (g.kind == kPair ? 2 : 1);
    L.NTY = (int32_t)((H + L.th - 1) / L.th);
    L.NTX = (int32_t)((W + c.tw - 1) / c.tw);
    L.NT = L.NTY * L.NTX;
    L.nm = L.th * (c.tw / 32);
    L.rcap = c.nsr * (c.tw / 2);
    L.rw = L.rcap / 32;
    L.cap = 2 * (L.th + c.tw);
    // the rank scan runs over (row, tile column) segments, or over tiles in
    // provisional order
    const int64_t nseg = g.order == CCL_ORDER_PROVISIONAL ? (int64_t)L.NT : H * (int64_t)L.NTX;
    L.nseg = (int32_t)nseg;
    L.nblk = (int32_t)((nseg + kScanChunk - 1) / kScanChunk);
    L.nedge = (int32_t)((L.NTY - 1) * ((W + 31) / 32) + (L.NTX - 1) * ((H + 31) / 32));
    {
        const int rx = region_rx(c.tw, gray ? 0 : g.kind == kPair ? 2 : 1), ry = region_ry(L.th);
        L.nreg = ((L.NTY + ry - 1) / ry) * ((L.NTX + rx - 1) / rx);
    }
    const size_t NT = (size_t)L.NT;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L.masks = take(NT * L.nm * sizeof(uint32_t) * (gray ? 2 : 1));  // gray: foreground, then same-as-left
    L.rt = take(NT * L.rcap * sizeof(uint16_t));
    L.cb = take(NT * L.rw * sizeof(uint32_t));
    L.cf = take(NT * L.rcap * sizeof(int32_t));
    L.tcnt = take(NT * 4 * sizeof(int32_t));
    L.hep = (int32_t)((W + 31) / 32 * 32);
    L.vep = (int32_t)((H + 31) / 32 * 32);
    L.he = take((size_t)L.NTY * 2 * L.hep * sizeof(uint16_t));
    L.ve = take((size_t)L.NTX * 2 * L.vep * sizeof(uint16_t));
    L.uf = take(NT * L.cap * sizeof(uint64_t));
    L.bval = take(NT * L.cap * sizeof(int32_t));
    L.bkey = take(NT * L.cap * sizeof(uint16_t));
    L.seg = take((size_t)nseg * sizeof(int32_t));
    L.blk = take((size_t)L.nblk * sizeof(int32_t));
    L.bytes = off;
    return L;
}

// The global union-find addresses the boundary components as tile * CAP +
// index in 32 bits (and the kernels form that product in int32): images so
// elongated that their tiles' boundary slots reach 2^31 are refused.
bool fits_ids(const Layout &L) { return (int64_t)L.NT * L.cap < (int64_t)INT32_MAX; }

int check_image(const void *img, int64_t H, int64_t W, int64_t stride, int conn, const void *labels) {
    if (!img || !labels)
        return CCL_ERR_NULL;
    if (H <= 0 || W <= 0)
        return CCL_ERR_SHAPE;
    if (stride < W)
        return CCL_ERR_STRIDE;
    if (conn != 4 && conn != 8)
        return CCL_ERR_CONN;
    // (sides are rounded up to whole tiles and edge lines in int32)
    if (H >= (int64_t)INT32_MAX - 255 || W >= (int64_t)INT32_MAX - 255 || H * W >= (int64_t)INT32_MAX)
        return CCL_ERR_TOO_LARGE;
    return CCL_OK;
}

int check_level(int level) { return (level < 0 || level > 255) ? CCL_ERR_LEVEL : CCL_OK; }

int check_tile(int tile) { return (tile < 0 || tile > kNumTiles) ? CCL_ERR_TILE : CCL_OK; }

int check_opts(const Desc &d) {
    if (d.scan != CCL_SCAN_PAIR && d.scan != CCL_SCAN_ROW)
        return CCL_ERR_SCAN;
    if (d.gray != 0 && d.gray != 1)
        return CCL_ERR_GRAY;
    if (d.order != CCL_ORDER_CANONICAL && d.order != CCL_ORDER_PROVISIONAL)
        return CCL_ERR_ORDER;
    int st = check_tile(d.tile);
    return st != CCL_OK ? st : check_level(d.level);
}

int check_desc(const Desc &d) {
    const int st = check_image(d.img, d.H, d.W, d.stride, d.conn, d.labels);
    return st != CCL_OK ? st : check_opts(d);
}

// ------------------------------------------------------------- workspace
// Per (device, stream): the device workspace, and two pinned host buffers
// that stage batch tables (a copy from pinned memory is asynchronous; each
// buffer is rewritten only once its previous copy has run).
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
    char *stage[2] = {nullptr, nullptr};
    size_t stage_bytes[2] = {0, 0};
    hipEvent_t stage_done[2] = {nullptr, nullptr};
    int next_stage = 0;
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

// A pinned staging buffer of at least `need` bytes for a table copy on
// `stream` (not capturing), and the event to record after that copy.
int get_stage(hipStream_t stream, size_t need, char **out, hipEvent_t *done) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return CCL_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace &w = g_ws[{dev, stream}];
    const int i = w.next_stage;
    w.next_stage ^= 1;
    if (w.stage_done[i] && hipEventSynchronize(w.stage_done[i]) != hipSuccess)
        return CCL_ERR_HIP;
    if (!w.stage_done[i] && hipEventCreateWithFlags(&w.stage_done[i], hipEventDisableTiming) != hipSuccess)
        return CCL_ERR_HIP;
    if (w.stage_bytes[i] < need) {
        if (w.stage[i])
            (void)hipHostFree(w.stage[i]);
        w.stage[i] = nullptr;
        w.stage_bytes[i] = 0;
        const size_t grow = std::max(need, (size_t)64 << 10);
        if (hipHostMalloc(reinterpret_cast<void **>(&w.stage[i]), grow) != hipSuccess) {
            (void)hipGetLastError();
            return CCL_ERR_NOMEM;
        }
        w.stage_bytes[i] = grow;
    }
    *out = w.stage[i];
    *done = w.stage_done[i];
    return CCL_OK;
}

// ----------------------------------------------------- static scratch
// Workspace of ccl_label_noalloc: a file-scope device array, so that the
// call allocates nothing.  The loader gives every device the library runs on
// its own copy, held until the process ends.  In host code `scratch` names a
// host-side stand-in, not device memory: kernels get the device address that
// hipGetSymbolAddress reports, looked up once per device with that device
// current.  Every call on a device shares the array, so calls that overlap
// on one device race (calls on one stream are ordered by the stream).  No
// kernel relies on zeroed workspace (each writes what it later reads), so
// nothing is cleared between calls.
__device__ __align__(256) char scratch[CCL_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_at[kMaxDevices];  // device address of `scratch` per device, once looked up

int scratch_of_current_device(char **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return CCL_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices)
        return CCL_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_at[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return CCL_ERR_HIP;
        }
        g_scratch_at[dev] = p;
    }
    *out = static_cast<char *>(g_scratch_at[dev]);
    return CCL_OK;
}

void free_workspace(Workspace &w) {
    (void)hipFree(w.ptr);
    for (int i = 0; i < 2; i++) {
        if (w.stage[i])
            (void)hipHostFree(w.stage[i]);
        if (w.stage_done[i])
            (void)hipEventDestroy(w.stage_done[i]);
    }
}

// Sets a pointer field of an Img (whose device view is in the global
// address space) from a device address.
template <class P>
static void set_ptr(P &field, const void *p) {
    field = (P)(uintptr_t)p;
}

// Fill an Img from a descriptor, its layout and its workspace base.
Img make_img(const Desc &d, const Layout &L, char *base) {
    Img im{};
    set_ptr(im.img, d.img);
    set_ptr(im.labels, d.labels);
    set_ptr(im.ncomp, d.num_components);
    set_ptr(im.masks, base + L.masks);
    set_ptr(im.rt, base + L.rt);
    set_ptr(im.cb, base + L.cb);
    set_ptr(im.cf, base + L.cf);
    set_ptr(im.tcnt, base + L.tcnt);
    set_ptr(im.he, base + L.he);
    set_ptr(im.ve, base + L.ve);
    set_ptr(im.uf, base + L.uf);
    set_ptr(im.bval, base + L.bval);
    set_ptr(im.bkey, base + L.bkey);
    set_ptr(im.seg, base + L.seg);
    set_ptr(im.blk, base + L.blk);
    im.stride = d.stride;
    im.H = (int32_t)d.H;
    im.W = (int32_t)d.W;
    im.NTY = L.NTY;
    im.NTX = L.NTX;
    im.conn = d.conn;
    im.level = d.level;
    im.hep = L.hep;
    im.vep = L.vep;
    im.nblk = L.nblk;
    im.nseg = L.nseg;
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
    // allow = false: no events at all (the allocation-free entry point)
    PhaseMarks(hipStream_t st, bool allow) : s(st) {
        {
            std::lock_guard<std::mutex> lk(g_prof_mu);
            on = allow && g_prof_on;
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

template <int NSR, int TW, int BH, int ORD>
int launch_all(const Batch &b, int64_t tiles, const int64_t *form_tiles, int64_t edges, int64_t regions,
               int64_t blocks, int nimg,
               hipStream_t s, bool marks) {
    if (tiles > INT32_MAX || edges > INT32_MAX || blocks > INT32_MAX || regions > INT32_MAX)
        return CCL_ERR_TOO_LARGE;
    const dim3 blk(kThreads);
    const dim3 tile_groups((uint32_t)((tiles + kWaves - 1) / kWaves));
    PhaseMarks pm(s, marks);
    pm.mark();
    if constexpr (BH != 0) {
        // row pairs and single rows: the compact form, then the tiles with
        // more nodes than it holds (a grid of at least tiles / 64 groups)
        hipLaunchKernelGGL((k_tile_scan_c<NSR, TW, BH, ORD>), dim3((uint32_t)tiles), dim3(kScanThreadsC), 0, s, b);
        const int64_t rest = std::min<int64_t>(
            tiles, std::max<int64_t>(persistent_groups<k_tile_scan_rest<NSR, TW, BH, ORD>>(kTileThreads), (tiles + 63) / 64));
        hipLaunchKernelGGL((k_tile_scan_rest<NSR, TW, BH, ORD>), dim3((uint32_t)rest), dim3(kTileThreads), 0, s, b,
                           (int32_t)tiles);
    } else {
        hipLaunchKernelGGL((k_tile_scan<NSR, TW, BH, ORD>), dim3((uint32_t)tiles), dim3(kTileThreads), 0, s, b);
    }
    pm.mark();
    if (edges > 0) {
        hipLaunchKernelGGL((k_merge_local<NSR, TW, BH, ORD>), dim3((uint32_t)regions), blk, 0, s, b);
        hipLaunchKernelGGL((k_merge<NSR, TW, BH>), dim3((uint32_t)((merge_split(BH) * edges + kThreads - 1) / kThreads)),
                           blk, 0, s, b);
    }
    pm.mark();
    if (ORD == kCanonical)
        hipLaunchKernelGGL((k_flatten<NSR, TW, BH>), tile_groups, blk, 0, s, b, (int32_t)tiles);
    else
        hipLaunchKernelGGL((k_flatten_prov<NSR, TW, BH>), tile_groups, blk, 0, s, b, (int32_t)tiles);
    pm.mark();
    hipLaunchKernelGGL(k_scan_blocks, dim3((uint32_t)blocks), blk, 0, s, b);
    pm.mark();
    hipLaunchKernelGGL(k_scan_top, dim3((uint32_t)nimg), blk, 0, s, b);
    pm.mark();
    if (ORD == kCanonical)
        hipLaunchKernelGGL((k_comp_labels<NSR, TW, BH>), tile_groups, blk, 0, s, b, (int32_t)tiles);
    else
        hipLaunchKernelGGL((k_comp_labels_prov<NSR, TW, BH>), tile_groups, blk, 0, s, b, (int32_t)tiles);
    pm.mark();
    // one labeling-pass launch per store form, over that form's tile range
    int64_t tbeg = 0;
    for (int f = 0; f < kForms; f++) {
        const int64_t nt = form_tiles[f];
        if (nt <= 0)
            continue;
#define CCL_RELABEL(F_)                                                                                       \
    hipLaunchKernelGGL((k_relabel<NSR, TW, BH, F_>),                                                          \
                       dim3((uint32_t)std::min<int64_t>(nt, persistent_groups<k_relabel<NSR, TW, BH, F_>>(kTileThreads))), \
                       dim3(kTileThreads), 0, s, b, (int32_t)tbeg, (int32_t)nt)
        if (kFormOrder[f] == kStore16)
            CCL_RELABEL(kStore16);
        else if (kFormOrder[f] == kStore4)
            CCL_RELABEL(kStore4);
        else
            CCL_RELABEL(kStoreAny);
#undef CCL_RELABEL
        tbeg += nt;
    }
    pm.mark();
    return hipGetLastError() == hipSuccess ? CCL_OK : CCL_ERR_HIP;
}

int dispatch(const GroupKey &g, const Batch &b, int64_t tiles, const int64_t *form_tiles, int64_t edges,
             int64_t regions, int64_t blocks, int nimg, hipStream_t s, bool marks = true) {
    const TileCfg &c = kTiles[g.tile - 1];
#define CCL_ORD(N_, W_, B_) \
    (g.order == CCL_ORDER_PROVISIONAL ? launch_all<N_, W_, B_, kProvisional>(b, tiles, form_tiles, edges, regions, blocks, nimg, s, marks) \
                                      : launch_all<N_, W_, B_, kCanonical>(b, tiles, form_tiles, edges, regions, blocks, nimg, s, marks))
#define CCL_TILE_CASE(N_, W_)                                                                       \
    if (c.nsr == N_ && c.tw == W_)                                                                  \
        return g.kind == kPair ? CCL_ORD(N_, W_, 2) : g.kind == kRow ? CCL_ORD(N_, W_, 1) : CCL_ORD(N_, W_, 0);
    CCL_TILE_CASE(32, 256)
    CCL_TILE_CASE(16, 256)
    CCL_TILE_CASE(16, 512)
    CCL_TILE_CASE(64, 128)
    CCL_TILE_CASE(32, 128)
    CCL_TILE_CASE(8, 512)
    CCL_TILE_CASE(64, 256)
#undef CCL_TILE_CASE
#undef CCL_ORD
    return CCL_ERR_TILE;
}

// ------------------------------------------------------------- batches
// Table of a group of n images: n Img entries, then the n tile0, n edge0,
// n scan0 and n region0 keys as a compact array (searched by find_img).
size_t group_table_bytes(size_t n) { return align_up(n * (sizeof(Img) + 4 * sizeof(int32_t))); }

// The most table bytes a batch of n images can need (every image a group of
// its own at worst).
size_t max_tables_bytes(size_t n) { return n * group_table_bytes(1); }
static_assert(sizeof(Img) + 4 * sizeof(int32_t) <= 256, "a group's table takes at most 256 bytes per image");

// The layout of a batch's workspace: the tables of its launch groups (in
// key order), then one region per image.
struct Plan {
    std::vector<GroupKey> keys;
    std::vector<std::vector<int>> members;
    std::vector<size_t> tab_at;       // table offset of each group
    std::vector<Layout> lays;         // per image
    std::vector<size_t> offs;         // region offset of each image
    size_t tables = 0, bytes = 0;
    bool upload = false;              // some group has more than one image (needs its table on the device)
    bool fits = true;                 // every image's boundary slots fit 32-bit ids (fits_ids)
};

Plan plan_batch(const Desc *descs, int n, int call_tile) {
    Plan P;
    std::map<GroupKey, std::vector<int>> by;
    for (int i = 0; i < n; i++)
        by[key_of(descs[i], call_tile)].push_back(i);
    for (auto &kv : by)
        std::stable_sort(kv.second.begin(), kv.second.end(),
                         [&](int a, int c) { return form_rank(store_form(descs[a])) < form_rank(store_form(descs[c])); });
    for (auto &kv : by) {
        P.keys.push_back(kv.first);
        P.tab_at.push_back(P.tables);
        P.tables += group_table_bytes(kv.second.size());
        P.upload |= kv.second.size() > 1;
        P.members.push_back(std::move(kv.second));
    }
    size_t off = P.tables;
    P.lays.resize(n);
    P.offs.resize(n);
    for (int i = 0; i < n; i++) {
        P.lays[i] = layout_of(descs[i], key_of(descs[i], call_tile));
        P.fits &= fits_ids(P.lays[i]);
        P.offs[i] = off;
        off += P.lays[i].bytes;
    }
    P.bytes = off;
    return P;
}

size_t batch_bytes(const Desc *descs, int n, int call_tile) { return plan_batch(descs, n, call_tile).bytes; }

// One group's launch arguments, its table written to `tab_bytes` (host).
struct GroupRun {
    Batch b;
    int64_t tiles, edges, regions, blocks;
    int64_t form_tiles[kForms];   // tiles of the 16-byte, 4-byte and plain-store images, in that order
};

int build_group(const Desc *descs, const Plan &P, size_t g, char *base, char *tab_bytes, GroupRun *out) {
    const std::vector<int> &idx = P.members[g];
    const int n = (int)idx.size();
    Img *tab = reinterpret_cast<Img *>(tab_bytes);
    int32_t *keys = reinterpret_cast<int32_t *>(tab_bytes + (size_t)n * sizeof(Img));
    int64_t tiles = 0, edges = 0, regions = 0, blocks = 0;
    Batch b{};
    b.n = n;
    int64_t form_tiles[kForms] = {0, 0, 0};
    for (int k = 0; k < n; k++) {
        const int i = idx[k];
        const Desc &d = descs[i];
        tab[k] = make_img(d, P.lays[i], base + P.offs[i]);
        tab[k].tile0 = (int32_t)tiles;
        tab[k].edge0 = (int32_t)edges;
        tab[k].scan0 = (int32_t)blocks;
        tab[k].region0 = (int32_t)regions;
        keys[k] = tab[k].tile0;
        keys[n + k] = tab[k].edge0;
        keys[2 * n + k] = tab[k].scan0;
        keys[3 * n + k] = tab[k].region0;
        tiles += P.lays[i].NT;
        edges += P.lays[i].nedge;
        regions += P.lays[i].nreg;
        blocks += P.lays[i].nblk;
        if (tiles > INT32_MAX || edges > INT32_MAX || blocks > INT32_MAX || regions > INT32_MAX)
            return CCL_ERR_TOO_LARGE;
        form_tiles[form_rank(store_form(d))] += P.lays[i].NT;
    }
    if (n == 1) {
        b.one = tab[0];
    } else {
        b.tab = reinterpret_cast<const Img *>(base + P.tab_at[g]);
        b.keys = reinterpret_cast<const int32_t *>(base + P.tab_at[g] + (size_t)n * sizeof(Img));
    }
    out->b = b;
    for (int f = 0; f < kForms; f++)
        out->form_tiles[f] = form_tiles[f];
    out->tiles = tiles;
    out->edges = edges;
    out->regions = regions;
    out->blocks = blocks;
    return CCL_OK;
}

// Builds every group's table into `host` (P.tables bytes, laid out as the
// start of the workspace) and the launch arguments.
int build_plan(const Desc *descs, const Plan &P, char *base, char *host, std::vector<GroupRun> *runs) {
    runs->resize(P.keys.size());
    for (size_t g = 0; g < P.keys.size(); g++) {
        const int st = build_group(descs, P, g, base, host + P.tab_at[g], &(*runs)[g]);
        if (st != CCL_OK)
            return st;
    }
    return CCL_OK;
}

int launch_plan(const Plan &P, const std::vector<GroupRun> &runs, hipStream_t stream) {
    for (size_t g = 0; g < P.keys.size(); g++) {
        const int st = dispatch(P.keys[g], runs[g].b, runs[g].tiles, runs[g].form_tiles, runs[g].edges,
                                runs[g].regions, runs[g].blocks, (int)P.members[g].size(), stream);
        if (st != CCL_OK)
            return st;
    }
    return CCL_OK;
}

// The tables of a stream being captured: stored by k_put_words launches that
// carry them in their arguments, so that every replay writes them again
// (a copy node would keep a pointer to host memory that does not outlive
// the call).
int put_tables_captured(char *dst, const char *host, size_t bytes, hipStream_t stream) {
    static_assert(sizeof(WordChunk) == 4 * kChunkWords, "chunk layout");
    const size_t words = bytes / 4;   // table sizes are multiples of 256
    for (size_t at = 0; at < words; at += kChunkWords) {
        WordChunk ch;
        const int cnt = (int)std::min<size_t>(kChunkWords, words - at);
        memcpy(ch.w, host + 4 * at, 4 * (size_t)cnt);
        hipLaunchKernelGGL(k_put_words, dim3(1), dim3(kChunkWords), 0, stream, reinterpret_cast<uint32_t *>(dst) + at,
                           cnt, ch);
    }
    return hipGetLastError() == hipSuccess ? CCL_OK : CCL_ERR_HIP;
}

// Launch a batch into a workspace of at least P.bytes bytes.  The tables go
// through `htab` (pinned host memory of at least P.tables bytes that stays
// untouched until the stream has passed the copy) when given, else through
// the stream's staging buffers, or kernel arguments while capturing.
int run_plan_in(const Desc *descs, const Plan &P, hipStream_t stream, char *base, char *htab = nullptr) {
    std::vector<GroupRun> runs;
    if (!P.upload) {
        std::vector<char> local(P.tables);
        const int st = build_plan(descs, P, base, local.data(), &runs);
        return st != CCL_OK ? st : launch_plan(P, runs, stream);
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess)
        return CCL_ERR_HIP;
    if (cs != hipStreamCaptureStatusNone) {
        std::vector<char> local(P.tables);
        int st = build_plan(descs, P, base, local.data(), &runs);
        if (st == CCL_OK)
            st = put_tables_captured(base, local.data(), P.tables, stream);
        return st != CCL_OK ? st : launch_plan(P, runs, stream);
    }
    hipEvent_t done = nullptr;
    char *host = htab;
    if (!host) {
        const int st = get_stage(stream, P.tables, &host, &done);
        if (st != CCL_OK)
            return st;
    }
    int st = build_plan(descs, P, base, host, &runs);
    if (st != CCL_OK)
        return st;
    if (hipMemcpyAsync(base, host, P.tables, hipMemcpyHostToDevice, stream) != hipSuccess ||
        (done && hipEventRecord(done, stream) != hipSuccess))
        return CCL_ERR_HIP;
    return launch_plan(P, runs, stream);
}

int run_batch(const Desc *descs, int n, int call_tile, hipStream_t stream) {
    const Plan P = plan_batch(descs, n, call_tile);
    if (!P.fits)
        return CCL_ERR_TOO_LARGE;
    void *ws = nullptr;
    const int st = get_workspace(stream, P.bytes, &ws);
    if (st != CCL_OK)
        return st;
    return run_plan_in(descs, P, stream, static_cast<char *>(ws));
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
    Desc d{img, H, W, stride, conn, labels, num_components, level, CCL_SCAN_PAIR, 0, CCL_ORDER_CANONICAL, tile};
    const int st = check_desc(d);
    return st != CCL_OK ? st : run_batch(&d, 1, 0, stream);
}

int ccl_label_gray(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int level, int conn,
                   int32_t *labels, int32_t *num_components, int tile, hipStream_t stream) {
    Desc d{img, H, W, stride, conn, labels, num_components, level, CCL_SCAN_ROW, 1, CCL_ORDER_CANONICAL, tile};
    const int st = check_desc(d);
    return st != CCL_OK ? st : run_batch(&d, 1, 0, stream);
}

int ccl_label_provisional(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn, int32_t *labels,
                          int32_t *num_components, int tile, hipStream_t stream) {
    Desc d{img, H, W, stride, conn, labels, num_components, 0, CCL_SCAN_PAIR, 0, CCL_ORDER_PROVISIONAL, tile};
    const int st = check_desc(d);
    return st != CCL_OK ? st : run_batch(&d, 1, 0, stream);
}

int ccl_label_ex(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn, int32_t *labels,
                 int32_t *num_components, int tile, hipStream_t stream) {
    return ccl_label_level(img, H, W, stride, 0, conn, labels, num_components, tile, stream);
}

int ccl_label(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn, int32_t *labels,
              hipStream_t stream) {
    return ccl_label_ex(img, H, W, stride, conn, labels, nullptr, 0, stream);
}

int ccl_label_noalloc(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn, int32_t *labels,
                      int32_t *num_components, hipStream_t stream) {
    const Desc d{img, H, W, stride, conn, labels, num_components, 0, CCL_SCAN_PAIR, 0, CCL_ORDER_CANONICAL, 0};
    int st = check_desc(d);
    if (st != CCL_OK)
        return st;
    // the same layout as a ccl_label call: one image region after a table
    // slot, so that ccl_workspace_bytes states what the call needs
    const GroupKey g = key_of(d, 0);
    const Layout L = layout_of(d, g);
    if (!fits_ids(L))
        return CCL_ERR_TOO_LARGE;
    const size_t at = group_table_bytes(1);
    if (at + L.bytes > (size_t)CCL_NOALLOC_SCRATCH_BYTES)
        return CCL_ERR_SCRATCH;
    char *base = nullptr;
    if ((st = scratch_of_current_device(&base)) != CCL_OK)
        return st;
    // a single image travels in the kernel arguments (no table upload)
    Batch b{};
    b.n = 1;
    b.one = make_img(d, L, base + at);
    int64_t form_tiles[kForms] = {0, 0, 0};
    form_tiles[form_rank(store_form(d))] = L.NT;
    return dispatch(g, b, L.NT, form_tiles, L.nedge, L.nreg, L.nblk, 1, stream, false);
}

int ccl_label_batch_ex(const ccl_image_desc_ex *descs, int n, int tile, hipStream_t stream) {
    if (n < 0 || (n > 0 && !descs))
        return CCL_ERR_BATCH;
    int st = check_tile(tile);
    if (st != CCL_OK)
        return st;
    if (n == 0)
        return CCL_OK;
    for (int i = 0; i < n; i++)
        if ((st = check_desc(descs[i])) != CCL_OK)
            return st;
    return run_batch(descs, n, tile, stream);
}

int ccl_label_batch(const ccl_image_desc *descs, int n, hipStream_t stream) {
    if (n < 0 || (n > 0 && !descs))
        return CCL_ERR_BATCH;
    std::vector<Desc> ex((size_t)n);
    for (int i = 0; i < n; i++) {
        const ccl_image_desc &d = descs[i];
        ex[i] = Desc{d.img, d.H, d.W, d.stride, d.conn, d.labels, d.num_components, 0, CCL_SCAN_PAIR, 0,
                     CCL_ORDER_CANONICAL, 0};
    }
    return ccl_label_batch_ex(ex.data(), n, 0, stream);
}

size_t ccl_workspace_bytes(int64_t H, int64_t W, int conn) {
    int8_t dummy;
    Desc d{reinterpret_cast<const uint8_t *>(&dummy), H, W, W, conn, reinterpret_cast<int32_t *>(&dummy), nullptr,
           0, CCL_SCAN_PAIR, 0, CCL_ORDER_CANONICAL, 0};
    if (check_desc(d) != CCL_OK)
        return 0;
    return batch_bytes(&d, 1, 0);
}

size_t ccl_batch_workspace_bytes(const ccl_image_desc_ex *descs, int n, int tile) {
    if (check_tile(tile) != CCL_OK || n < 0 || (n > 0 && !descs))
        return 0;
    int8_t dummy;
    std::vector<Desc> v(descs, descs + n);
    for (Desc &d : v) {
        // the buffers are not used: only the shapes and options count
        d.img = reinterpret_cast<const uint8_t *>(&dummy);
        d.labels = reinterpret_cast<int32_t *>(&dummy);
        if (check_desc(d) != CCL_OK)
            return 0;
    }
    return batch_bytes(v.data(), n, tile);
}

int ccl_batch_graph_create(const ccl_image_desc_ex *descs, int n, int tile, ccl_graph **out) {
    if (!out)
        return CCL_ERR_NULL;
    *out = nullptr;
    if (n <= 0 || !descs)
        return CCL_ERR_BATCH;
    int st = check_tile(tile);
    if (st != CCL_OK)
        return st;
    for (int i = 0; i < n; i++)
        if ((st = check_desc(descs[i])) != CCL_OK)
            return st;
    const Plan P = plan_batch(descs, n, tile);
    if (!P.fits)
        return CCL_ERR_TOO_LARGE;
    ccl_graph *g = new ccl_graph();
    if (hipMalloc(&g->ws, P.bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete g;
        return CCL_ERR_NOMEM;
    }
    char *base = static_cast<char *>(g->ws);
    // the tables go to the graph's own workspace once, before capture: the
    // graph holds kernel nodes only
    std::vector<char> host(P.tables);
    std::vector<GroupRun> runs;
    st = build_plan(descs, P, base, host.data(), &runs);
    if (st == CCL_OK && hipMemcpy(base, host.data(), P.tables, hipMemcpyHostToDevice) != hipSuccess)
        st = CCL_ERR_HIP;
    hipStream_t cs = nullptr;
    if (st == CCL_OK && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
        st = CCL_ERR_HIP;
    if (st == CCL_OK) {
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            st = CCL_ERR_HIP;
        } else {
            const int s2 = launch_plan(P, runs, cs);
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
            free_workspace(it->second);
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

int ccl_tile_default(int conn, int scan, int gray) {
    if ((conn != 4 && conn != 8) || (scan != CCL_SCAN_PAIR && scan != CCL_SCAN_ROW) || (gray != 0 && gray != 1))
        return 0;
    return kDefaultTile[kind_of(conn, scan, gray)];
}

int ccl_tile_config(int id, int *tile_h, int *tile_w) {
    if (check_tile(id) != CCL_OK)
        return CCL_ERR_TILE;
    const TileCfg &c = kTiles[(id ? id : 1) - 1];
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
    case CCL_ERR_TOO_LARGE: return "image too large: H*W must be below 2^31-1, each side below 2^31-256, and the tiles' boundary slots below 2^31";
    case CCL_ERR_NOMEM: return "workspace allocation failed";
    case CCL_ERR_HIP: return "HIP runtime call or kernel launch failed";
    case CCL_ERR_TILE: return "unknown tile configuration";
    case CCL_ERR_CAPTURE: return "workspace cannot grow while the stream is being captured (call ccl_reserve first)";
    case CCL_ERR_BATCH: return "invalid batch (n < 0 or descs NULL)";
    case CCL_ERR_LEVEL: return "level must be in 0..255";
    case CCL_ERR_SCAN: return "unknown scan strategy";
    case CCL_ERR_BUDGET: return "request needs more workspace than a server slot holds";
    case CCL_ERR_TICKET: return "unknown server ticket";
    case CCL_ERR_GRAY: return "gray must be 0 or 1";
    case CCL_ERR_ORDER: return "unknown output order";
    case CCL_ERR_SCRATCH: return "image needs more workspace than the static scratch of ccl_label_noalloc holds";
    default: return "unknown status";
    }
}

}  // extern "C"

// ---------------------------------------------------------------- server
// Continuous batching (see ccl_server_create in ccl.h).  One scheduler
// thread per server owns the slots; submitters only touch the queue.
namespace ccl {
namespace {

using Clock = std::chrono::steady_clock;

struct ServerReq {
    ccl::Desc d;
    uint64_t ticket;
    hipEvent_t ready;      // recorded on the submitter's stream, or NULL
    size_t bytes;          // this image's workspace region
    Clock::time_point t_submit;
};

struct ServerSlot {
    hipStream_t stream = nullptr;
    char *ws = nullptr;      // device workspace of ws_bytes
    char *htab = nullptr;    // pinned host image tables (for up to max_batch images)
    hipEvent_t done = nullptr;
    std::vector<ServerReq> batch;
    bool busy = false;
};

}  // namespace
}  // namespace ccl

struct ccl_server {
    int dev = 0;
    ccl_server_config cfg{};
    int tile = 0;                    // tile id of images whose descriptor names none
    size_t ws_bytes = 0;
    std::vector<ccl::ServerSlot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<ccl::ServerReq> pending;
    std::unordered_set<uint64_t> outstanding;
    std::vector<double> lat_ms;      // by ticket - 1; < 0 while not done
    std::vector<hipEvent_t> ev_free;
    uint64_t next_ticket = 1;
    int64_t rejected = 0, batches = 0, in_flight_max = 0, completed = 0;
    double px_done = 0;
    bool stop = false;
    int error = CCL_OK;              // first HIP failure seen by the scheduler
    std::thread th;

    size_t bytes_of(const ccl::Desc &d) const { return ccl::layout_of(d, ccl::key_of(d, tile)).bytes; }

    void finish(ccl::ServerSlot &sl, Clock::time_point now) {
        for (auto &r : sl.batch) {
            lat_ms[r.ticket - 1] = std::chrono::duration<double, std::milli>(now - r.t_submit).count();
            outstanding.erase(r.ticket);
            px_done += (double)r.d.H * (double)r.d.W;
            completed++;
            if (r.ready)
                ev_free.push_back(r.ready);
        }
        sl.batch.clear();
        sl.busy = false;
    }

    // Take the longest queue prefix that fits one slot.  The footprint of a
    // candidate batch is what plan_batch lays out in the slot's workspace:
    // the table of every launch group, then the image regions.
    std::vector<ccl::ServerReq> take_batch() {
        std::vector<ccl::ServerReq> b;
        std::map<ccl::GroupKey, size_t> members;
        size_t used = 0, tables = 0;
        int64_t px = 0;
        while (!pending.empty() && (int)b.size() < cfg.max_batch) {
            const ccl::ServerReq &r = pending.front();
            const int64_t n = r.d.H * r.d.W;
            const ccl::GroupKey g = ccl::key_of(r.d, tile);
            const size_t m = members.count(g) ? members[g] : 0;
            const size_t tables2 = tables - ccl::group_table_bytes(m) + ccl::group_table_bytes(m + 1);
            if (!b.empty() && (px + n > cfg.max_batch_pixels || tables2 + used + r.bytes > ws_bytes))
                break;
            members[g] = m + 1;
            tables = tables2;
            used += r.bytes;
            px += n;
            b.push_back(r);
            pending.pop_front();
        }
        return b;
    }

    void loop() {
        (void)hipSetDevice(dev);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            int busy = 0;
            for (auto &sl : slots) {
                if (!sl.busy)
                    continue;
                const hipError_t q = hipEventQuery(sl.done);
                if (q == hipSuccess) {
                    finish(sl, Clock::now());
                    cv_done.notify_all();
                } else if (q != hipErrorNotReady) {
                    if (error == CCL_OK)
                        error = CCL_ERR_HIP;
                    finish(sl, Clock::now());
                    cv_done.notify_all();
                } else {
                    busy++;
                }
            }
            for (auto &sl : slots) {
                if (sl.busy || pending.empty())
                    continue;
                std::vector<ccl::ServerReq> b = take_batch();
                lk.unlock();
                std::vector<ccl::Desc> descs;
                int st = CCL_OK;
                for (auto &r : b) {
                    descs.push_back(r.d);
                    if (r.ready && hipStreamWaitEvent(sl.stream, r.ready, 0) != hipSuccess)
                        st = CCL_ERR_HIP;
                }
                if (st == CCL_OK) {
                    const ccl::Plan P = ccl::plan_batch(descs.data(), (int)descs.size(), tile);
                    st = ccl::run_plan_in(descs.data(), P, sl.stream, sl.ws, sl.htab);
                }
                if (st == CCL_OK && hipEventRecord(sl.done, sl.stream) != hipSuccess)
                    st = CCL_ERR_HIP;
                lk.lock();
                sl.batch = std::move(b);
                sl.busy = true;
                batches++;
                if (st != CCL_OK) {
                    if (error == CCL_OK)
                        error = st;
                    finish(sl, Clock::now());
                    cv_done.notify_all();
                    continue;
                }
                busy++;
                in_flight_max = std::max<int64_t>(in_flight_max, busy);
            }
            if (stop && pending.empty() && busy == 0)
                return;
            if (busy)
                cv_work.wait_for(lk, std::chrono::microseconds(20));
            else
                cv_work.wait(lk, [&] { return stop || !pending.empty(); });
        }
    }
};

extern "C" {

int ccl_server_create(const ccl_server_config *cfg, ccl_server **out) {
    if (!cfg || !out)
        return CCL_ERR_NULL;
    *out = nullptr;
    if (cfg->n_streams < 1 || cfg->max_batch < 1 || cfg->max_batch_pixels < 1 || cfg->hbm_budget == 0)
        return CCL_ERR_BATCH;
    int st = ccl::check_tile(cfg->tile);
    if (st != CCL_OK)
        return st;
    ccl_server *s = new ccl_server();
    s->cfg = *cfg;
    s->tile = cfg->tile;
    s->ws_bytes = cfg->hbm_budget / (size_t)cfg->n_streams;
    if (hipGetDevice(&s->dev) != hipSuccess) {
        delete s;
        return CCL_ERR_HIP;
    }
    s->slots.resize(cfg->n_streams);
    for (auto &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&sl.htab),
                          ccl::max_tables_bytes(cfg->max_batch)) != hipSuccess)
            st = CCL_ERR_HIP;
        else if (hipMalloc(reinterpret_cast<void **>(&sl.ws), s->ws_bytes) != hipSuccess)
            st = CCL_ERR_NOMEM;
        if (st != CCL_OK)
            break;
    }
    if (st != CCL_OK) {
        (void)hipGetLastError();
        for (auto &sl : s->slots) {
            if (sl.ws) (void)hipFree(sl.ws);
            if (sl.htab) (void)hipHostFree(sl.htab);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        delete s;
        return st;
    }
    s->th = std::thread([s] { s->loop(); });
    *out = s;
    return CCL_OK;
}

int ccl_server_submit(ccl_server *s, const ccl_image_desc_ex *d, hipStream_t ready, uint64_t *ticket) {
    if (!s || !d || !ticket)
        return CCL_ERR_NULL;
    const int st = ccl::check_desc(*d);
    if (st != CCL_OK)
        return st;
    if (!ccl::fits_ids(ccl::layout_of(*d, ccl::key_of(*d, s->tile))))
        return CCL_ERR_TOO_LARGE;
    ccl::ServerReq r{};
    r.d = *d;
    r.bytes = s->bytes_of(*d);
    if (ccl::group_table_bytes(1) + r.bytes > s->ws_bytes) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->rejected++;
        return CCL_ERR_BUDGET;
    }
    r.ready = nullptr;
    if (ready) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (!s->ev_free.empty()) {
                r.ready = s->ev_free.back();
                s->ev_free.pop_back();
            }
        }
        if (!r.ready && hipEventCreateWithFlags(&r.ready, hipEventDisableTiming) != hipSuccess)
            return CCL_ERR_HIP;
        if (hipEventRecord(r.ready, ready) != hipSuccess) {
            (void)hipEventDestroy(r.ready);
            return CCL_ERR_HIP;
        }
    }
    r.t_submit = ccl::Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            if (r.ready)
                s->ev_free.push_back(r.ready);
            return CCL_ERR_BATCH;
        }
        r.ticket = s->next_ticket++;
        s->lat_ms.push_back(-1.0);
        s->outstanding.insert(r.ticket);
        s->pending.push_back(r);
        *ticket = r.ticket;
    }
    s->cv_work.notify_one();
    return CCL_OK;
}

int ccl_server_poll(ccl_server *s, uint64_t ticket, double *latency_ms) {
    if (!s)
        return CCL_ERR_NULL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (ticket == 0 || ticket >= s->next_ticket)
        return CCL_ERR_TICKET;
    if (s->outstanding.count(ticket))
        return 0;
    if (latency_ms)
        *latency_ms = s->lat_ms[ticket - 1];
    return 1;
}

int ccl_server_wait(ccl_server *s, uint64_t ticket, double *latency_ms) {
    if (!s)
        return CCL_ERR_NULL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (ticket == 0 || ticket >= s->next_ticket)
        return CCL_ERR_TICKET;
    s->cv_done.wait(lk, [&] { return !s->outstanding.count(ticket); });
    if (latency_ms)
        *latency_ms = s->lat_ms[ticket - 1];
    return s->error;
}

int ccl_server_drain(ccl_server *s) {
    if (!s)
        return CCL_ERR_NULL;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->outstanding.empty(); });
    return s->error;
}

int ccl_server_stats_get(ccl_server *s, ccl_server_stats *out) {
    if (!s || !out)
        return CCL_ERR_NULL;
    std::vector<double> lat;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        out->submitted = (int64_t)(s->next_ticket - 1);
        out->completed = s->completed;
        out->rejected = s->rejected;
        out->batches = s->batches;
        out->in_flight_max = s->in_flight_max;
        out->pixels_completed = s->px_done;
        for (double v : s->lat_ms)
            if (v >= 0)
                lat.push_back(v);
    }
    out->p50_ms = out->p99_ms = out->mean_ms = 0;
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        const size_t n = lat.size();
        out->p50_ms = lat[std::min(n - 1, (size_t)(0.50 * n))];
        out->p99_ms = lat[std::min(n - 1, (size_t)(0.99 * n))];
        double sum = 0;
        for (double v : lat)
            sum += v;
        out->mean_ms = sum / (double)n;
    }
    return s->error;
}

int ccl_server_destroy(ccl_server *s) {
    if (!s)
        return CCL_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->th.joinable())
        s->th.join();
    const int err = s->error;
    for (auto &sl : s->slots) {
        (void)hipStreamSynchronize(sl.stream);
        (void)hipFree(sl.ws);
        (void)hipHostFree(sl.htab);
        (void)hipEventDestroy(sl.done);
        (void)hipStreamDestroy(sl.stream);
    }
    for (hipEvent_t e : s->ev_free)
        (void)hipEventDestroy(e);
    delete s;
    return err;
}

}  // extern "C"
