// Device side of the gfx950 two-pass connected component labeling library.
//
// Method (Gupta et al., arXiv 1606.05973, Sections III-IV), re-designed for
// one MI355X:
//   * the image is cut into tiles; one workgroup scans one tile (the local
//     phase of PARemSP, Algorithm 7, with 2-D tiles instead of row chunks);
//   * the scan works on runs held as 32-bit foreground masks.  Under
//     8-connectivity it takes two rows at a time, as ARemSP does with the
//     mask of Fig. 1b: in a pair of rows every maximal stretch of columns
//     holding a foreground pixel (a block run) is one connected set, so it is
//     one union-find node.  Under 4-connectivity a node is a row run;
//   * nodes are numbered in raster order of their start; every pair of
//     nodes in consecutive block rows that touch is united once with Rem's
//     union with splicing (Algorithm 2) on an LDS parent array, all lanes
//     at once, the root link being a compare-and-swap as in the concurrent
//     merger (Algorithm 8, locks replaced by CAS);
//   * flatten (Algorithm 3's role) resolves every node; the tile then stores
//     a node -> local component table, the canonical key of each local
//     component (its first pixel in raster order), its foreground bitmask,
//     the component of every tile-edge pixel, and per-row counts of the
//     components that do not touch a shared tile edge;
//   * a second kernel unites components across tile edges (Algorithm 7's
//     boundary loop) with the same CAS-based RemSP on a compact global
//     array whose entries pack (canonical key of parent, parent id), so the
//     root of every set is its component's first raster pixel;
//   * components are ranked by that pixel through counts per (image row,
//     tile column) segment and a device exclusive scan;
//   * the labeling pass (second pass) streams the tile's bitmask and tables
//     and writes every int32 label once.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccl {

constexpr int kThreads = 256;       // threads per workgroup of the small kernels (4 wave64)
constexpr int kWaves = kThreads / 64;  // tiles per workgroup where one wave handles a tile
constexpr int kTileThreads = 512;   // threads per workgroup of the tile scan and labeling pass (8 wave64)
constexpr uint16_t kNone = 0xFFFFu;  // background pixel in the edge buffers
constexpr int kScanChunk = 1024;     // segment counts per scan block (256 x 4)

// Per-image description used by every kernel.  img / labels / ncomp belong
// to the caller, the rest lives in the library workspace.  NT = NTY * NTX
// tiles; RCAP, RW, CAP and NM are per-tile capacities fixed by the tile
// shape (see Geo).
// In the device pass the data pointers are typed as global-address-space
// pointers (they all address device memory), so that the compiler emits
// global rather than flat instructions: a flat access also counts in the LDS
// wait counter, and every LDS wait would then wait for the stores in flight.
// The host pass sees plain pointers of the same size and layout.
#if defined(__HIP_DEVICE_COMPILE__)
#define CCL_GLOBAL __attribute__((address_space(1)))
#else
#define CCL_GLOBAL
#endif
struct Img {
    CCL_GLOBAL const uint8_t *img;   // H rows, pitch `stride` bytes
    CCL_GLOBAL int32_t *labels;      // H x W, pitch W
    CCL_GLOBAL int32_t *ncomp;       // optional K output (device)
    CCL_GLOBAL uint32_t *masks;      // [NT][NM]    foreground bitmask of each tile
    CCL_GLOBAL uint16_t *rt;         // [NT][RCAP]  local component of each node
    CCL_GLOBAL uint32_t *cb;         // [NT][RW]    local component touches a shared tile edge (bit)
    CCL_GLOBAL int32_t *cf;          // [NT][RCAP]  canonical key (local pixel index) of each local
                                     //             component, replaced by its final label by the
                                     //             component-label kernel
    CCL_GLOBAL int32_t *tcnt;        // [NT][4]     nodes, components, boundary components
    CCL_GLOBAL uint16_t *he;         // [NTY][2][hep] boundary index of each top(0)/bottom(1) tile-row pixel
    CCL_GLOBAL uint16_t *ve;         // [NTX][2][vep] same for the left(0)/right(1) tile columns
    CCL_GLOBAL uint64_t *uf;         // [NT][CAP]   global union-find: (key of parent << 32) | parent id
    CCL_GLOBAL int32_t *bval;        // [NT][CAP]   interior roots before it in its row -> offset -> final label
    CCL_GLOBAL uint16_t *bkey;       // [NT][CAP]   canonical key of boundary component j
    CCL_GLOBAL int32_t *seg;         // [nseg]      canonical order: roots per (row, tile column) segment,
                                     //             [H][NTX]; provisional order: roots per tile, [NT];
                                     //             then their exclusive scan
    CCL_GLOBAL int32_t *blk;         // [nblk]      scan block totals -> exclusive scan
    int64_t stride;
    int32_t H, W, NTY, NTX, conn;
    int32_t level;        // foreground iff byte > level (0..255; 0 = nonzero)
    int32_t hep, vep;     // edge line pitches: W and H rounded up to 32 entries (64-byte lines)
    int32_t tile0;        // first tile of this image in a batch-wide tile numbering
    int32_t edge0;        // first edge segment (global merge pass, K2b)
    int32_t scan0;        // first scan block
    int32_t region0;      // first region (regional merge pass, K2a)
    int32_t nblk;
    int32_t nseg;         // entries of seg
};

// Output numbering (the ccl_order values): components ranked by smallest
// raster index, or numbered in the order of their smallest provisional label
// (tile, then component within the tile).
enum Order { kCanonical = 0, kProvisional = 1 };

struct Batch {
    const Img *tab;         // device table of n images (n > 1)
    const int32_t *keys;    // n tile0, then n edge0, then n scan0 of the table (n > 1)
    Img one;                // the image when n == 1
    int32_t n;
};
constexpr int32_t kVecMaxW = 1 << 22;  // keeps a tile's row offsets in bytes below 2^31

enum Key { kTile = 0, kEdge = 1, kScan = 2, kRegion = 3 };

// Image owning global work item `item` (binary search over the start keys).
// Returned by value: the table is read through the constant address space
// (it is written by the host before the launch and never by a kernel), so
// the fields arrive by scalar loads, not vector loads that would be counted
// together with the kernel's own stores.
typedef __attribute__((address_space(4))) const Img ConstImg;

// The search runs over a compact array of start keys, whose few cache lines
// stay in the scalar cache.
__device__ __forceinline__ Img find_img(const Batch &b, int32_t item, int which) {
    if (b.n == 1)
        return b.one;
    const ConstImg *tab = (const ConstImg *)(uintptr_t)b.tab;
    typedef __attribute__((address_space(4))) const int32_t ConstKey;
    const ConstKey *key = (const ConstKey *)(uintptr_t)(b.keys + (int64_t)which * b.n);
    int lo = 0, hi = b.n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (key[mid] <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    static_assert(sizeof(Img) % 4 == 0, "image descriptor copied as words");
    typedef __attribute__((address_space(4))) const uint32_t ConstWord;
    const ConstWord *src = (const ConstWord *)(tab + lo);
    Img r;
    uint32_t *dst = reinterpret_cast<uint32_t *>(&r);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(Img) / 4); i++)
        dst[i] = src[i];
    return r;
}

// A chunk of host data carried in the kernel arguments and stored to
// device memory.  A launch captured into a graph keeps its arguments, so
// every replay writes the same words again: this is how the image table of
// a batch call captured into a graph reaches the device without a host
// buffer that would have to outlive the graph.
constexpr int kChunkWords = 512;
struct WordChunk {
    uint32_t w[kChunkWords];
};
__global__ __launch_bounds__(kChunkWords) void k_put_words(uint32_t *dst, int n, WordChunk c) {
    const int i = threadIdx.x;
    if (i < n)
        dst[i] = c.w[i];
}

// Workgroups are dealt to the eight XCDs round robin (workgroup b runs on
// XCD b % 8, each XCD with its own L2).  This gives each XCD a contiguous
// range of the n tiles in raster order, so horizontally adjacent tiles, which
// share the cache lines straddling their common edge, are read through the
// same L2 at about the same time.  A bijection of [0, n).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int q = n / kXcds, r = n % kXcds, x = b % kXcds, j = b / kXcds;
    return x * q + (x < r ? x : r) + j;
}

// ------------------------------------------------------------------------
// Tile geometry.  NSR block rows of BH image rows (BH = 2: runs of row
// pairs, 8-conn; BH = 1: runs of single rows), TW columns, NW mask words per
// row.  BH = 0 is the gray-level form: single rows, NSR / 2 of them, so that
// the node capacity (NSR * TW / 2) covers every pixel of the tile (runs of
// equal bytes may touch each other).
// ------------------------------------------------------------------------
template <int NSR, int TW, int BH>
struct Geo {
    static constexpr bool GRAY = BH == 0;
    static constexpr int RB = GRAY ? 1 : BH;          // image rows per block row
    static constexpr int NBR = GRAY ? NSR / 2 : NSR;  // block rows
    static constexpr int TH = NBR * RB;
    static constexpr int NW = TW / 32;
    static constexpr int NU = NBR * NW;                        // (block row, word) units
    static constexpr int NM = TH * NW;                         // mask words
    static constexpr int RCAP = NSR * (TW / 2);                // most nodes a tile can hold
    static constexpr int RW = RCAP / 32;                       // words of a node/component bitmask
    static constexpr int CAP = 2 * (TH + TW);                  // > pixels on the tile perimeter
    static_assert(TW % 64 == 0, "tile width must be a multiple of 64");
    static_assert(TH * TW <= 65535, "local pixel indices must fit 16 bits with one spare value");
    static_assert(RCAP <= 65535, "local component ordinals must fit 16 bits");
};

// ------------------------------------------------------------------------
// Relaxed atomics at a chosen scope (workgroup for LDS, agent for the
// global array: the L2 caches of the eight XCDs are not coherent with each
// other, so every access to a shared parent entry is an agent-scope atomic).
// ------------------------------------------------------------------------
// (P may carry an address space; V is the plain value type.)
template <int S, class P>
__device__ __forceinline__ auto aload(P *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, S);
}
template <int S, class P, class V>
__device__ __forceinline__ void astore(P *p, V v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, S);
}
// Compare-and-swap; returns the value found at *p (== expect on success).
template <int S, class P, class V>
__device__ __forceinline__ V acas(P *p, V expect, V v) {
    __hip_atomic_compare_exchange_strong(p, &expect, v, __ATOMIC_RELAXED, __ATOMIC_RELAXED, S);
    return expect;
}

// Rem's union with splicing (Algorithm 2), safe for concurrent callers as in
// Algorithm 8.  Each step takes the side whose parent is larger (node n with
// parent pn, other side's parent q < pn) and tries one compare-and-swap
// P[n]: pn -> q.  If n is a root (pn == n) a success is the link and ends
// the union; otherwise a success is the splice and the step moves up to pn.
// A failed CAS means another caller changed P[n]; the step re-reads it.
// Every successful CAS lowers an entry (q < pn <= n), so there are finitely
// many of them, every root stays its set's smallest node, and the loop ends.
// The splice done by CAS rather than a plain store only skips a splice that
// a concurrent change made stale.
// (The unions of the scan and of the boundary merge run this step inside
// their own flat per-lane loops; on the global array the entries are packed
// (key of parent << 32 | parent id), so comparing packed parents compares
// their keys and every set's root is the node with the smallest key.)

// Find after all unions are done, on a parent array of byte offsets (4 x
// node): the roots are fixed, so each node stores its own root and nothing
// else (a concurrent walk reads either the old parent, an ancestor, or the
// root).  Every node has its own thread, so the path's other nodes are set
// by theirs; compressing them too measured slower.  Returns the root's
// byte offset.
template <int S>
__device__ int32_t find_root_store(int32_t *P, int32_t x) {
    char *base = reinterpret_cast<char *>(P);
    int32_t r = 4 * x, p;
    while ((p = aload<S>(reinterpret_cast<int32_t *>(base + r))) != r)
        r = p;
    if (r != 4 * x)
        astore<S>(P + x, r);
    return r;
}

// ------------------------------------------------------------------------
// Bit helpers.  Bit j of a mask word is column 32*w + j.
// ------------------------------------------------------------------------
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t mask_le(int b) { return 0xFFFFFFFFu >> (31 - b); }  // bits 0..b
// set bits of s at positions 0..b (0 <= b <= 31): shifted to the top, one
// instruction fewer than masking
__device__ __forceinline__ int popc_le(uint32_t s, int b) { return __popc(s << (31 - b)); }
__device__ __forceinline__ uint32_t mask_lt(int b) { return (1u << b) - 1u; }          // bits 0..b-1
__device__ __forceinline__ uint32_t mask_ge(int b) { return 0xFFFFFFFFu << b; }        // bits b..31

__device__ __forceinline__ int popc_before(const uint32_t *row, int c) {
    int w = c >> 5, n = 0;
    for (int k = 0; k < w; k++)
        n += __popc(row[k]);
    return n + __popc(row[w] & mask_lt(c & 31));
}

// 4 bytes -> 4 bits (byte > level), for the foreground test.  With
// level < 128: adding 127 - level to the low 7 bits of a byte sets its bit 7
// iff those bits exceed level (no carry crosses a byte); OR-ing the byte adds
// every byte >= 128.  With level >= 128 the byte needs bit 7 itself and low
// bits above level - 128: add 255 - level and AND with the byte.  (level 0
// is the plain nonzero test.)  The multiply gathers bits 7, 15, 23, 31 into
// bits 28..31.
template <bool HI>
__device__ __forceinline__ uint32_t gt4(uint32_t x, uint32_t k) {
    const uint32_t s = (x & 0x7f7f7f7fu) + k;
    const uint32_t t = (HI ? (s & x) : (s | x)) & 0x80808080u;
    return (t * 0x00204081u) >> 28;
}

template <bool HI>
__device__ __forceinline__ uint32_t gt16(u32x4 v, uint32_t k) {
    return gt4<HI>(v.x, k) | (gt4<HI>(v.y, k) << 4) | (gt4<HI>(v.z, k) << 8) | (gt4<HI>(v.w, k) << 12);
}

// 4 bytes -> 4 bits: byte == 0 (the complement of the nonzero test above).
__device__ __forceinline__ uint32_t z4(uint32_t x) {
    const uint32_t t = ~((((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x)) & 0x80808080u;
    return (t * 0x00204081u) >> 28;
}

// 32 equality bits of two 32-byte groups (8 dwords each).
__device__ __forceinline__ uint32_t eq32(const uint32_t *a, const uint32_t *b) {
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < 8; j++)
        m |= z4(a[j] ^ b[j]) << (4 * j);
    return m;
}

// 32 bytes from a row address p that is not 16-byte aligned, as 8 dwords:
// the nine aligned dwords that cover them are loaded (two 16-byte loads at
// 4-byte alignment and one dword) and shifted into place with byte aligns.
// The loaded dwords reach at most 3 bytes before p and after p + 31; an
// aligned dword holding one byte of the image lies in a page of the image,
// so those bytes are readable (and unused).
typedef uint32_t u32x4a4 __attribute__((ext_vector_type(4), aligned(4)));
__device__ __forceinline__ void load_unaligned32(const uint8_t *p, uint32_t *d) {
    // (the aligned address by pointer arithmetic, so that the compiler keeps
    // the global address space and emits global, not flat, loads)
    const uint32_t sh = (uint32_t)(reinterpret_cast<uintptr_t>(p) & 3u);
    const uint32_t *a = reinterpret_cast<const uint32_t *>(p - sh);
    const u32x4a4 lo = __builtin_nontemporal_load(reinterpret_cast<const u32x4a4 *>(a));
    const u32x4a4 hi = __builtin_nontemporal_load(reinterpret_cast<const u32x4a4 *>(a + 4));
    const uint32_t w8 = sh ? a[8] : 0u;
    const uint32_t w[9] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w, w8};
#pragma unroll
    for (int j = 0; j < 8; j++)
        d[j] = __builtin_amdgcn_alignbyte(w[j + 1], w[j], sh);
}

// The 32 bytes of row y from column x (x % 32 == 0) as 8 dwords; bytes
// outside the image read as 0.
__device__ __forceinline__ void load_bytes(const Img &im, int y, int x, uint32_t *d) {
#pragma unroll
    for (int j = 0; j < 8; j++)
        d[j] = 0u;
    if (y >= im.H || x >= im.W)
        return;
    const uint8_t *p = im.img + (int64_t)y * im.stride + x;
    if (x + 32 <= im.W && ((reinterpret_cast<uintptr_t>(p) & 15u) == 0)) {
        const u32x4 a = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
        const u32x4 b = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p + 16));
        d[0] = a.x; d[1] = a.y; d[2] = a.z; d[3] = a.w;
        d[4] = b.x; d[5] = b.y; d[6] = b.z; d[7] = b.w;
        return;
    }
    if (x + 32 <= im.W) {
        load_unaligned32(p, d);
        return;
    }
    const int n = im.W - x < 32 ? im.W - x : 32;
#pragma unroll
    for (int j = 0; j < 8; j++)
#pragma unroll
        for (int q = 0; q < 4; q++)
            if (4 * j + q < n)
                d[j] |= (uint32_t)p[4 * j + q] << (8 * q);
}

// Foreground bits (byte > level) of 32 bytes held as 8 dwords.
__device__ __forceinline__ uint32_t fg32(const uint32_t *d, int lv) {
    uint32_t m = 0;
    if (lv < 128) {
        const uint32_t k = (uint32_t)(127 - lv) * 0x01010101u;
#pragma unroll
        for (int j = 0; j < 8; j++)
            m |= gt4<false>(d[j], k) << (4 * j);
    } else {
        const uint32_t k = (uint32_t)(255 - lv) * 0x01010101u;
#pragma unroll
        for (int j = 0; j < 8; j++)
            m |= gt4<true>(d[j], k) << (4 * j);
    }
    return m;
}

// 32 pixels of row y starting at column x (x % 32 == 0), foreground iff the
// byte exceeds the image's level; outside = 0.
__device__ __forceinline__ uint32_t load_word(const Img &im, int y, int x) {
    if (y >= im.H || x >= im.W)
        return 0u;
    const uint8_t *p = im.img + (int64_t)y * im.stride + x;
    const int lv = im.level;
    if (x + 32 <= im.W && ((reinterpret_cast<uintptr_t>(p) & 15u) == 0)) {
        u32x4 a = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
        u32x4 b = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p + 16));
        if (lv < 128) {
            const uint32_t k = (uint32_t)(127 - lv) * 0x01010101u;
            return gt16<false>(a, k) | (gt16<false>(b, k) << 16);
        }
        const uint32_t k = (uint32_t)(255 - lv) * 0x01010101u;
        return gt16<true>(a, k) | (gt16<true>(b, k) << 16);
    }
    if (x + 32 <= im.W) {
        uint32_t d[8];
        load_unaligned32(p, d);
        return fg32(d, lv);
    }
    uint32_t m = 0;
    int n = im.W - x < 32 ? im.W - x : 32;
    for (int i = 0; i < n; i++)
        m |= (uint32_t)((int)p[i] > lv) << i;
    return m;
}

// Exclusive prefix sum of v over a workgroup of NT threads; *total gets the
// sum.  Contains two barriers; every thread must call it.
// Inclusive prefix sum over the 64 lanes of a wave with DPP moves: shifts by
// 1, 2, 4, 8 inside each row of 16 lanes (lanes without a source add 0),
// then the last lane of row 0 / 2 is added to row 1 / 3 and the last lane
// of row 1 to rows 2 and 3.
__device__ __forceinline__ int32_t wave_inclusive_scan(int32_t v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
    return v;
}

template <int NT>
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t *total) {
    __shared__ int32_t wsum[NT / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int32_t incl = wave_inclusive_scan(v);
    if (lane == 63)
        wsum[wv] = incl;
    __syncthreads();
    int32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; k++) {
        int32_t s = wsum[k];
        before += (k < wv) ? s : 0;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

// LDS written by some lanes of a wave, then read by others: keeps the
// compiler from moving LDS accesses across this point (a wave's LDS
// operations are carried out in order).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive popcount prefix of n bitmask words by one whole wave (all 64
// lanes call it); returns the total.
__device__ __forceinline__ int32_t wave_popcount_prefix(const uint32_t *bits, int32_t *pref, int n, int lane) {
    int32_t carry = 0;
    for (int base = 0; base < n; base += 64) {
        const int i = base + lane;
        const int32_t v = i < n ? __popc(bits[i]) : 0;
        const int32_t incl = wave_inclusive_scan(v);
        if (i < n)
            pref[i] = carry + incl - v;
        carry += __builtin_amdgcn_readlane(incl, 63);
    }
    return carry;
}

__device__ __forceinline__ int32_t rank_of(const uint32_t *bits, const int32_t *pref, int32_t k) {
    return pref[k >> 5] + __popc(bits[k >> 5] & mask_lt(k & 31));
}

// ------------------------------------------------------------------------
// Block runs of a tile: masks, starts and node ordinals.  Shared by the
// scan and the labeling pass so both number the nodes identically.
// ------------------------------------------------------------------------
template <int NSR, int TW, int BH>
struct RunLds {
    using G = Geo<NSR, TW, BH>;
    uint32_t M[G::NM];      // foreground masks, row-major
    uint32_t S[G::NU];      // block-run starts per (block row, word)
    int32_t base[G::NU];    // ordinal of the first node starting in the unit
};

template <int NSR, int TW, int BH>
__device__ __forceinline__ uint32_t block_mask(const uint32_t *M, int R, int w) {
    constexpr int NW = Geo<NSR, TW, BH>::NW, RB = Geo<NSR, TW, BH>::RB;
    uint32_t m = M[(R * RB) * NW + w];
    if (RB == 2)
        m |= M[(R * RB + 1) * NW + w];
    return m;
}

// Node ordinal of the block run of block row R containing column c (which
// must be foreground in that block row).
template <int NSR, int TW, int BH>
__device__ __forceinline__ int32_t node_at(const RunLds<NSR, TW, BH> &t, int R, int c) {
    constexpr int NW = Geo<NSR, TW, BH>::NW;
    const int u = R * NW + (c >> 5);
    return t.base[u] - 1 + popc_le(t.S[u], c & 31);
}

// Fills S and base from M; returns the number of nodes (same on all threads).
// Gray-level images (one row per block row): a run starts at every object
// pixel that does not continue its left neighbour's run (E: same value as
// the left neighbour).
template <int NSR, int TW, int BH, int NT>
__device__ int32_t number_runs(RunLds<NSR, TW, BH> &t, const uint32_t *E = nullptr) {
    using G = Geo<NSR, TW, BH>;
    constexpr bool GRAY = G::GRAY;
    constexpr int NW = G::NW;
    constexpr int UPT = (G::NU + NT - 1) / NT;
    int32_t carry = 0;
#pragma unroll
    for (int k = 0; k < UPT; k++) {
        const int u = threadIdx.x + k * NT;
        int32_t cnt = 0;
        if (u < G::NU) {
            const int R = u / NW, w = u % NW;
            uint32_t s;
            if (GRAY) {
                s = t.M[u] & ~E[u];
            } else {
                uint32_t bm = block_mask<NSR, TW, BH>(t.M, R, w);
                uint32_t bl = w ? block_mask<NSR, TW, BH>(t.M, R, w - 1) : 0u;
                s = bm & ~((bm << 1) | (bl >> 31));
            }
            t.S[u] = s;
            cnt = __popc(s);
        }
        int32_t tot;
        int32_t ex = block_exclusive_scan<NT>(cnt, &tot);
        if (u < G::NU)
            t.base[u] = carry + ex;
        carry += tot;
    }
    return carry;
}

// ------------------------------------------------------------------------
// K1: tile scan.
// ------------------------------------------------------------------------
// Node ordinals around the (block row, word) unit u of a contact row, from
// run starts and bases: the node of block row R whose run covers column c of
// the word, and the node of block row R - 1 covering column pc (-1 .. 32: a
// partner one column past either end of the word).  The upper row's starts
// sit in a 64-bit window, shifted up one bit, with bit 0 of the next word's
// starts above them: the nodes up to pc are the window's bits 0 .. pc + 1
// (bit 0, column -1, is never set: a partner left of the word is the last
// node before the word's own, bU).  Plain values throughout: a select between
// the addresses of struct members would leave them in private memory.
#define CCL_UNIT_RUNS(t, u)                                                            \
    const int w_ = (u) % NW, uu_ = (u) - NW;                                           \
    const uint32_t sR = t.S[u];                                                        \
    const int32_t bR = t.base[u] - 1, bU = t.base[uu_] - 1;                            \
    const uint64_t wU = ((uint64_t)((w_ < NW - 1) ? (t.S[uu_ + 1] & 1u) : 0u) << 33) | \
                        ((uint64_t)t.S[uu_] << 1)
__device__ __forceinline__ int32_t run_node(uint32_t s, int32_t b, int c) { return b + popc_le(s, c); }
__device__ __forceinline__ int32_t upper_node(int pc, uint64_t wU, int32_t bU) {
    return bU + __popcll(wU << (62 - pc));
}

// Node capacity of the tile scan's LDS arrays (a multiple of 32).  The full
// form holds the most nodes a tile can have (G::RCAP); the compact form holds
// 17/32 of that, which covers every i.i.d. image: a run of the scanned rows
// starts at a given column with probability q(1 - q) <= 1/4 (q = that the
// column is occupied), i.e. 1/2 of the capacity on average, with a spread of
// a few dozen nodes per tile.  A tile with more nodes (stripes,
// checkerboards) is left to the full form.  (With 17/32 the compact form of
// a 64x256 row-pair tile takes 20 KB of LDS: eight tiles share a CU.)
template <int NSR, int TW, int BH>
constexpr int compact_cap() { return Geo<NSR, TW, BH>::RCAP / 32 * 17; }

template <int NSR, int TW, int BH, int CAPN>
struct ScanLate {
    using G = Geo<NSR, TW, BH>;
    static constexpr int CW = CAPN / 32;
    uint16_t RT[CAPN];      // root of each node, then its component ordinal
    uint32_t RFB[CW];       // root nodes (bit per node)
    uint32_t RBB[CW];       // components touching a shared tile edge (bit per component)
    int32_t RFP[CW];        // prefix counts of RFB, later of RBB
    uint32_t RK[G::NM];     // keys of interior components (bit per pixel)
    int32_t rowcnt[G::TH];
    int32_t ncomp;          // local component count, for every wave
};

template <int NSR, int TW, int BH, int CAPN>
struct ScanLds : RunLds<NSR, TW, BH> {
    using G = Geo<NSR, TW, BH>;
    static constexpr bool GRAY = G::GRAY;
    static constexpr int PRCAP = (int)(sizeof(ScanLate<NSR, TW, BH, CAPN>) / 4);
    static constexpr int GN = GRAY ? G::NM : 1;
    static_assert(CAPN % 32 == 0 && CAPN <= G::RCAP, "node capacity");
    int32_t P[CAPN];        // parent array over nodes; later the key of each component
    // gray levels, bit per pixel: same value as the left neighbour (GE), as
    // the pixel above (GV), above-left (GD1), above-right (GD2)
    uint32_t GE[GN], GV[GN], GD1[GN], GD2[GN];
    union {
        uint32_t PR[PRCAP];  // during the union step: touching node pairs (x | y << 16)
        ScanLate<NSR, TW, BH, CAPN> late;
        uint8_t BY[GRAY ? G::TH * TW : 1];  // gray levels: the tile's bytes, until the masks exist
    };
    static_assert(!GRAY || sizeof(BY) <= sizeof(ScanLate<NSR, TW, BH, CAPN>), "gray tile layout");
};

// Scan of one tile by NT threads with LDS for CAPN nodes.  With COMPACT a
// tile whose runs outnumber CAPN is not scanned: its node count is stored
// as -1 (kOverflow) and k_tile_scan_rest scans it later.
constexpr int32_t kOverflow = -1;
template <int NSR, int TW, int BH, int ORD, int NT, int CAPN, bool COMPACT>
__device__ __forceinline__ void scan_tile(const Batch &b, const int tile, ScanLds<NSR, TW, BH, CAPN> &t) {
    using G = Geo<NSR, TW, BH>;
    constexpr bool GRAY = G::GRAY;
    constexpr int MPT = (G::NM + NT - 1) / NT;
    constexpr int UPT = (G::NU + NT - 1) / NT;
    // threads per (block row, word) unit in the union step, and the bits each takes
    constexpr int LPU = NT >= G::NU ? NT / G::NU : 1;
    constexpr int UPT2 = (G::NU * LPU + NT - 1) / NT;
    static_assert(NT < G::NU || NT % G::NU == 0, "unit count must divide the thread count");
    constexpr int NW = G::NW, TH = G::TH;
    constexpr int WG = __HIP_MEMORY_SCOPE_WORKGROUP;
    using L = ScanLds<NSR, TW, BH, CAPN>;
    constexpr int CW = CAPN / 32;   // words of the LDS node and component bitmasks
    const Img &im = find_img(b, tile, kTile);
    const int ti = tile - im.tile0;
    const int ty = ti / im.NTX, tx = ti % im.NTX;
    const int y0 = ty * TH, x0 = tx * TW;
    const int tid = threadIdx.x;
    const bool conn8 = im.conn == 8;

    // 1. foreground masks (kept in LDS; stored for the labeling pass at the
    // end, so that no barrier waits on those stores)
    uint32_t mreg[MPT];
    uint32_t ereg[GRAY ? MPT : 1];
#pragma unroll
    for (int k = 0; k < MPT; k++) {
        const int i = tid + k * NT;
        if (i < G::NM) {
            const int r = i / NW, w = i % NW;
            if (GRAY) {
                uint32_t d[8];
                load_bytes(im, y0 + r, x0 + (w << 5), d);
                mreg[k] = fg32(d, im.level);
                uint32_t *by = reinterpret_cast<uint32_t *>(t.BY + r * TW + (w << 5));
#pragma unroll
                for (int j = 0; j < 8; j++)
                    by[j] = d[j];
            } else {
                mreg[k] = load_word(im, y0 + r, x0 + (w << 5));
            }
            t.M[i] = mreg[k];
        }
    }
    __syncthreads();
    if (GRAY) {
        // equality of each object pixel with its left, upper, upper-left and
        // upper-right neighbours inside the tile (bytes shifted by one)
#pragma unroll
        for (int k = 0; k < MPT; k++) {
            const int i = tid + k * NT;
            if (i < G::NM) {
                const int r = i / NW, w = i % NW;
                const uint32_t *cur = reinterpret_cast<const uint32_t *>(t.BY + r * TW + (w << 5));
                uint32_t c[8], sh[8];
#pragma unroll
                for (int j = 0; j < 8; j++)
                    c[j] = cur[j];
                const uint32_t m = mreg[k];
                const uint32_t lb = w ? (uint32_t)t.BY[r * TW + (w << 5) - 1] : 0u;
#pragma unroll
                for (int j = 0; j < 8; j++)
                    sh[j] = (c[j] << 8) | (j ? c[j - 1] >> 24 : lb);
                // bit 0 of the tile row has no left neighbour in the tile
                const uint32_t e = m & eq32(c, sh) & (w ? 0xFFFFFFFFu : 0xFFFFFFFEu);
                ereg[k] = e;
                t.GE[i] = e;
                uint32_t v = 0u, d1 = 0u, d2 = 0u;
                if (r > 0) {
                    const uint32_t *up = reinterpret_cast<const uint32_t *>(t.BY + (r - 1) * TW + (w << 5));
                    uint32_t u[8];
#pragma unroll
                    for (int j = 0; j < 8; j++)
                        u[j] = up[j];
                    v = m & eq32(c, u);
                    const uint32_t ul = w ? (uint32_t)t.BY[(r - 1) * TW + (w << 5) - 1] : 0u;
                    const uint32_t ur = (w < NW - 1) ? (uint32_t)t.BY[(r - 1) * TW + (w << 5) + 32] : 0u;
#pragma unroll
                    for (int j = 0; j < 8; j++)
                        sh[j] = (u[j] << 8) | (j ? u[j - 1] >> 24 : ul);
                    d1 = m & eq32(c, sh) & (w ? 0xFFFFFFFFu : 0xFFFFFFFEu);
#pragma unroll
                    for (int j = 0; j < 8; j++)
                        sh[j] = (u[j] >> 8) | ((j < 7 ? u[j + 1] : ur) << 24);
                    d2 = m & eq32(c, sh) & ((w < NW - 1) ? 0xFFFFFFFFu : 0x7FFFFFFFu);
                }
                t.GV[i] = v;
                t.GD1[i] = d1;
                t.GD2[i] = d2;
            }
        }
        __syncthreads();
    }

    // 2. block runs, their ordinals and start positions (the starts serve
    // the canonical keys only)
    const int32_t n_runs = number_runs<NSR, TW, BH, NT>(t, t.GE);
    if (COMPACT && n_runs > CAPN) {
        if (tid == 0)
            im.tcnt[ti * 4 + 0] = kOverflow;
        return;
    }
    // The parent array holds byte offsets (4 x node) until the flatten, so
    // that a union step addresses a parent without a shift.
    for (int k = tid; k < n_runs; k += NT)
        t.P[k] = 4 * k;
    __syncthreads();
    auto at = [&](int32_t off) { return reinterpret_cast<int32_t *>(reinterpret_cast<char *>(t.P) + off); };

    // 3. unite touching nodes of block rows R-1 and R.  The contact rows are
    // the last row of R-1 (u) and the first row of R (m).  Each touching pair
    // of row runs is met exactly once: U1 at the first column of their
    // overlap, U2 (8-conn) where the upper run starts just right of the
    // lower one's end, U3 (8-conn) where the lower run starts just right of
    // the upper one's end.  The contacts are first listed as node pairs
    // (compacted by a block scan), then the pairs are dealt out evenly to
    // the threads, which apply Rem's union with splicing to them.  A tile
    // with more contacts than the list holds is done in several rounds.
    // Contacts to list, one per column: the partner is at c + d with d = 0
    // (U1), -1 where the column's bit is set in cn (U3), +1 where it is set
    // in cp (U2).  A column with more than one contact (U3 and U2 at a lone
    // lower pixel; with gray levels also U1 and a diagonal) lists the others
    // from cx: low half d = -1, high half d = +1.  The direct links (the
    // first contact of a run starting in the word) use the same one-per-
    // column form in df, dn, dp.
    uint32_t cl[UPT2], cn[UPT2], cp[UPT2];
    uint64_t cx[UPT2];
    uint32_t df[UPT2], dn[UPT2], dp[UPT2];
    int32_t coff[UPT2];
    int32_t n_pairs = 0;
#pragma unroll
    for (int k = 0; k < UPT2; k++) {
        const int v = tid + k * NT;
        const int u = v % G::NU, h = v / G::NU;
        const int R = u / NW, w = u % NW;
        cl[k] = cn[k] = cp[k] = 0u;
        cx[k] = 0;
        df[k] = dn[k] = dp[k] = 0u;
        if (GRAY && h < LPU && R > 0) {
            // gray levels (one row per block row): U1 at the first column of
            // each stretch where the pixel above has the same value and both
            // rows continue their runs; the diagonal contacts unless the
            // vertical contact at c already joins the same two runs
            const uint32_t V = t.GV[u], Vl = w ? t.GV[u - 1] >> 31 : 0u;
            const uint32_t Em = t.GE[u], Eu = t.GE[u - NW];
            const uint32_t EuR = (w < NW - 1) ? t.GE[u - NW + 1] : 0u;
            const uint32_t u1 = V & ~(((V << 1) | Vl) & Em & Eu);
            uint32_t u2 = 0u, u3 = 0u;
            if (conn8) {
                u3 = t.GD1[u] & ~(V & Eu);
                u2 = t.GD2[u] & ~(V & ((Eu >> 1) | (EuR << 31)));
            }
            constexpr int PART = 32 / LPU;
            const uint32_t mine = (PART == 32 ? 0xFFFFFFFFu : ((1u << PART) - 1u)) << (h * PART);
            cl[k] = (u1 | u2 | u3) & mine;
            cn[k] = u3 & ~u1 & mine;
            cp[k] = u2 & ~u1 & ~u3 & mine;
            cx[k] = (uint64_t)(u3 & u1 & mine) | ((uint64_t)(u2 & (u1 | u3) & mine) << 32);
        } else if (!GRAY && h < LPU && R > 0) {
            const int rm = R * G::RB, ru = R * G::RB - 1;
            const uint32_t m = t.M[rm * NW + w];
            const uint32_t mL = w ? t.M[rm * NW + w - 1] : 0u;
            const uint32_t up = t.M[ru * NW + w];
            const uint32_t uL = w ? t.M[ru * NW + w - 1] : 0u;
            const uint32_t o = m & up;
            uint32_t u1 = o & ~((o << 1) | ((mL & uL) >> 31));
            uint32_t u2 = 0u, u3 = 0u;
            if (conn8) {
                const uint32_t mR = (w < NW - 1) ? t.M[rm * NW + w + 1] : 0u;
                const uint32_t uR = (w < NW - 1) ? t.M[ru * NW + w + 1] : 0u;
                const uint32_t mn = (m >> 1) | (mR << 31);
                const uint32_t un = (up >> 1) | (uR << 31);
                const uint32_t mp = (m << 1) | (mL >> 31);
                const uint32_t upp = (up << 1) | (uL >> 31);
                u2 = m & ~mn & ~up & un;
                u3 = m & ~mp & ~up & upp;
            }
            // first contact of each run that starts in this word: the carry
            // of (run bits without contacts) + (run starts) stops at it
            const uint32_t B = block_mask<NSR, TW, BH>(t.M, R, w);
            const uint32_t C = u1 | u2 | u3;
            const uint32_t F = ((B & ~C) + t.S[u]) & C;
            const uint32_t d3 = F & u3, d1 = F & ~u3 & u1, d2 = F & ~u3 & ~u1 & u2;
            if (G::RB == 2) {
                // Row pairs: two contacts in one run of A (both block rows
                // foreground) join the same two block runs (the partners,
                // one column aside at most, are foreground next to that
                // run), so only the first contact of each A run in the word
                // is kept; where a U3 and a U2 share that column, the U2
                // repeats it.  The direct link is the first contact of its
                // block run, so it is always a kept one.
                const uint32_t A = B & block_mask<NSR, TW, BH>(t.M, R - 1, w);
                const uint32_t CA = C & A;
                const uint32_t first = ((A & ~CA) + (A & ~(A << 1))) & CA;
                const uint32_t keep = ~(CA & ~first);
                u1 &= keep;
                u3 &= keep;
                u2 &= keep & ~(first & u3);
            }
            // this thread's share of the word's contact positions
            constexpr int PART = 32 / LPU;
            const uint32_t mine = (PART == 32 ? 0xFFFFFFFFu : ((1u << PART) - 1u)) << (h * PART);
            // (row runs never give U1 and U3 at one column: the pixel above
            // decides which)
            const uint32_t l1 = u1 & ~d1, l3 = u3 & ~d3, l2 = u2 & ~d2;
            cl[k] = (l1 | l2 | l3) & mine;
            cn[k] = l3 & mine;
            cp[k] = l2 & ~l3 & mine;
            cx[k] = (uint64_t)(l2 & l3 & mine) << 32;
            df[k] = F & mine;
            dn[k] = d3 & mine;
            dp[k] = d2 & mine;
        }
        int32_t tot;
        coff[k] = n_pairs + block_exclusive_scan<NT>(__popc(cl[k]) + __popcll(cx[k]), &tot);
        n_pairs += tot;
    }
    // direct links (the scan's copy step: a pixel whose first neighbour is
    // found takes that neighbour's set without a merge): the first contact
    // of each run makes the run's node a child of the upper node.  The node
    // is still a fresh root and the upper node has the smaller ordinal, so
    // parents stay below their children, as the Rem steps require; the run's
    // further contacts are merged as before.
#pragma unroll
    for (int k = 0; k < UPT2; k++) {
        uint32_t l = df[k];
        if (!l)
            continue;
        const int u = (tid + k * NT) % G::NU;
        CCL_UNIT_RUNS(t, u);
        do {
            const int c = __ffs(l) - 1;
            l &= l - 1u;
            const int d = (int)((dp[k] >> c) & 1u) - (int)((dn[k] >> c) & 1u);
            t.P[run_node(sR, bR, c)] = 4 * upper_node(c + d, wU, bU);
        } while (l);
    }
    for (int r0 = 0; r0 < n_pairs; r0 += L::PRCAP) {
        const int r1 = r0 + L::PRCAP;
#pragma unroll
        for (int k = 0; k < UPT2; k++) {
            int32_t idx = coff[k];
            uint32_t l = cl[k];
            uint64_t x2 = cx[k];
            if ((!l && !x2) || idx >= r1)
                continue;
            const int u = (tid + k * NT) % G::NU;
            CCL_UNIT_RUNS(t, u);
            while (l && idx < r1) {
                const int c = __ffs(l) - 1;
                l &= l - 1u;
                const int d = (int)((cp[k] >> c) & 1u) - (int)((cn[k] >> c) & 1u);
                if (idx >= r0)
                    t.PR[idx - r0] = (uint32_t)run_node(sR, bR, c) |
                                     ((uint32_t)upper_node(c + d, wU, bU) << 16);
                idx++;
            }
            while (x2 && idx < r1) {
                const int bit = __ffsll((unsigned long long)x2) - 1;
                x2 &= x2 - 1;
                const int c = bit & 31, d = (bit >> 5) ? 1 : -1;
                if (idx >= r0)
                    t.PR[idx - r0] = (uint32_t)run_node(sR, bR, c) |
                                     ((uint32_t)upper_node(c + d, wU, bU) << 16);
                idx++;
            }
        }
        __syncthreads();
        if (r0 == 0) {
            // one pointer-jumping round over the direct links: every node
            // takes its grandparent, which halves the chains of direct links
            // that the union steps and the flatten walk (a concurrent update
            // leaves an ancestor either way, so the sets do not change)
            for (int k = tid; k < n_runs; k += NT) {
                const int32_t p = aload<WG>(t.P + k);
                astore<WG>(t.P + k, aload<WG>(at(p)));
            }
            __syncthreads();
        }
        // Each lane steps its own union (one load pair and one CAS per step)
        // and takes its next pair as soon as the current union ends.
        const int np = min(n_pairs - r0, L::PRCAP);
        int q = tid;
        int32_t rx = 0, ry = 0;  // byte offsets of the two nodes
        if (q < np) {
            const uint32_t pr = t.PR[q];
            rx = (int32_t)((pr & 0xFFFFu) << 2);
            ry = (int32_t)((pr >> 16) << 2);
        }
        // Branch-free step: when both parents are equal the compare-and-swap
        // puts the value onto itself and changes nothing.
        while (q < np) {
            const int32_t px = aload<WG>(at(rx));
            const int32_t py = aload<WG>(at(ry));
            const bool xs = px > py;
            const int32_t n = xs ? rx : ry;
            const int32_t pn = xs ? px : py;
            const int32_t seen = acas<WG>(at(n), pn, xs ? py : px);
            const bool ok = seen == pn;
            const bool next = px == py || (ok && pn == n);
            rx = ok && xs ? pn : rx;
            ry = ok && !xs ? pn : ry;
            if (next) {
                q += NT;
                const uint32_t pr = t.PR[min(q, np - 1)];
                rx = (int32_t)((pr & 0xFFFFu) << 2);
                ry = (int32_t)((pr >> 16) << 2);
            }
        }
        __syncthreads();
    }
    __syncthreads();
    if (ORD == kCanonical) {
        for (int i = tid; i < G::NM; i += NT)
            t.late.RK[i] = 0u;
        for (int r = tid; r < TH; r += NT)
            t.late.rowcnt[r] = 0;
    }
    for (int i = tid; i < CW; i += NT) {
        t.late.RFB[i] = 0u;
        t.late.RBB[i] = 0u;
    }
    __syncthreads();

    // 4. flatten; roots are numbered in node order (local components).  A
    // wave handles 64 consecutive nodes, so its ballot is two words of the
    // root bitmask.
    const int wave = tid >> 6, lane = tid & 63;
    for (int k0 = 0; k0 < n_runs; k0 += NT) {
        const int k = k0 + tid;
        bool root = false;
        if (k < n_runs)
            root = find_root_store<WG>(t.P, k) == 4 * k;
        const uint64_t bal = __ballot(root);
        const int wd = (k0 + wave * 64) >> 5;
        if (lane == 0 && wd < CW)
            t.late.RFB[wd] = (uint32_t)bal;
        if (lane == 32 && wd + 1 < CW)
            t.late.RFB[wd + 1] = (uint32_t)(bal >> 32);
    }
    __syncthreads();
    // (prefixes over at most RW words: one wave does them, the others skip)
    if (wave == 0) {
        const int32_t tot = wave_popcount_prefix(t.late.RFB, t.late.RFP, (n_runs + 31) >> 5, lane);
        if (lane == 0)
            t.late.ncomp = tot;
    }
    __syncthreads();
    // every node notes its root (a node index); the root's rank among the
    // roots, the node's local component, is taken below per (block row,
    // word) unit, where the node's block row and first column are known
    for (int k = tid; k < n_runs; k += NT)
        t.late.RT[k] = (uint16_t)(t.P[k] >> 2);
    __syncthreads();
    const int32_t n_comp = t.late.ncomp;

    // 5. canonical key of each component: its first pixel in raster order.
    // It lies in the block row of the component's root (the root is its
    // first node in block-row order), so only the nodes of that row offer
    // their first pixel (top row first); the key is the least of those.
    if (ORD == kCanonical) {
        for (int c = tid; c < n_comp; c += NT)
            t.P[c] = 0x7FFFFFFF;
        __syncthreads();
    }
    for (int u = tid; u < G::NU; u += NT) {
        const int R = u / NW, w = u % NW;
        const int32_t row_first = t.base[R * NW];  // first node of the block row
        uint32_t bits = t.S[u];
        int32_t k = t.base[u];
        while (bits) {
            const int col = (w << 5) + __ffs(bits) - 1;
            bits &= bits - 1u;
            const int32_t root = t.late.RT[k];
            const int32_t c = rank_of(t.late.RFB, t.late.RFP, root);
            t.late.RT[k] = (uint16_t)c;
            // (the root precedes its nodes, so it lies in this block row iff it
            // is not before the row's first node)
            if (ORD == kCanonical && root >= row_first) {
                int32_t key;
                if (G::RB == 1) {
                    key = R * TW + col;
                } else {
                    const int r0 = R * G::RB;
                    key = (r0 + 1) * TW + col;  // no top pixel: the run's start in the lower row
                    int ww = col >> 5, from = col & 31;
                    for (;;) {
                        const uint32_t tt = t.M[r0 * NW + ww] & mask_ge(from);
                        const uint32_t gap = ~block_mask<NSR, TW, BH>(t.M, R, ww) & mask_ge(from);
                        if (tt && (!gap || __ffs(tt) < __ffs(gap))) {
                            key = r0 * TW + (ww << 5) + __ffs(tt) - 1;
                            break;
                        }
                        if (gap || ww == NW - 1)
                            break;
                        ww++;
                        from = 0;
                    }
                }
                atomicMin(&t.P[c], key);
            }
            k++;
        }
    }
    __syncthreads();

    // 6. components touching an edge shared with another tile
    const bool top = ty > 0, bot = ty < im.NTY - 1, left = tx > 0, right = tx < im.NTX - 1;
    // one item per pixel of the top and bottom rows (marked where a run of
    // the row starts) and of the left and right columns
    for (int i = tid; i < 2 * TW + 2 * TH; i += NT) {
        int r, c;
        bool on;
        if (i < 2 * TW) {
            const int side = i / TW;
            c = i % TW;
            r = side ? TH - 1 : 0;
            const int w = c >> 5, bt = c & 31;
            bool start;
            if (G::RB == 1) {
                start = (t.S[r * NW + w] >> bt) & 1u;   // run starts of the row itself
            } else {
                const uint32_t m = t.M[r * NW + w];
                const uint32_t prev = bt ? (m >> (bt - 1)) & 1u : (w ? t.M[r * NW + w - 1] >> 31 : 0u);
                start = ((m >> bt) & 1u) && !prev;
            }
            on = (side ? bot : top) && start;
        } else {
            const int q = i - 2 * TW, side = q / TH;
            r = q % TH;
            c = side ? TW - 1 : 0;
            on = (side ? right : left) && ((t.M[r * NW + (c >> 5)] >> (c & 31)) & 1u);
        }
        if (on) {
            const int32_t comp = t.late.RT[node_at(t, r / G::RB, c)];
            atomicOr(&t.late.RBB[comp >> 5], 1u << (comp & 31));
        }
    }
    __syncthreads();
    int32_t n_bound = 0;  // known to the first wave, which exports it
    if (wave == 0)
        n_bound = wave_popcount_prefix(t.late.RBB, t.late.RFP, (n_comp + 31) >> 5, lane);
    for (int c = tid; c < (ORD == kCanonical ? n_comp : 0); c += NT) {
        if (!((t.late.RBB[c >> 5] >> (c & 31)) & 1u)) {
            const int32_t key = t.P[c];
            atomicOr(&t.late.RK[key >> 5], 1u << (key & 31));
            atomicAdd(&t.late.rowcnt[key / TW], 1);
        }
    }
    __syncthreads();

    // 7. exports
    const int64_t cbase = (int64_t)ti * G::CAP;
    for (int c = tid; c < n_comp; c += NT) {
        if ((t.late.RBB[c >> 5] >> (c & 31)) & 1u) {
            const int32_t j = rank_of(t.late.RBB, t.late.RFP, c);
            const uint32_t id = (uint32_t)(cbase + j);
            if (ORD == kCanonical) {
                const int32_t key = t.P[c];
                const int kr = key / TW, kc = key % TW;
                const uint32_t gkey = (uint32_t)((y0 + kr) * im.W + x0 + kc);
                im.bkey[id] = (uint16_t)key;
                im.bval[id] = popc_before(&t.late.RK[kr * NW], kc);
                im.uf[id] = ((uint64_t)gkey << 32) | id;
            } else {
                // the provisional label of a boundary component orders like
                // its id (tile, then boundary index, which follows the
                // component ordinal), so the id is its key
                im.uf[id] = ((uint64_t)id << 32) | id;
            }
        }
    }
    // edge buffers: boundary index of the component of every edge pixel
    for (int i = tid; i < 2 * TW + 2 * TH; i += NT) {
        int r, c;
        uint16_t *dst;
        bool on;
        if (i < 2 * TW) {
            const int side = i / TW;
            c = i % TW;
            r = side ? TH - 1 : 0;
            on = (side ? bot : top) && x0 + c < im.W;
            dst = im.he + ((int64_t)ty * 2 + side) * im.hep + x0 + c;
        } else {
            const int q = i - 2 * TW, side = q / TH;
            r = q % TH;
            c = side ? TW - 1 : 0;
            on = (side ? right : left) && y0 + r < im.H;
            dst = im.ve + ((int64_t)tx * 2 + side) * im.vep + y0 + r;
        }
        if (!on)
            continue;
        uint16_t v = kNone;
        if ((t.M[r * NW + (c >> 5)] >> (c & 31)) & 1u)
            v = (uint16_t)rank_of(t.late.RBB, t.late.RFP, t.late.RT[node_at(t, r / G::RB, c)]);
        *dst = v;
    }
    if (ORD == kCanonical) {
        for (int r = tid; r < TH; r += NT)
            if (y0 + r < im.H)
                im.seg[(int64_t)(y0 + r) * im.NTX + tx] = t.late.rowcnt[r];
    }
    // node -> component, two entries per store (an odd count writes one
    // unused entry past the end, inside the tile's capacity)
    uint32_t *grt2 = reinterpret_cast<uint32_t *>(im.rt + (int64_t)ti * G::RCAP);
    const uint32_t *RT2 = reinterpret_cast<const uint32_t *>(t.late.RT);
    for (int k = tid; 2 * k < n_runs; k += NT)
        grt2[k] = RT2[k];
    int32_t *gck = im.cf + (int64_t)ti * G::RCAP;
    for (int c = tid; c < (ORD == kCanonical ? n_comp : 0); c += NT)
        gck[c] = t.P[c];
    uint32_t *gcb = im.cb + (int64_t)ti * G::RW;
    for (int i = tid; i < ((n_comp + 31) >> 5); i += NT)
        gcb[i] = t.late.RBB[i];
    if (tid == 0) {
        im.tcnt[ti * 4 + 0] = n_runs;
        im.tcnt[ti * 4 + 1] = n_comp;
        im.tcnt[ti * 4 + 2] = n_bound;
    }
    uint32_t *gmask = im.masks + (int64_t)ti * G::NM * (GRAY ? 2 : 1);
#pragma unroll
    for (int k = 0; k < MPT; k++) {
        const int i = tid + k * NT;
        if (i < G::NM) {
            gmask[i] = mreg[k];
            if (GRAY)
                gmask[G::NM + i] = ereg[k];
        }
    }
}

// Full form: eight waves per tile and per SIMD (four workgroups per CU, as
// the LDS for every possible node allows); the register allocator is held
// to the matching scalar-register budget.
template <int NSR, int TW, int BH, int ORD>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_tile_scan(Batch b) {
    constexpr int C = Geo<NSR, TW, BH>::RCAP;
    __shared__ ScanLds<NSR, TW, BH, C> t;
    scan_tile<NSR, TW, BH, ORD, kTileThreads, C, false>(b, xcd_tile(blockIdx.x, gridDim.x), t);
}

// Compact form: four waves per tile, each lane taking a whole (block row,
// word) unit, with LDS for compact_cap() nodes, so that eight tiles share a
// CU.  Fewer waves per tile issue fewer instructions for the same tile (the
// per-wave work of each step is paid by half as many waves).
constexpr int kScanThreadsC = 256;
template <int NSR, int TW, int BH, int ORD>
__global__ __launch_bounds__(kScanThreadsC) __attribute__((amdgpu_waves_per_eu(8))) void k_tile_scan_c(Batch b) {
    constexpr int C = compact_cap<NSR, TW, BH>();
    __shared__ ScanLds<NSR, TW, BH, C> t;
    scan_tile<NSR, TW, BH, ORD, kScanThreadsC, C, true>(b, xcd_tile(blockIdx.x, gridDim.x), t);
}

// The tiles the compact form left (node count kOverflow), scanned by the
// full form.  Workgroup g checks the node counts of a stretch of at most 64
// consecutive tiles (the host launches at least ntiles / 64 workgroups) and
// scans the marked ones one after another; with none marked it ends at once.
template <int NSR, int TW, int BH, int ORD>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_tile_scan_rest(Batch b,
                                                                                                       int32_t ntiles) {
    constexpr int C = Geo<NSR, TW, BH>::RCAP;
    __shared__ ScanLds<NSR, TW, BH, C> t;
    __shared__ uint64_t marked;
    const int32_t per = (ntiles + (int32_t)gridDim.x - 1) / (int32_t)gridDim.x;
    const int32_t first = (int32_t)blockIdx.x * per;
    if (first >= ntiles)
        return;
    if (threadIdx.x < 64) {
        const int32_t tile = first + (int32_t)threadIdx.x;
        bool m = false;
        if ((int32_t)threadIdx.x < per && tile < ntiles) {
            const Img &im = find_img(b, tile, kTile);
            m = im.tcnt[(tile - im.tile0) * 4] == kOverflow;
        }
        const uint64_t bal = __ballot(m);
        if (threadIdx.x == 0)
            marked = bal;
    }
    __syncthreads();
    uint64_t bits = marked;
    while (bits) {
        const int i = __ffsll((unsigned long long)bits) - 1;
        bits &= bits - 1;
        scan_tile<NSR, TW, BH, ORD, kTileThreads, C, false>(b, first + i, t);
        __syncthreads();
    }
}

// ------------------------------------------------------------------------
// K2: boundary merge (Algorithm 7's boundary loop with Algorithm 8's
// merger), in two kernels (see the two-level merge below).  The work items
// are the 32-pixel segments of every shared tile edge.  The two pixel lines
// facing each other across the edge are treated as two rows of runs.  Runs are cut where a perpendicular tile edge crosses the line,
// so every run lies in one tile and belongs to one local component; then
// every pair of runs that touch (8-conn: also diagonally) is united once:
//   U1 at the first position of their overlap,
//   U2 where the earlier line's run starts just after the later line's run
//      ends (diagonal),
//   U3 where the later line's run starts just after the earlier line's run
//      ends (diagonal).
// At a cut U1 and U3 can both hold, so they are walked separately.
// ------------------------------------------------------------------------
// Foreground bits of positions from..from+31 of an edge line (from % 32 == 0,
// lines 64-byte aligned): four 16-byte loads; positions at or past n are 0.
// PARTS > 1: the PARTS adjacent lanes of a segment (lane % PARTS = its
// part) each load 32 / PARTS of the entries and combine their bits.
template <int PARTS = 1>
__device__ __forceinline__ uint32_t line_mask(const uint16_t *line, int from, int n) {
    static_assert(PARTS == 1 || PARTS == 2 || PARTS == 4, "a part is whole 16-byte loads");
    const u32x4 *q = reinterpret_cast<const u32x4 *>(line + from);
    const int k0 = PARTS == 1 ? 0 : (int)(threadIdx.x % PARTS) * (4 / PARTS);
    uint32_t m = 0;
#pragma unroll
    for (int kk = 0; kk < 4 / PARTS; kk++) {
        const int k = k0 + kk;
        const u32x4 v = q[k];
        const uint32_t d[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int bit = k * 8 + j * 2;
            m |= (uint32_t)((d[j] & 0xFFFFu) != kNone) << bit;
            m |= (uint32_t)((d[j] >> 16) != kNone) << (bit + 1);
        }
    }
#pragma unroll
    for (int x = 1; x < PARTS; x <<= 1)
        m |= (uint32_t)__shfl_xor((int)m, x, 64);
    const int left = n - from;
    return left >= 32 ? m : (left <= 0 ? 0u : m & ((1u << left) - 1u));
}

__device__ __forceinline__ bool fg_at(const uint16_t *line, int pos, int n) {
    return pos >= 0 && pos < n && line[pos] != kNone;
}

// Gray levels: the byte at position `pos` of an edge line (a tile row for a
// horizontal edge, a tile column for a vertical one); 0 outside the image.
__device__ __forceinline__ uint32_t line_byte(const Img &im, bool horiz, int fixed, int pos, int n) {
    if (pos < 0 || pos >= n)
        return 0u;
    return horiz ? im.img[(int64_t)fixed * im.stride + pos] : im.img[(int64_t)pos * im.stride + fixed];
}

// Gray levels: the 32 bytes at positions from..from+31 of an edge line (row
// `fixed` for a horizontal edge, column `fixed` for a vertical one) as 8
// dwords; 0 outside the image.
__device__ __forceinline__ void line_bytes(const Img &im, bool horiz, int fixed, int from, uint32_t *d) {
    if (horiz) {
        load_bytes(im, fixed, from, d);
        return;
    }
#pragma unroll
    for (int j = 0; j < 8; j++) {
        uint32_t w = 0u;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int pos = from + 4 * j + q;
            if (pos < im.H)
                w |= (uint32_t)im.img[(int64_t)pos * im.stride + fixed] << (8 * q);
        }
        d[j] = w;
    }
}

// threads per segment in the boundary merge's global pass (K2b) and in its
// regional pass (K2a), by run kind: row-pair runs 2 and 4, single rows and
// gray levels 4 and 8
constexpr int merge_split(int bh) { return bh == 2 ? 2 : 4; }
constexpr int region_split(int bh) { return bh == 2 ? 4 : 8; }
constexpr int kMergeBatch = 8;   // contacts whose parents K2b loads together (row-pair runs)

// The contacts of one 32-pixel segment of a shared tile edge: the segment
// starts at position `from` of the edge line between tile row (horizontal
// edge) or tile column (vertical edge) `later_t` and the one before it.  lo
// and hi are set to the later and the earlier line; cm1 bit c holds a U1
// contact at position c (partner at c), bit 32 + c a U3 contact (partner at
// c - 1); cm2 bit c a U2 contact (partner at c + 1).
template <int NSR, int TW, int BH, int PARTS = 1>
__device__ __forceinline__ void segment_contacts(const Img &im, bool horiz, int later_t, int from,
                                                 const uint16_t *&lo, const uint16_t *&hi, uint64_t &cm1,
                                                 uint32_t &cm2) {
    using G = Geo<NSR, TW, BH>;
    constexpr bool GRAY = G::GRAY;
    constexpr int TH = G::TH;
    const bool conn8 = im.conn == 8;
    int n;
    // cut[c]: a perpendicular tile edge lies between positions c-1 and c.
    // Segments start at multiples of 32 and tile sides are powers of two:
    // a side of 32 or more puts at most bit 0 in the mask, a shorter one
    // (tile heights 4, 8, 16) a bit every TH positions.
    static_assert((TW & (TW - 1)) == 0 && (TH & (TH - 1)) == 0, "tile sides are powers of two");
    constexpr uint32_t kRowCuts = TH >= 32 ? 1u : TH == 16 ? 0x00010001u : TH == 8 ? 0x01010101u : 0x11111111u;
    uint32_t cut, cutn;
    if (horiz) {
        n = im.W;
        lo = im.he + ((int64_t)later_t * 2 + 0) * im.hep;
        hi = im.he + ((int64_t)(later_t - 1) * 2 + 1) * im.hep;
        cut = from % TW == 0 ? 1u : 0u;
        cutn = (from + 32) % TW == 0 ? 0x80000000u : 0u;
    } else {
        n = im.H;
        lo = im.ve + ((int64_t)later_t * 2 + 0) * im.vep;
        hi = im.ve + ((int64_t)(later_t - 1) * 2 + 1) * im.vep;
        cut = TH >= 32 ? (from % TH == 0 ? 1u : 0u) : kRowCuts;
        cutn = TH >= 32 ? ((from + 32) % TH == 0 ? 0x80000000u : 0u) : (kRowCuts >> 1) | 0x80000000u;
    }
    const uint32_t m = line_mask<PARTS>(lo, from, n), up = line_mask<PARTS>(hi, from, n);
    const uint32_t mL = fg_at(lo, from - 1, n) ? 1u : 0u, uL = fg_at(hi, from - 1, n) ? 1u : 0u;
    const uint32_t mR = fg_at(lo, from + 32, n) ? 1u : 0u, uR = fg_at(hi, from + 32, n) ? 1u : 0u;
    const uint32_t mp = ((m << 1) | mL) & ~cut;         // same run continues from c-1
    const uint32_t upp = (up << 1) | uL;                // earlier line at c-1
    const uint32_t mn = ((m >> 1) | (mR << 31)) & ~cutn; // same run continues to c+1
    const uint32_t un = (up >> 1) | (uR << 31);          // earlier line at c+1
    const uint32_t o = m & up;
    const uint32_t u1 = o & ~(mp & upp & ~cut);
    uint32_t u2 = 0u, u3 = 0u;
    if (conn8) {
        u2 = m & ~mn & un & ~(up & ~cutn);             // earlier run starts at c+1
        u3 = m & ~mp & upp & ~(up & ~cut);             // earlier run ends at c-1
    }
    cm1 = (uint64_t)u1 | ((uint64_t)u3 << 32);  // partner at c (U1) or c-1 (U3)
    cm2 = u2;                                    // partner at c+1 (U2)
    if (GRAY) {
        // gray levels: object pixels face each other across the edge and
        // connect when their bytes are equal; every such position is a
        // contact (repeats of one component pair are skipped below)
        // The 32 bytes of each line are loaded at once (independent loads),
        // then compared four at a time: the later line with the earlier one
        // at c, c - 1 and c + 1.
        const int lo_fixed = horiz ? later_t * TH : later_t * TW;
        uint32_t lb[8], hb[8], sp[8], sn[8];
        line_bytes(im, horiz, lo_fixed, from, lb);
        line_bytes(im, horiz, lo_fixed - 1, from, hb);
        const uint32_t hprev = line_byte(im, horiz, lo_fixed - 1, from - 1, n);
        const uint32_t hnext = line_byte(im, horiz, lo_fixed - 1, from + 32, n);
#pragma unroll
        for (int j = 0; j < 8; j++) {
            sp[j] = (hb[j] << 8) | (j ? hb[j - 1] >> 24 : hprev);              // byte c: earlier line at c - 1
            sn[j] = (hb[j] >> 8) | ((j < 7 ? hb[j + 1] : hnext) << 24);        // byte c: earlier line at c + 1
        }
        const uint32_t v = m & eq32(lb, hb), d1 = m & eq32(lb, sp), d2 = m & eq32(lb, sn);
        // (an equal byte is an object pixel too, since the levels match; a
        // position outside the image reads 0, which no object byte equals)
        cm1 = (uint64_t)v | (conn8 ? ((uint64_t)(d1 & (from > 0 ? 0xFFFFFFFFu : 0xFFFFFFFEu)) << 32) : 0ull);
        cm2 = conn8 ? d2 : 0u;
    }
}

// Rem's union (the step documented above) over the contacts in cm1 / cm2 of
// the segment starting at `from`, on the packed parent array P at scope S;
// node_of(pa, pb, rx, ry) gives the nodes of the pixels at positions pa
// (later line) and pb (earlier line).  A contact joining the same two nodes
// as the previous one is skipped (long stretches of one component along an
// edge).  With LASTP the walk of a contact sharing a node with the previous
// pair starts at the node that union ended on, which lies nearer the root
// (uniting a set through any of its members is the same union), and a pair
// whose both ends map to it is done; with row-pair runs on the large
// components of dense noise that measured slower, so it is off there.
// Entries pack (key << NB) | node, so that comparing two parents compares
// their keys.
template <int S, bool LASTP, int NB, class PT, class NodeOf>
__device__ __forceinline__ void unite_contacts(PT *P, uint64_t cm1, uint32_t cm2, int from, NodeOf node_of) {
    using V = decltype(aload<S>(P));
    constexpr V NODE = NB >= 8 * (int)sizeof(V) ? ~(V)0 : (V)(((V)1 << NB) - 1);
    // flat loop: one union step per iteration, next contact when one ends
    bool busy = false;
    uint32_t rx = 0, ry = 0, lastx = 0xFFFFFFFFu, lasty = 0xFFFFFFFFu, lastp = 0xFFFFFFFFu;
    for (;;) {
        if (!busy) {
            if (!cm1 && !cm2)
                break;
            int c, d;
            if (cm1) {
                const int bit = __ffsll((unsigned long long)cm1) - 1;
                cm1 &= cm1 - 1;
                c = bit & 31;
                d = (bit >> 5) ? -1 : 0;
            } else {
                c = __ffs(cm2) - 1;
                cm2 &= cm2 - 1u;
                d = 1;
            }
            node_of(from + c, from + c + d, rx, ry);
            if (rx == lastx && ry == lasty)
                continue;
            if constexpr (LASTP) {
                const uint32_t sx = (rx == lastx || rx == lasty) ? lastp : rx;
                const uint32_t sy = (ry == lastx || ry == lasty) ? lastp : ry;
                lastx = rx;
                lasty = ry;
                if (sx == sy)
                    continue;
                rx = sx;
                ry = sy;
            } else {
                lastx = rx;
                lasty = ry;
            }
            busy = true;
        }
        const V px = aload<S>(P + rx);
        const V py = aload<S>(P + ry);
        if (px == py) {
            if constexpr (LASTP)
                lastp = (uint32_t)(px & NODE);
            busy = false;
            continue;
        }
        const bool xs = px > py;
        const uint32_t n = xs ? rx : ry;
        const V pn = xs ? px : py;
        const V seen = acas<S>(P + n, pn, xs ? py : px);
        if (seen == pn) {
            if ((uint32_t)(pn & NODE) == n) {
                if constexpr (LASTP)
                    lastp = (uint32_t)((xs ? py : px) & NODE);
                busy = false;
                continue;
            }
            rx = xs ? (uint32_t)(pn & NODE) : rx;
            ry = xs ? ry : (uint32_t)(pn & NODE);
        }
    }
}

// Takes the next contact of cm1 / cm2 (lowest bit first): position c and
// partner offset d.  Returns false when there is none.
__device__ __forceinline__ bool next_contact(uint64_t &cm1, uint32_t &cm2, int &c, int &d) {
    if (cm1) {
        const int bit = __ffsll((unsigned long long)cm1) - 1;
        cm1 &= cm1 - 1;
        c = bit & 31;
        d = (bit >> 5) ? -1 : 0;
        return true;
    }
    if (cm2) {
        c = __ffs(cm2) - 1;
        cm2 &= cm2 - 1u;
        d = 1;
        return true;
    }
    return false;
}

// As unite_contacts, for the device-scope pass: the first MAXC contacts
// (repeats of the previous node pair skipped) have their two parents loaded
// together, one round trip for all of them instead of one per union; a
// contact whose parents are equal is done, and one whose parent pair repeats
// the previous union's is skipped (its nodes are in those two sets, now one).
// The others are united from their parents (the same union: parents lie in
// their children's sets).  Contacts beyond the first MAXC go through
// unite_contacts.
template <int S, int NB, int MAXC, class PT, class NodeOf>
__device__ __forceinline__ void unite_contacts_batched(PT *P, uint64_t cm1, uint32_t cm2, int from, NodeOf node_of) {
    using V = decltype(aload<S>(P));
    constexpr V NODE = NB >= 8 * (int)sizeof(V) ? ~(V)0 : (V)(((V)1 << NB) - 1);
    uint32_t ax[MAXC], ay[MAXC];
    bool have[MAXC];
    uint32_t lx = 0xFFFFFFFFu, ly = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < MAXC; i++) {
        have[i] = false;
        int c, d;
        while (next_contact(cm1, cm2, c, d)) {
            uint32_t rx, ry;
            node_of(from + c, from + c + d, rx, ry);
            if (rx == lx && ry == ly)
                continue;
            lx = rx;
            ly = ry;
            ax[i] = rx;
            ay[i] = ry;
            have[i] = true;
            break;
        }
    }
    V px[MAXC], py[MAXC];
#pragma unroll
    for (int i = 0; i < MAXC; i++)
        if (have[i]) {
            px[i] = aload<S>(P + ax[i]);
            py[i] = aload<S>(P + ay[i]);
        }
    uint32_t qx = 0xFFFFFFFFu, qy = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < MAXC; i++) {
        if (!have[i] || px[i] == py[i])
            continue;
        uint32_t rx = (uint32_t)(px[i] & NODE), ry = (uint32_t)(py[i] & NODE);
        if (rx == qx && ry == qy)
            continue;
        qx = rx;
        qy = ry;
        for (;;) {
            const V vx = aload<S>(P + rx);
            const V vy = aload<S>(P + ry);
            if (vx == vy)
                break;
            const bool xs = vx > vy;
            const uint32_t n = xs ? rx : ry;
            const V pn = xs ? vx : vy;
            const V seen = acas<S>(P + n, pn, xs ? vy : vx);
            if (seen == pn) {
                if ((uint32_t)(pn & NODE) == n)
                    break;
                rx = xs ? (uint32_t)(pn & NODE) : rx;
                ry = xs ? ry : (uint32_t)(pn & NODE);
            }
        }
    }
    if (cm1 || cm2)
        unite_contacts<S, false, NB>(P, cm1, cm2, from, node_of);
}

// Keeps part `part` of `parts` equal parts of a segment's positions.
__device__ __forceinline__ void keep_part(uint64_t &cm1, uint32_t &cm2, int part, int parts) {
    if (parts > 1) {
        const int w = 32 / parts;
        const uint32_t hm = ((1u << w) - 1u) << (part * w);
        cm1 &= (uint64_t)hm | ((uint64_t)hm << 32);
        cm2 &= hm;
    }
}

// ------------------------------------------------------------------------
// The boundary merge in two levels.  Tiles are grouped into regions of RY x
// RX tiles (region_ry / region_rx: 4 x 2, or 4 x 1 for gray levels and
// 512-wide tiles; RY * TH is a multiple of 32, so that every
// 32-pixel segment of a vertical edge lies in one region row).  K2a unites
// the contacts whose two pixels lie in one region on a union-find in LDS, one
// workgroup per region, and stores the result in the global array: every
// boundary component whose set has another member gets that set's
// smallest-key member as its parent (a valid state of the global array:
// parents only point to smaller keys of the same set).  K2b then unites the
// remaining contacts, those across region borders (with 8-connectivity also
// the diagonal ones at a region's corners), with the device-scope Rem steps.
// Fewer device-scope atomics: with 4 x 2 tiles about 70% of the shared-edge
// pixels lie inside a region.
// ------------------------------------------------------------------------
// (gray levels: one tile column per region measured faster)
constexpr int region_rx(int tw, int bh) { return bh == 0 || tw > 256 ? 1 : 2; }
constexpr int region_ry(int th) { return th >= 8 ? 4 : 32 / th; }
static_assert(region_ry(4) * 4 % 32 == 0 && region_ry(8) * 8 % 32 == 0, "region rows: a multiple of 32");
constexpr int bits_for(int n) { return n <= 1 ? 0 : 1 + bits_for((n + 1) / 2); }   // ceil(log2 n)

template <int NSR, int TW, int BH>
__host__ __device__ constexpr int region_period(bool horiz) {
    return horiz ? TW * region_rx(TW, BH) : Geo<NSR, TW, BH>::TH * region_ry(Geo<NSR, TW, BH>::TH);
}

// rs bit c: a region edge lies between positions from + c - 1 and from + c;
// re bit c: between from + c and from + c + 1 (period: region size along the
// line, at least 32, so each mask has at most one bit).
__device__ __forceinline__ void region_bits(int from, int period, uint32_t &rs, uint32_t &re) {
    const int m = from % period;
    const int cs = m == 0 ? 0 : period - m, ce = period - 1 - m;
    rs = cs < 32 ? 1u << cs : 0u;
    re = ce < 32 ? 1u << ce : 0u;
}

// One segment of a region's inner edges (K2a): its line, start, the region
// tiles of its first later-line and earlier-line pixel, and its contacts.
struct RegionSeg {
    const uint16_t *lo, *hi;
    uint64_t cm1;
    uint32_t cm2;
    int from, jl, jh;
    bool horiz;
};

// Item `item` of a region (MS items per segment): the horizontal edges
// between the region's tile rows (each tile column's TW / 32 segments) come
// first, then the vertical edges between its tile columns (the region's
// rows, in 32-row segments).  Contacts whose partner lies outside the region
// are dropped.
// (The region: tile rows ty0 .. ty0 + nty - 1, columns tx0 .. tx0 + ntx - 1;
// nh segments along each inner horizontal edge, nvs along each vertical one,
// its first row row0.)
template <int NSR, int TW, int BH, int MS>
__device__ __forceinline__ RegionSeg region_segment(const Img &im, int item, int ty0, int tx0, int nty, int ntx,
                                                    int nh, int nvs, int row0) {
    RegionSeg g;
    int k = item / MS, later_t;
    if (k < (nty - 1) * nh) {
        const int tb = 1 + k / nh, c = (k % nh) / (TW / 32);
        g.horiz = true;
        later_t = ty0 + tb;
        g.from = (tx0 * (TW / 32) + k % nh) << 5;
        g.jl = tb * ntx + c;
        g.jh = (tb - 1) * ntx + c;
    } else {
        k -= (nty - 1) * nh;
        const int cb = 1 + k / nvs;
        g.horiz = false;
        later_t = tx0 + cb;
        g.from = row0 + ((k % nvs) << 5);
        g.jl = cb;
        g.jh = cb - 1;
    }
    segment_contacts<NSR, TW, BH, (MS < 4 ? MS : 4)>(im, g.horiz, later_t, g.from, g.lo, g.hi, g.cm1, g.cm2);
    uint32_t rs, re;
    region_bits(g.from, region_period<NSR, TW, BH>(g.horiz), rs, re);
    g.cm1 &= ~((uint64_t)rs << 32);   // U3 partners left of / above the region
    g.cm2 &= ~re;                     // U2 partners right of / below it
    keep_part(g.cm1, g.cm2, item % MS, MS);
    return g;
}

// K2a.  Node j * CAP + b of the LDS array is boundary component b of the
// region's tile j (row-major); its entry packs (key << NB) | parent node,
// where the key is the component's first pixel as a raster index inside the
// region (canonical order; the order of the image's raster indices among
// the region's pixels) or the node itself (provisional order: tiles, then
// boundary index, as the global ids).
template <int NSR, int TW, int BH, int ORD>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_merge_local(Batch b) {
    using G = Geo<NSR, TW, BH>;
    constexpr int TH = G::TH, CAP = G::CAP, RX = region_rx(TW, BH), RY = region_ry(TH), NTR = RX * RY;
    constexpr int NN = NTR * CAP, RW = RX * TW;
    constexpr int NB = bits_for(NN), KB = ORD == kCanonical ? bits_for(RY * TH * RW) : NB;
    static_assert(NB + KB <= 32, "packed region entries fit 32 bits");
    constexpr int WG = __HIP_MEMORY_SCOPE_WORKGROUP;
    constexpr int MS = region_split(BH);
    __shared__ uint32_t P[NN];
    __shared__ int32_t nb[NTR];
    const int tid = threadIdx.x;
    const Img &im = find_img(b, blockIdx.x, kRegion);
    const int r = blockIdx.x - im.region0;
    const int nrx = (im.NTX + RX - 1) / RX;
    const int ty0 = (r / nrx) * RY, tx0 = (r % nrx) * RX;
    const int nty = min(RY, im.NTY - ty0), ntx = min(RX, im.NTX - tx0), nt = nty * ntx;
    const int NTX = im.NTX;
    const int nxs = (im.W + 31) >> 5;
    const int hl = min(TW / 32, nxs - (tx0 + ntx - 1) * (TW / 32));   // segments of the last tile column
    const int nh = (ntx - 1) * (TW / 32) + hl;
    const int row0 = ty0 * TH, row1 = min((ty0 + nty) * TH, im.H);
    const int nvs = (row1 + 31) / 32 - row0 / 32;
    const int items = MS * ((nty - 1) * nh + (ntx - 1) * nvs);
    // loads: counts, keys (two at a time: CAP is even, so a pair lies in one
    // tile), the first segment's lines
    static_assert(CAP % 2 == 0, "key pairs");
    // region tile j -> (row, column) inside the region (division by RX
    // at compile time when the region is full width)
    auto jrow = [&](int j) { return ntx == RX ? j / RX : j; };
    auto jcol = [&](int j) { return ntx == RX ? j % RX : 0; };
    if (tid < nt)
        nb[tid] = im.tcnt[((ty0 + jrow(tid)) * NTX + tx0 + jcol(tid)) * 4 + 2];
    constexpr int KPT = (NN / 2 + kThreads - 1) / kThreads;
    uint32_t kv[KPT];
    const CCL_GLOBAL uint32_t *bkey2 = reinterpret_cast<const CCL_GLOBAL uint32_t *>(im.bkey);
#pragma unroll
    for (int i = 0; i < KPT; i++) {
        const int e = 2 * (tid + i * kThreads), j = e / CAP;
        kv[i] = 0u;
        if (ORD == kCanonical && e < nt * CAP)
            kv[i] = bkey2[((int64_t)((ty0 + jrow(j)) * NTX + tx0 + jcol(j)) * CAP + e % CAP) >> 1];
    }
#pragma unroll
    for (int i = 0; i < KPT; i++) {
        const int e = 2 * (tid + i * kThreads), j = e / CAP;
        if (e < NN) {
#pragma unroll
            for (int h = 0; h < 2; h++) {
                uint32_t key = (uint32_t)(e + h);
                if (ORD == kCanonical) {
                    const int kk = (int)((kv[i] >> (16 * h)) & 0xFFFFu);
                    key = (uint32_t)((jrow(j) * TH + kk / TW) * RW + jcol(j) * TW + kk % TW);
                }
                P[e + h] = (key << NB) | (uint32_t)(e + h);
            }
        }
    }
    __syncthreads();
    for (int item = tid; item < items; item += kThreads) {
        const RegionSeg g = region_segment<NSR, TW, BH, MS>(im, item, ty0, tx0, nty, ntx, nh, nvs, row0);
        const uint16_t *lo = g.lo, *hi = g.hi;
        const int jl = g.jl - (g.horiz ? g.from / TW : ty0 * ntx), jh = g.jh - (g.horiz ? g.from / TW : ty0 * ntx);
        const bool horiz = g.horiz;
        unite_contacts<WG, BH != 2, NB>(P, g.cm1, g.cm2, g.from, [=](int pa, int pb, uint32_t &rx, uint32_t &ry) {
            const int da = horiz ? pa / TW : (pa / TH) * ntx, db = horiz ? pb / TW : (pb / TH) * ntx;
            rx = (uint32_t)((jl + da) * CAP + lo[pa]);
            ry = (uint32_t)((jh + db) * CAP + hi[pb]);
        });
    }
    __syncthreads();
    // every node that is not its set's root gets the root (the set's
    // smallest key) as its global parent
    constexpr uint32_t NODE = (1u << NB) - 1u;
    for (int e = tid; e < nt * CAP; e += kThreads) {
        const int j = e / CAP;
        if (e % CAP >= nb[j])
            continue;
        uint32_t q = (uint32_t)e, pv = P[q];
        while ((pv & NODE) != q) {
            q = pv & NODE;
            pv = P[q];
        }
        if (q == (uint32_t)e)
            continue;
        const int jq = (int)q / CAP;
        const uint32_t qid = (uint32_t)(((ty0 + jrow(jq)) * NTX + tx0 + jcol(jq)) * CAP + (int)q % CAP);
        uint64_t key = qid;
        if (ORD == kCanonical) {
            const uint32_t lk = pv >> NB;
            key = (uint64_t)(row0 + (int)(lk / RW)) * (uint64_t)im.W + (uint64_t)(tx0 * TW + (int)(lk % RW));
        }
        im.uf[(int64_t)((ty0 + jrow(j)) * NTX + tx0 + jcol(j)) * CAP + e % CAP] = (key << 32) | qid;
    }
}

// K2b: the contacts left by K2a, merge_split(BH) items per 32-pixel segment
// of every shared tile edge (segments wholly inside a region end at once).
template <int NSR, int TW, int BH>
__global__ __launch_bounds__(kThreads) void k_merge(Batch b) {
    using G = Geo<NSR, TW, BH>;
    constexpr int TH = G::TH, RX = region_rx(TW, BH), RY = region_ry(TH);
    // MS threads per 32-pixel segment, each taking 32 / MS of its positions:
    // the longest chains of dependent union steps get MS times shorter (the
    // contacts at the parts' seams may repeat a union; the edge lines are
    // loaded once, a part by each thread)
    constexpr int MS = merge_split(BH);
    const int32_t item2 = blockIdx.x * kThreads + threadIdx.x;
    const int32_t item = item2 / MS;
    const Img &im = find_img(b, item, kEdge);
    int32_t e = item - im.edge0;
    const int32_t nxs = (im.W + 31) >> 5, nys = (im.H + 31) >> 5;
    const int32_t nH = (im.NTY - 1) * nxs, nV = (im.NTX - 1) * nys;
    if (e < 0 || e >= nH + nV)
        return;
    const bool horiz = e < nH;
    if (!horiz)
        e -= nH;
    const int32_t per = horiz ? nxs : nys;
    const int later_t = 1 + e / per, earlier_t = later_t - 1, from = (e % per) << 5;
    // on an edge inside a region only the diagonal contacts across the
    // region's border are left
    uint64_t keep1 = ~0ull;
    uint32_t keep2 = ~0u;
    if (horiz ? later_t % RY != 0 : later_t % RX != 0) {
        if (im.conn != 8)
            return;
        uint32_t rs, re;
        region_bits(from, region_period<NSR, TW, BH>(horiz), rs, re);
        if (!(rs | re))
            return;
        keep1 = (uint64_t)rs << 32;
        keep2 = re;
    }
    const uint16_t *lo, *hi;
    uint64_t cm1;
    uint32_t cm2;
    segment_contacts<NSR, TW, BH, (MS < 4 ? MS : 4)>(im, horiz, later_t, from, lo, hi, cm1, cm2);
    cm1 &= keep1;
    cm2 &= keep2;
    keep_part(cm1, cm2, item2 & (MS - 1), MS);
    constexpr int AG = __HIP_MEMORY_SCOPE_AGENT;
    const int NTX = im.NTX;
    const auto node_of = [&](int pa, int pb, uint32_t &rx, uint32_t &ry) {
        if (horiz) {
            rx = (uint32_t)(((int64_t)later_t * NTX + pa / TW) * G::CAP + lo[pa]);
            ry = (uint32_t)(((int64_t)earlier_t * NTX + pb / TW) * G::CAP + hi[pb]);
        } else {
            rx = (uint32_t)(((int64_t)(pa / TH) * NTX + later_t) * G::CAP + lo[pa]);
            ry = (uint32_t)(((int64_t)(pb / TH) * NTX + earlier_t) * G::CAP + hi[pb]);
        }
    };
    // row pairs: parents of a batch of contacts loaded together; single rows
    // and gray levels: the walk from the last union's node (LASTP)
    if constexpr (BH == 2)
        unite_contacts_batched<AG, 32, kMergeBatch>(im.uf, cm1, cm2, from, node_of);
    else
        unite_contacts<AG, true, 32>(im.uf, cm1, cm2, from, node_of);
}

// ------------------------------------------------------------------------
// K3a: flatten the boundary components of one tile; a component that is its
// set's root owns the set's first raster pixel.  Adds those roots to the
// segment counts and turns their "interior roots before" into the offset
// inside their row segment.  One wave per tile (kWaves tiles per
// workgroup): the kernel is bound by the latency of its dependent loads, so
// many tiles in flight matter more than many lanes per tile.
// ------------------------------------------------------------------------
template <int NSR, int TW, int BH>
__global__ __launch_bounds__(kThreads) void k_flatten(Batch b, int32_t ntiles) {
    using G = Geo<NSR, TW, BH>;
    constexpr int NW = G::NW, TH = G::TH;
    constexpr int CW = (G::CAP + 31) / 32;
    __shared__ uint32_t RKs[kWaves][G::NM];
    __shared__ uint32_t RBs[kWaves][CW];   // boundary component j is its set's root (bit)
    __shared__ int32_t rowcs[kWaves][TH];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = blockIdx.x * kWaves + wv;
    if (tile >= ntiles)
        return;
    const Img &im = find_img(b, tile, kTile);
    const int ti = tile - im.tile0;
    const int n = im.tcnt[ti * 4 + 2];
    if (n == 0)
        return;
    uint32_t *RK = RKs[wv], *RB = RBs[wv];
    int32_t *rowc = rowcs[wv];
    const int ty = ti / im.NTX, tx = ti % im.NTX;
    const int y0 = ty * TH;
    for (int i = lane; i < G::NM; i += 64)
        RK[i] = 0u;
    for (int i = lane; i < CW; i += 64)
        RB[i] = 0u;
    for (int r = lane; r < TH; r += 64)
        rowc[r] = 0;
    wave_sync();
    const int64_t cbase = (int64_t)ti * G::CAP;
    // flat loop: every lane walks its components' parent chains one load per
    // iteration, without waiting for other lanes' longer chains; the walk's
    // end (the root entry) is written back to the component's own entry.
    // All unions are done (previous kernel), so plain loads suffice: an entry
    // read before another workgroup's write-back still points up the same
    // tree, and roots never change here.
    int j = lane;
    uint32_t r = (uint32_t)(cbase + j);
    while (j < n) {
        const uint64_t v = im.uf[r];
        if ((uint32_t)v != r) {
            r = (uint32_t)v;
            continue;
        }
        const uint32_t id = (uint32_t)(cbase + j);
        const bool is = r == id;
        if (!is)
            im.uf[id] = v;
        if (is) {
            const int key = im.bkey[id];
            atomicOr(&RB[j >> 5], 1u << (j & 31));
            atomicOr(&RK[key >> 5], 1u << (key & 31));
            atomicAdd(&rowc[key / TW], 1);
        }
        j += 64;
        r = (uint32_t)(cbase + j);
    }
    wave_sync();
    for (int j = lane; j < n; j += 64) {
        const uint32_t id = (uint32_t)(cbase + j);
        if ((RB[j >> 5] >> (j & 31)) & 1u) {
            const int key = im.bkey[id];
            im.bval[id] += popc_before(&RK[(key / TW) * NW], key % TW);
        }
    }
    for (int r = lane; r < TH; r += 64)
        if (rowc[r] && y0 + r < im.H)
            im.seg[(int64_t)(y0 + r) * im.NTX + tx] += rowc[r];
}

// ------------------------------------------------------------------------
// K3a, provisional order: flatten the boundary components of one tile (as
// above), then number the tile's roots -- its interior components and the
// boundary components that are their set's root -- in component order.
// seg[tile] gets the tile's root count; each local component's slot in cf
// gets its rank among the tile's roots (a root) or ~(id of its set's root)
// (a boundary component that is not a root), for the component-label
// kernel.  One wave per tile, as above.
// ------------------------------------------------------------------------
template <int NSR, int TW, int BH>
__global__ __launch_bounds__(kThreads) void k_flatten_prov(Batch b, int32_t ntiles) {
    using G = Geo<NSR, TW, BH>;
    __shared__ uint32_t CBs[kWaves][G::RW];   // boundary components (bit per component)
    __shared__ int32_t CPs[kWaves][G::RW];    // popcount prefix of CB
    __shared__ uint32_t RBs[kWaves][G::RW];   // roots (bit per component)
    __shared__ int32_t RPs[kWaves][G::RW];    // popcount prefix of RB
    __shared__ uint32_t RIDs[kWaves][G::CAP]; // id of the set root of each boundary component
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = blockIdx.x * kWaves + wv;
    if (tile >= ntiles)
        return;
    const Img &im = find_img(b, tile, kTile);
    const int ti = tile - im.tile0;
    const int n_comp = im.tcnt[ti * 4 + 1], n = im.tcnt[ti * 4 + 2];
    const int ncw = (n_comp + 31) >> 5;
    uint32_t *CB = CBs[wv], *RB = RBs[wv], *RID = RIDs[wv];
    int32_t *CP = CPs[wv], *RP = RPs[wv];
    const uint32_t *gcb = im.cb + (int64_t)ti * G::RW;
    for (int i = lane; i < ncw; i += 64)
        CB[i] = gcb[i];
    const int64_t cbase = (int64_t)ti * G::CAP;
    // find the set root of every boundary component (all unions are done:
    // plain loads, as in the canonical form); kept in LDS, so that the
    // lanes below read what other lanes found
    int j = lane;
    uint32_t r = (uint32_t)(cbase + j);
    while (j < n) {
        const uint64_t v = im.uf[r];
        if ((uint32_t)v != r) {
            r = (uint32_t)v;
            continue;
        }
        RID[j] = r;
        j += 64;
        r = (uint32_t)(cbase + j);
    }
    wave_sync();
    wave_popcount_prefix(CB, CP, ncw, lane);
    wave_sync();
    // root bitmap: interior components, and boundary components that are
    // their set's root; one wave ballot covers two words
    for (int c0 = 0; c0 < n_comp; c0 += 64) {
        const int c = c0 + lane;
        bool root = false;
        if (c < n_comp) {
            root = true;
            if ((CB[c >> 5] >> (c & 31)) & 1u) {
                const int32_t jb = rank_of(CB, CP, c);
                root = RID[jb] == (uint32_t)(cbase + jb);
            }
        }
        const uint64_t bal = __ballot(root);
        if (lane == 0)
            RB[c0 >> 5] = (uint32_t)bal;
        if (lane == 32 && (c0 >> 5) + 1 < G::RW)
            RB[(c0 >> 5) + 1] = (uint32_t)(bal >> 32);
    }
    wave_sync();
    const int32_t roots = wave_popcount_prefix(RB, RP, ncw, lane);
    wave_sync();
    int32_t *gcf = im.cf + (int64_t)ti * G::RCAP;
    for (int c = lane; c < n_comp; c += 64) {
        const bool root = (RB[c >> 5] >> (c & 31)) & 1u;
        const bool bnd = (CB[c >> 5] >> (c & 31)) & 1u;
        if (root) {
            const int32_t k = rank_of(RB, RP, c);
            gcf[c] = k;
            if (bnd)
                im.bval[cbase + rank_of(CB, CP, c)] = k;
        } else {
            gcf[c] = ~(int32_t)RID[rank_of(CB, CP, c)];
        }
    }
    if (lane == 0)
        im.seg[ti] = roots;
}

// ------------------------------------------------------------------------
// K4a / K4b: exclusive scan of the segment counts in raster order.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_scan_blocks(Batch b) {
    const Img &im = find_img(b, blockIdx.x, kScan);
    const int c = blockIdx.x - im.scan0;
    const int64_t L = im.nseg;
    static_assert(kScanChunk == 4 * kThreads, "four counts per thread");
    // four consecutive counts per thread, one 16-byte load where all four
    // lie in the array (the array starts 256-byte aligned)
    const int64_t base = (int64_t)c * kScanChunk + threadIdx.x * 4;
    int32_t v[4];
    if (base + 3 < L) {
        const i32x4 q = *reinterpret_cast<const CCL_GLOBAL i32x4 *>(im.seg + base);
        v[0] = q.x;
        v[1] = q.y;
        v[2] = q.z;
        v[3] = q.w;
    } else {
#pragma unroll
        for (int i = 0; i < 4; i++)
            v[i] = (base + i < L) ? im.seg[base + i] : 0;
    }
    const int32_t sum = v[0] + v[1] + v[2] + v[3];
    int32_t total;
    int32_t run = block_exclusive_scan<kThreads>(sum, &total);
    int32_t o[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        o[i] = run;
        run += v[i];
    }
    if (base + 3 < L) {
        i32x4 q;
        q.x = o[0];
        q.y = o[1];
        q.z = o[2];
        q.w = o[3];
        *reinterpret_cast<CCL_GLOBAL i32x4 *>(im.seg + base) = q;
    } else {
#pragma unroll
        for (int i = 0; i < 4; i++)
            if (base + i < L)
                im.seg[base + i] = o[i];
    }
    if (threadIdx.x == 0)
        im.blk[c] = total;
}

__global__ __launch_bounds__(kThreads) void k_scan_top(Batch b) {
    const Img &im = (b.n == 1) ? b.one : b.tab[blockIdx.x];
    // four block totals per thread and step
    int32_t carry = 0;
    for (int base = 0; base < im.nblk; base += 4 * kThreads) {
        const int i = base + 4 * threadIdx.x;
        int32_t v[4];
#pragma unroll
        for (int k = 0; k < 4; k++)
            v[k] = i + k < im.nblk ? im.blk[i + k] : 0;
        int32_t total;
        int32_t ex = carry + block_exclusive_scan<kThreads>(v[0] + v[1] + v[2] + v[3], &total);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if (i + k < im.nblk)
                im.blk[i + k] = ex;
            ex += v[k];
        }
        carry += total;
    }
    if (threadIdx.x == 0 && im.ncomp)
        *im.ncomp = carry;
}

// ------------------------------------------------------------------------
// K4c: final label of every local component of a tile, stored in its table.
//   label(root of a set) = 1 + roots before its row segment + its offset
//   inside the segment (both known after K3a and K4), computable from any
//   tile, so a non-root boundary component reads its root's entries
//   directly; interior components are ranked inside their row segment
//   among the segment's roots (interior and boundary).  One wave per tile,
//   as in K3a.
// ------------------------------------------------------------------------
template <int NSR, int TW, int BH>
__device__ __forceinline__ int32_t segment_base(const Img &im, int tile, int key) {
    constexpr int TH = Geo<NSR, TW, BH>::TH;
    const int ty = tile / im.NTX, tx = tile % im.NTX;
    const int64_t sg = (int64_t)(ty * TH + key / TW) * im.NTX + tx;
    return im.seg[sg] + im.blk[sg / kScanChunk];
}

template <int NSR, int TW, int BH>
__global__ __launch_bounds__(kThreads) void k_comp_labels(Batch b, int32_t ntiles) {
    using G = Geo<NSR, TW, BH>;
    constexpr int NW = G::NW, TH = G::TH;
    __shared__ uint32_t BFBs[kWaves][G::RW];
    __shared__ int32_t BFPs[kWaves][G::RW];
    __shared__ uint32_t RMs[kWaves][G::NM];   // keys of the segment roots (bit per pixel)
    __shared__ int32_t rowbases[kWaves][TH];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = blockIdx.x * kWaves + wv;
    if (tile >= ntiles)
        return;
    uint32_t *BFB = BFBs[wv], *RM = RMs[wv];
    int32_t *BFP = BFPs[wv], *rowbase = rowbases[wv];
    const Img &im = find_img(b, tile, kTile);
    const int ti = tile - im.tile0;
    const int ty = ti / im.NTX;
    const int y0 = ty * TH;
    const int n_comp = im.tcnt[ti * 4 + 1];
    const int ncw = (n_comp + 31) >> 5;
    const uint32_t *gcb = im.cb + (int64_t)ti * G::RW;
    for (int i = lane; i < ncw; i += 64)
        BFB[i] = gcb[i];
    for (int i = lane; i < G::NM; i += 64)
        RM[i] = 0u;
    for (int r = lane; r < TH; r += 64)
        rowbase[r] = (y0 + r < im.H) ? segment_base<NSR, TW, BH>(im, ti, r * TW) : 0;
    wave_sync();
    wave_popcount_prefix(BFB, BFP, ncw, lane);
    wave_sync();
    // each slot holds the component's key until this kernel writes its label
    int32_t *gcf = im.cf + (int64_t)ti * G::RCAP;
    const int32_t *gck = gcf;
    const int64_t cbase = (int64_t)ti * G::CAP;
    // boundary components: label from the scan (roots) or from the root's
    // entries; every root's key goes into RM
    // (after the flatten a boundary component's entry holds its set's root,
    // itself for a root: one load tells both)
    auto first = [&](int c, int key) {
        if ((BFB[c >> 5] >> (c & 31)) & 1u) {
            const uint32_t id = (uint32_t)(cbase + rank_of(BFB, BFP, c));
            const uint32_t rid = (uint32_t)im.uf[id];
            if (rid == id) {
                gcf[c] = 1 + rowbase[key / TW] + im.bval[id];
                atomicOr(&RM[key >> 5], 1u << (key & 31));
            } else {
                gcf[c] = 1 + segment_base<NSR, TW, BH>(im, (int)(rid / G::CAP), im.bkey[rid]) + im.bval[rid];
            }
        } else {
            atomicOr(&RM[key >> 5], 1u << (key & 31));
        }
    };
    // interior components: ranked among the roots of their row segment
    auto second = [&](int c, int key) {
        if (!((BFB[c >> 5] >> (c & 31)) & 1u)) {
            const int kr = key / TW;
            gcf[c] = 1 + rowbase[kr] + popc_before(&RM[kr * NW], key % TW);
        }
    };
    // the keys of a lane's first KR components are loaded at once and kept
    // in registers for both passes (more overlap of the load latency)
    constexpr int KR = 8;
    int32_t kreg[KR];
#pragma unroll
    for (int i = 0; i < KR; i++) {
        const int c = lane + i * 64;
        kreg[i] = c < n_comp ? gck[c] : 0;
    }
#pragma unroll
    for (int i = 0; i < KR; i++) {
        const int c = lane + i * 64;
        if (c < n_comp)
            first(c, kreg[i]);
    }
    for (int c = lane + KR * 64; c < n_comp; c += 64)
        first(c, gck[c]);
    wave_sync();
#pragma unroll
    for (int i = 0; i < KR; i++) {
        const int c = lane + i * 64;
        if (c < n_comp)
            second(c, kreg[i]);
    }
    for (int c = lane + KR * 64; c < n_comp; c += 64)
        second(c, gck[c]);
}

// ------------------------------------------------------------------------
// K4c, provisional order: final label of every local component.  A root's
// label is 1 + the roots of the tiles before its tile (the scan of the
// per-tile counts) + its rank in its tile; a boundary component that is not
// a root takes its set root's label, computed the same way from the root's
// tile and rank.  One wave per tile.
// ------------------------------------------------------------------------
template <int NSR, int TW, int BH>
__global__ __launch_bounds__(kThreads) void k_comp_labels_prov(Batch b, int32_t ntiles) {
    using G = Geo<NSR, TW, BH>;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = blockIdx.x * kWaves + wv;
    if (tile >= ntiles)
        return;
    const Img &im = find_img(b, tile, kTile);
    const int ti = tile - im.tile0;
    const int n_comp = im.tcnt[ti * 4 + 1];
    const int32_t base = 1 + im.seg[ti] + im.blk[ti / kScanChunk];
    int32_t *gcf = im.cf + (int64_t)ti * G::RCAP;
    for (int c = lane; c < n_comp; c += 64) {
        const int32_t v = gcf[c];
        if (v >= 0) {
            gcf[c] = base + v;
        } else {
            const uint32_t rid = ~(uint32_t)v;
            const int rt = (int)(rid / G::CAP);
            gcf[c] = 1 + im.seg[rt] + im.blk[rt / kScanChunk] + im.bval[rid];
        }
    }
}

// ------------------------------------------------------------------------
// K5: labeling pass.  Rebuild the node numbering from the stored bitmask,
// look every pixel's label up through its node and component, write all pixels with
// 16-byte stores.
// ------------------------------------------------------------------------
template <int NSR, int TW, int BH>
struct RelabelLds : RunLds<NSR, TW, BH> {
    using G = Geo<NSR, TW, BH>;
    static constexpr bool GRAY = G::GRAY;
    int32_t CF[G::RCAP];    // final label of each local component
    int32_t RF[G::RCAP];    // final label of each node
    uint32_t E[GRAY ? G::NM : 1];  // gray levels: same value as the left neighbour
};

// Label stores.  Buffer stores with the tile's first row as base: a lane
// whose pixels lie right of the image, or whose row lies below it, gets an
// offset past the buffer's size and its store is dropped by the hardware.
// Every wave so issues the same, fixed number of stores per tile, with no
// branch around them, so the compiler can wait for the next tile's table
// loads (issued before the stores) without waiting for the stores too.
//   kStore16: W % 4 == 0 and 16-byte aligned labels; one 16-byte store per
//             lane covers four adjacent pixels.
//   kStore4:  any width or alignment; four 4-byte stores per lane, lane L
//             taking pixels L, L + 64, ... of the row segment, so that each
//             store instruction writes 64 adjacent pixels.  Plain (cached)
//             stores: a row segment that does not start on a cache line
//             shares its first and last lines with the neighbouring tiles,
//             which the workgroups of the same XCD label at the same time,
//             and the L2 merges the parts (nontemporal partial lines were
//             1.4x slower).
//   kStoreAny: plain stores (images wider than kVecMaxW).
// A batch's images are ordered by store form inside their launch group, so
// each form's tiles are one range [tbeg, tbeg + ntiles) of the group's tile
// numbering, labeled by a launch of that form.
typedef __attribute__((address_space(4))) const int32_t ConstI32;
constexpr int kBufferWord3 = 0x00020000;  // raw 32-bit buffer (gfx9 descriptor word 3)
constexpr uint32_t kDropped = 0x80000000u;  // offset past every buffer this kernel builds (>= its size)
// cache policy of the 16-byte label stores: nontemporal (nt) at system
// coherence scope (sc1); measured ~2% faster than nt alone, cached stores
// ~8% slower.  (The 4-byte form keeps cached stores: with sc1 its partial
// lines are no longer merged in the L2, 12% slower on the batch.)
constexpr int kStoreNtSc1 = 2 | 16;

enum StoreForm { kStoreAny = 0, kStore4 = 1, kStore16 = 2 };

template <int NSR, int TW, int BH, int STORE>
__global__ __launch_bounds__(kTileThreads) void k_relabel(Batch b, int32_t tbeg, int32_t ntiles) {
    using G = Geo<NSR, TW, BH>;
    constexpr bool GRAY = G::GRAY;
    constexpr int NW = G::NW, TH = G::TH;
    constexpr int NT = kTileThreads;
    constexpr int MPT = (G::NM + NT - 1) / NT;
    // table entries prefetched per thread: node pairs (two u16 entries per
    // load) and components; a tile with more nodes or components loads the
    // rest when it is labeled (rare: dense noise has ~1/10 of the capacity)
    constexpr int PJ = G::RB == 2 ? 2 : 3, CJ = G::RB == 2 ? 1 : 2;
    static_assert(CJ * NT <= G::RCAP, "prefetched component slots lie in the table");
    __shared__ RelabelLds<NSR, TW, BH> t;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    // Persistent: each workgroup walks tiles blockIdx.x, +gridDim.x, ...
    // While a tile's labels are stored, the next tile's mask and tables are
    // already in flight into registers; they move into LDS once every wave
    // is done with the current tile.  The node and component counts (which
    // size the table loads) are read one tile further ahead, by scalar loads.
    uint32_t pm[MPT];
    uint32_t pe[GRAY ? MPT : 1];
    uint32_t prt[PJ];   // node pairs 2q, 2q+1 (q = tid + j * NT): components, packed
    int32_t pcf[CJ];
    int pn_runs = 0, pn_comp = 0;   // counts of the tile whose tables are in registers
    int qn_runs = 0, qn_comp = 0;   // counts of the tile after it
    auto tile_of = [&](int slot) { return tbeg + (STORE == kStore4 ? xcd_tile(slot, ntiles) : slot); };
    auto counts = [&](int slot) {
        if (slot < ntiles) {
            const int tile = tile_of(slot);
            const Img &im = find_img(b, tile, kTile);
            const ConstI32 *tc = (const ConstI32 *)(uintptr_t)(im.tcnt + (tile - im.tile0) * 4);
            qn_runs = tc[0];
            qn_comp = tc[1];
        }
    };
    auto fetch = [&](int slot) {
        const int tile = tile_of(slot);
        const Img &im = find_img(b, tile, kTile);
        const int ti = tile - im.tile0;
        pn_runs = qn_runs;
        pn_comp = qn_comp;
        const uint32_t *gmask = im.masks + (int64_t)ti * G::NM * (GRAY ? 2 : 1);
#pragma unroll
        for (int k = 0; k < MPT; k++) {
            const int i = tid + k * NT;
            pm[k] = i < G::NM ? gmask[i] : 0u;
            if (GRAY)
                pe[k] = i < G::NM ? gmask[G::NM + i] : 0u;
        }
        const uint32_t *grt2 = reinterpret_cast<const uint32_t *>(im.rt + (int64_t)ti * G::RCAP);
        const int32_t *gcf = im.cf + (int64_t)ti * G::RCAP;
#pragma unroll
        for (int j = 0; j < PJ; j++) {
            const int q = tid + j * NT;
            prt[j] = 2 * q < pn_runs ? grt2[q] : 0u;
        }
#pragma unroll
        for (int j = 0; j < CJ; j++) {
            const int c = tid + j * NT;
            pcf[j] = c < pn_comp ? gcf[c] : 0;
        }
    };
    // mask and component labels of `tile` from registers into LDS
    auto stage = [&](int slot) {
#pragma unroll
        for (int k = 0; k < MPT; k++) {
            const int i = tid + k * NT;
            if (i < G::NM) {
                t.M[i] = pm[k];
                if (GRAY)
                    t.E[i] = pe[k];
            }
        }
        // unconditional (entries past the tile's components are unused), so
        // that the wait for these loads, the youngest of the prefetch, is
        // on every path and no later use of the prefetch waits again
#pragma unroll
        for (int j = 0; j < CJ; j++)
            t.CF[tid + j * NT] = pcf[j];
        if (pn_comp > CJ * NT) {
            const int tile = tile_of(slot);
            const Img &im = find_img(b, tile, kTile);
            const int32_t *gcf = im.cf + (int64_t)(tile - im.tile0) * G::RCAP;
            for (int c = CJ * NT + tid; c < pn_comp; c += NT)
                t.CF[c] = gcf[c];
        }
    };
    // slots blockIdx.x, + gridDim.x, ...; with the 4-byte store form slot i
    // is tile xcd_tile(i), so that the workgroups of one XCD label
    // neighbouring tiles at the same time (their label rows share cache
    // lines where a row segment is not line aligned); aligned rows keep the
    // plain order (slightly faster there)
    int slot = blockIdx.x;
    if (slot >= ntiles)
        return;
    counts(slot);
    fetch(slot);
    counts(slot + gridDim.x);
    stage(slot);
    __syncthreads();
    for (;;) {
        const int tile = tile_of(slot);
        const Img &im = find_img(b, tile, kTile);
        const int ti = tile - im.tile0;
        const int ty = ti / im.NTX, tx = ti % im.NTX;
        const int y0 = ty * TH, x0 = tx * TW;
        number_runs<NSR, TW, BH, NT>(t, t.E);
#pragma unroll
        for (int j = 0; j < PJ; j++) {
            const int q = tid + j * NT;
            if (2 * q < pn_runs)
                t.RF[2 * q] = t.CF[prt[j] & 0xFFFFu];
            if (2 * q + 1 < pn_runs)
                t.RF[2 * q + 1] = t.CF[prt[j] >> 16];
        }
        if (pn_runs > 2 * PJ * NT) {
            const uint16_t *grt = im.rt + (int64_t)ti * G::RCAP;
            for (int k = 2 * PJ * NT + tid; k < pn_runs; k += NT)
                t.RF[k] = t.CF[grt[k]];
        }
        __syncthreads();
        const int next = slot + (int)gridDim.x;
        if (next < ntiles) {
            fetch(next);
            counts(next + (int)gridDim.x);
        }

        // write: one tile row segment of 256 pixels per wave instruction
        // buffer size: the bytes from the tile's first row to the end of
        // the image (rows below the image fall past it), at most kDropped
        const int64_t left = (int64_t)(im.H - y0) * im.W * 4;
        const uint32_t nrec = left < (int64_t)kDropped ? (uint32_t)left : kDropped;
        const __amdgpu_buffer_rsrc_t rsrc =
            __builtin_amdgcn_make_buffer_rsrc(im.labels + (int64_t)y0 * im.W, 0, (int)nrec, kBufferWord3);
        // (loops with compile-time trip counts: rows wave, wave + 8, ...;
        // fully unrolled, so each wave issues its stores back to back)
        constexpr int NWV = NT / 64;
        constexpr int RPW = (TH + NWV - 1) / NWV;
        if (STORE == kStore16) {
            constexpr int QPL = (TW / 4 + 63) / 64;
#pragma unroll
            for (int i = 0; i < RPW; i++) {
                const int r = wave + i * NWV;
                if (TH % NWV != 0 && r >= TH)
                    break;
                const int R = r / G::RB;
#pragma unroll
                for (int j = 0; j < QPL; j++) {
                    const int q = lane + 64 * j;
                    if ((TW / 4) % 64 != 0 && q >= TW / 4)
                        break;
                    const int c0 = q * 4;
                    const int w = c0 >> 5, b0 = c0 & 31;
                    const uint32_t m = t.M[r * NW + w] >> b0;
                    const uint32_t s = t.S[R * NW + w];
                    const int32_t bs = t.base[R * NW + w] - 1;
                    i32x4 o;
                    o.x = (m & 1u) ? t.RF[bs + __popc(s & mask_le(b0))] : 0;
                    o.y = (m & 2u) ? t.RF[bs + __popc(s & mask_le(b0 + 1))] : 0;
                    o.z = (m & 4u) ? t.RF[bs + __popc(s & mask_le(b0 + 2))] : 0;
                    o.w = (m & 8u) ? t.RF[bs + __popc(s & mask_le(b0 + 3))] : 0;
                    const uint32_t off = x0 + c0 < im.W ? (uint32_t)((r * im.W + x0 + c0) * 4) : kDropped;
                    __builtin_amdgcn_raw_buffer_store_b128(o, rsrc, (int)off, 0, kStoreNtSc1);
                }
            }
        } else if (STORE == kStore4) {
#pragma unroll
            for (int i = 0; i < RPW; i++) {
                const int r = wave + i * NWV;
                if (TH % NWV != 0 && r >= TH)
                    break;
                const int R = r / G::RB;
#pragma unroll
                for (int e = 0; e < TW / 64; e++) {
                    const int c = e * 64 + lane;
                    const int w = c >> 5, b0 = c & 31;
                    const bool fg = (t.M[r * NW + w] >> b0) & 1u;
                    const int32_t v =
                        fg ? t.RF[t.base[R * NW + w] - 1 + __popc(t.S[R * NW + w] & mask_le(b0))] : 0;
                    const uint32_t off = x0 + c < im.W ? (uint32_t)((r * im.W + x0 + c) * 4) : kDropped;
                    __builtin_amdgcn_raw_buffer_store_b32(v, rsrc, (int)off, 0, 0 /* cached */);
                }
            }
        } else {
            for (int r = wave; r < TH; r += NT / 64) {
                const int y = y0 + r;
                if (y >= im.H)
                    break;
                const int R = r / G::RB;
                for (int q = lane; q < TW / 4; q += 64) {
                    const int c0 = q * 4, x = x0 + c0;
                    if (x >= im.W)
                        continue;
                    const int w = c0 >> 5, b0 = c0 & 31;
                    const uint32_t m = t.M[r * NW + w] >> b0;
                    const uint32_t s = t.S[R * NW + w];
                    const int32_t bs = t.base[R * NW + w] - 1;
                    int32_t o[4];
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        o[e] = ((m >> e) & 1u) ? t.RF[bs + __popc(s & mask_le(b0 + e))] : 0;
                    int32_t *dst = im.labels + (int64_t)y * im.W + x;
                    const int nn = im.W - x < 4 ? im.W - x : 4;
                    for (int e = 0; e < nn; e++)
                        dst[e] = o[e];
                }
            }
        }
        if (next >= ntiles)
            break;
        __syncthreads();
        stage(next);
        __syncthreads();
        slot = next;
    }
}

}  // namespace ccl
