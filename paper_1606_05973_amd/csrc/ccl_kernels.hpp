// Device side of the gfx950 two-pass connected component labeling library.
//
// Method (Gupta et al., arXiv 1606.05973, Sections III-IV), re-designed for
// one MI355X:
//   * the image is cut into TH x TW tiles; one workgroup labels one tile in
//     LDS (the "local" phase of PARemSP, Algorithm 7, with 2-D tiles instead
//     of row chunks);
//   * inside a tile the scan works on horizontal runs held as 32-bit
//     foreground masks (one mask word per lane); every pair of runs in
//     consecutive rows that touch is united once with Rem's union with
//     splicing (Algorithm 2) on an LDS parent array, concurrently, with the
//     root link done by compare-and-swap as in the concurrent merger
//     (Algorithm 8, locks replaced by CAS);
//   * the union-find keys are local pixel indices of run starts; since every
//     link points to a smaller index, every set's root is the set's first
//     pixel in raster order;
//   * across tiles, components meet at tile edges; the edge pixels' local
//     roots are stored, and a second kernel unites them across every tile
//     edge with the same CAS-based RemSP, on a parent array keyed by global
//     raster index (the labels buffer itself, used sparsely);
//   * flatten resolves every boundary root; components are ranked by their
//     smallest raster index through counts per (image row, tile column)
//     segment and a device exclusive scan;
//   * the labeling pass (second pass) re-reads the image, rebuilds the tile
//     labeling in LDS (deterministic: the local partition and its minima do
//     not depend on scheduling) and writes every label once.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccl {

constexpr int kThreads = 256;          // threads per workgroup (4 wave64)
constexpr uint16_t kNone = 0xFFFFu;     // background in the edge buffers
constexpr int kScanChunk = 4096;        // segment counts per scan block (256 x 16)
constexpr int32_t kRootFlag = 1 << 30;  // boundary-list entry is a global root
constexpr int32_t kLocalMask = 0xFFFF;  // boundary-list entry: local pixel index

// Per-image description used by every kernel.  Arrays live in the library
// workspace except img / labels / ncomp, which belong to the caller.
struct Img {
    const uint8_t *img;   // H rows, pitch `stride` bytes
    int32_t *labels;      // H x W, pitch W; also the global parent array
    int32_t *ncomp;       // optional K output
    uint16_t *he;         // [NTY][2][W]: local root of each pixel on the top(0)/bottom(1) tile rows
    uint16_t *ve;         // [NTX][2][H]: same for the left(0)/right(1) tile columns
    int32_t *bl_idx;      // [NT][CAP]: boundary local roots (local index | kRootFlag)
    int32_t *bl_val;      // [NT][CAP]: interior roots before it in its row, then offset, then final label
    int32_t *bl_cnt;      // [NT]
    int32_t *seg;         // [H][NTX]: roots per (row, tile column) segment -> exclusive scan
    int32_t *blk;         // [nblk]: scan block totals -> exclusive scan
    int64_t stride;
    int32_t H, W, NTY, NTX, conn;
    int32_t tile0;        // first tile of this image in a batch-wide tile numbering
    int32_t edge0;        // first edge item (boundary merge kernel)
    int32_t scan0;        // first scan block
    int32_t nblk;
};

struct Batch {
    const Img *tab;  // device table of n images (n > 1)
    Img one;         // the image when n == 1
    int32_t n;
};

enum Key { kTile = 0, kEdge = 1, kScan = 2 };

__device__ __forceinline__ int32_t key_of(const Img &im, int which) {
    return which == kTile ? im.tile0 : (which == kEdge ? im.edge0 : im.scan0);
}

// Image owning global work item `item` (binary search over the start keys).
__device__ __forceinline__ const Img &find_img(const Batch &b, int32_t item, int which) {
    if (b.n == 1)
        return b.one;
    int lo = 0, hi = b.n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (key_of(b.tab[mid], which) <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return b.tab[lo];
}

// ------------------------------------------------------------------------
// Relaxed atomics at a chosen scope (workgroup for LDS, agent for the
// global parent array: the L2 caches of the eight XCDs are not coherent with
// each other, so every access to a shared parent entry is an agent-scope
// atomic).
// ------------------------------------------------------------------------
template <int S>
__device__ __forceinline__ int32_t aload(int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, S);
}
template <int S>
__device__ __forceinline__ void astore(int32_t *p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, S);
}
// Compare-and-swap; returns the value found at *p (== expect on success).
template <int S>
__device__ __forceinline__ int32_t acas(int32_t *p, int32_t expect, int32_t v) {
    __hip_atomic_compare_exchange_strong(p, &expect, v, __ATOMIC_RELAXED, __ATOMIC_RELAXED, S);
    return expect;
}

// Rem's union with splicing (Algorithm 2), made safe for concurrent callers
// as in Algorithm 8: the link of a root is a CAS that succeeds only if it is
// still a root; splices are plain atomic stores.  Every store writes a value
// smaller than the node's own index, so the forest stays acyclic and every
// root is the smallest element of its set.  Each iteration either returns,
// moves rx or ry to a strictly smaller index, or retries a link that another
// caller's successful link made fail (with the value that CAS observed), so
// the loop ends even if a plain load returned an older parent.
template <int S>
__device__ void rem_union(int32_t *P, int32_t x, int32_t y) {
    int32_t rx = x, ry = y;
    int32_t px = aload<S>(P + rx);
    int32_t py = aload<S>(P + ry);
    while (px != py) {
        if (px > py) {
            if (px == rx) {
                int32_t seen = acas<S>(P + rx, rx, py);
                if (seen == rx)
                    return;
                px = seen;
                continue;
            }
            astore<S>(P + rx, py);
            rx = px;
            px = aload<S>(P + rx);
        } else {
            if (py == ry) {
                int32_t seen = acas<S>(P + ry, ry, px);
                if (seen == ry)
                    return;
                py = seen;
                continue;
            }
            astore<S>(P + ry, px);
            ry = py;
            py = aload<S>(P + ry);
        }
    }
}

// Find with full path compression.  Only used after all unions are done,
// so the root is fixed and the only value ever stored is that root.
template <int S>
__device__ int32_t find_compress(int32_t *P, int32_t x) {
    int32_t r = x, p;
    while ((p = aload<S>(P + r)) != r)
        r = p;
    int32_t y = x;
    while (y != r) {
        int32_t nx = aload<S>(P + y);
        astore<S>(P + y, r);
        y = nx;
    }
    return r;
}

// ------------------------------------------------------------------------
// Foreground masks.  Bit j of a word is pixel x0 + j (nonzero byte).
// ------------------------------------------------------------------------
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

// 4 bytes -> 4 bits (byte != 0).  The add sets bit 7 of every byte whose
// low 7 bits are nonzero (no carry crosses a byte); OR-ing the byte covers
// bit 7 itself.  The multiply gathers bits 7, 15, 23, 31 into bits 28..31.
__device__ __forceinline__ uint32_t nz4(uint32_t x) {
    uint32_t t = (((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x) & 0x80808080u;
    return (t * 0x00204081u) >> 28;
}

__device__ __forceinline__ uint32_t nz16(u32x4 v) {
    return nz4(v.x) | (nz4(v.y) << 4) | (nz4(v.z) << 8) | (nz4(v.w) << 12);
}

// 32 pixels of row y starting at column x (x % 32 == 0); outside = 0.
__device__ __forceinline__ uint32_t load_word(const Img &im, int y, int x) {
    if (y >= im.H || x >= im.W)
        return 0u;
    const uint8_t *p = im.img + (int64_t)y * im.stride + x;
    if (x + 32 <= im.W && ((reinterpret_cast<uintptr_t>(p) & 15u) == 0)) {
        u32x4 a = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
        u32x4 b = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p + 16));
        return nz16(a) | (nz16(b) << 16);
    }
    uint32_t m = 0;
    int n = im.W - x < 32 ? im.W - x : 32;
    for (int i = 0; i < n; i++)
        m |= (uint32_t)(p[i] != 0) << i;
    return m;
}

// ------------------------------------------------------------------------
// Tile geometry and the LDS state of one tile.
// ------------------------------------------------------------------------
template <int TH, int TW>
struct Geo {
    static constexpr int NW = TW / 32;            // mask words per tile row
    static constexpr int NU = TH * NW;            // (row, word) units
    static constexpr int UPT = (NU + kThreads - 1) / kThreads;
    static constexpr int NPX = TH * TW;
    static constexpr int CAP = 2 * (TH + TW);     // > pixels on the tile perimeter
    static_assert(TW % 32 == 0, "tile width must be a multiple of 32");
    static_assert(NPX <= 65536, "local pixel indices must fit 16 bits");
};

template <int TH, int TW>
struct TileLds {
    using G = Geo<TH, TW>;
    uint32_t M[G::NU];    // foreground masks
    uint32_t S[G::NU];    // run-start masks
    int32_t IN[G::NU];    // start of the run covering bit 0 when it continues from the left
    uint32_t A[G::NU];    // flag bitmask (boundary roots in the scan; all roots in the relabel)
    uint32_t B[G::NU];    // flag bitmask (interior roots)
    int32_t P[G::NPX];    // parent array over local pixel indices (used at run starts)
    int32_t rowv[TH];
    int32_t list[G::CAP];
    int32_t nlist;
};

// Start (local pixel index) of the run containing foreground pixel (r, c).
template <int TH, int TW>
__device__ __forceinline__ int32_t run_start(const TileLds<TH, TW> &t, int r, int c) {
    constexpr int NW = Geo<TH, TW>::NW;
    int w = c >> 5, b = c & 31;
    uint32_t s = t.S[r * NW + w] & (0xFFFFFFFFu >> (31 - b));
    return s ? (r * TW + (w << 5) + 31 - __clz(s)) : t.IN[r * NW + w];
}

// Tile-local labeling: after it returns (behind a barrier) P[s] is the local
// root of run start s, and the local root is the component's first pixel in
// raster order inside the tile.
template <int TH, int TW>
__device__ void tile_label(TileLds<TH, TW> &t, const Img &im, int y0, int x0) {
    using G = Geo<TH, TW>;
    constexpr int NW = G::NW;
    const int tid = threadIdx.x;
    const bool conn8 = im.conn == 8;

    // load the tile as 32-bit foreground masks, clear the flag masks
#pragma unroll
    for (int k = 0; k < G::UPT; k++) {
        int u = tid + k * kThreads;
        if (u < G::NU) {
            int r = u / NW, w = u % NW;
            t.M[u] = load_word(im, y0 + r, x0 + (w << 5));
            t.A[u] = 0u;
            t.B[u] = 0u;
        }
    }
    if (tid == 0)
        t.nlist = 0;
    for (int r = tid; r < TH; r += kThreads)
        t.rowv[r] = 0;
    __syncthreads();

    // run starts: foreground with background (or the tile edge) on the left
#pragma unroll
    for (int k = 0; k < G::UPT; k++) {
        int u = tid + k * kThreads;
        if (u < G::NU) {
            int w = u % NW;
            uint32_t m = t.M[u];
            uint32_t mL = w ? t.M[u - 1] : 0u;
            t.S[u] = m & ~((m << 1) | (mL >> 31));
        }
    }
    __syncthreads();

    // run continuing into the word, and one parent entry per run start
#pragma unroll
    for (int k = 0; k < G::UPT; k++) {
        int u = tid + k * kThreads;
        if (u < G::NU) {
            int r = u / NW, w = u % NW;
            uint32_t m = t.M[u], st = t.S[u];
            int32_t in = -1;
            if ((m & 1u) && !(st & 1u)) {
                // every word between the run start and this one is all ones
                int kk = w - 1;
                while (kk > 0 && t.S[r * NW + kk] == 0u)
                    kk--;
                in = r * TW + (kk << 5) + 31 - __clz(t.S[r * NW + kk]);
            }
            t.IN[u] = in;
            uint32_t bits = st;
            while (bits) {
                int b = __ffs(bits) - 1;
                bits &= bits - 1u;
                int32_t s = r * TW + (w << 5) + b;
                t.P[s] = s;
            }
        }
    }
    __syncthreads();

    // unions between runs of row r and row r-1 that touch; each touching pair
    // is united exactly once:
    //   U1: first column of the overlap of the two runs,
    //   U2: (8-conn) the upper run starts right after the lower run ends,
    //   U3: (8-conn) the lower run starts right after the upper run ends.
#pragma unroll
    for (int k = 0; k < G::UPT; k++) {
        int u = tid + k * kThreads;
        if (u < G::NU) {
            int r = u / NW, w = u % NW;
            if (r == 0)
                continue;
            const int base = w << 5;
            uint32_t m = t.M[u];
            uint32_t mL = w ? t.M[u - 1] : 0u;
            uint32_t up = t.M[u - NW];
            uint32_t uL = w ? t.M[u - NW - 1] : 0u;
            uint32_t o = m & up;
            uint32_t u1 = o & ~((o << 1) | ((mL & uL) >> 31));
            while (u1) {
                int b = __ffs(u1) - 1;
                u1 &= u1 - 1u;
                rem_union<__HIP_MEMORY_SCOPE_WORKGROUP>(t.P, run_start(t, r, base + b),
                                                        run_start(t, r - 1, base + b));
            }
            if (conn8) {
                uint32_t mR = (w < NW - 1) ? t.M[u + 1] : 0u;
                uint32_t uR = (w < NW - 1) ? t.M[u - NW + 1] : 0u;
                uint32_t mn = (m >> 1) | (mR << 31);   // pixel c+1, same row
                uint32_t un = (up >> 1) | (uR << 31);  // pixel c+1, row above
                uint32_t mp = (m << 1) | (mL >> 31);   // pixel c-1, same row
                uint32_t upp = (up << 1) | (uL >> 31); // pixel c-1, row above
                uint32_t u2 = m & ~mn & ~up & un;
                uint32_t u3 = m & ~mp & ~up & upp;
                while (u2) {
                    int b = __ffs(u2) - 1;
                    u2 &= u2 - 1u;
                    rem_union<__HIP_MEMORY_SCOPE_WORKGROUP>(t.P, run_start(t, r, base + b),
                                                            (r - 1) * TW + base + b + 1);
                }
                while (u3) {
                    int b = __ffs(u3) - 1;
                    u3 &= u3 - 1u;
                    rem_union<__HIP_MEMORY_SCOPE_WORKGROUP>(t.P, r * TW + base + b,
                                                            run_start(t, r - 1, base + b - 1));
                }
            }
        }
    }
    __syncthreads();

    // flatten: every run start points straight at its root
#pragma unroll
    for (int k = 0; k < G::UPT; k++) {
        int u = tid + k * kThreads;
        if (u < G::NU) {
            int r = u / NW, w = u % NW;
            uint32_t bits = t.S[u];
            while (bits) {
                int b = __ffs(bits) - 1;
                bits &= bits - 1u;
                find_compress<__HIP_MEMORY_SCOPE_WORKGROUP>(t.P, r * TW + (w << 5) + b);
            }
        }
    }
    __syncthreads();
}

template <int TH, int TW>
__device__ __forceinline__ int32_t gidx(const Img &im, int ty, int tx, int32_t li) {
    return (ty * TH + li / TW) * im.W + tx * TW + li % TW;
}

__device__ __forceinline__ int popc_before(const uint32_t *row, int c) {
    int w = c >> 5, b = c & 31, n = 0;
    for (int k = 0; k < w; k++)
        n += __popc(row[k]);
    return n + __popc(row[w] & ((1u << b) - 1u));
}

// ------------------------------------------------------------------------
// K1: tile scan.  Local labeling, then the tile's exports:
//   edge buffers (local root per edge pixel, for the boundary merge),
//   boundary roots (components touching an edge that has a neighbour tile)
//     with the count of interior roots before them in their row,
//   interior root counts per row segment,
//   labels[g] = g for every boundary root g (global parent array).
// ------------------------------------------------------------------------
template <int TH, int TW>
__global__ __launch_bounds__(kThreads) void k_tile_scan(Batch b) {
    using G = Geo<TH, TW>;
    constexpr int NW = G::NW;
    __shared__ TileLds<TH, TW> t;
    const Img &im = find_img(b, blockIdx.x, kTile);
    const int ti = blockIdx.x - im.tile0;
    const int ty = ti / im.NTX, tx = ti % im.NTX;
    const int y0 = ty * TH, x0 = tx * TW;
    const int tid = threadIdx.x;
    tile_label<TH, TW>(t, im, y0, x0);

    const bool top = ty > 0, bot = ty < im.NTY - 1, left = tx > 0, right = tx < im.NTX - 1;
    // mark components that touch an edge shared with another tile
#pragma unroll
    for (int k = 0; k < G::UPT; k++) {
        int u = tid + k * kThreads;
        if (u < G::NU) {
            int r = u / NW, w = u % NW;
            uint32_t m = t.M[u];
            if ((r == 0 && top) || (r == TH - 1 && bot)) {
                uint32_t bits = t.S[u];
                while (bits) {
                    int bb = __ffs(bits) - 1;
                    bits &= bits - 1u;
                    int32_t root = t.P[r * TW + (w << 5) + bb];
                    atomicOr(&t.A[root >> 5], 1u << (root & 31));
                }
            }
            if (w == 0 && left && (m & 1u)) {
                int32_t root = t.P[r * TW];
                atomicOr(&t.A[root >> 5], 1u << (root & 31));
            }
            if (w == NW - 1 && right && (m >> 31)) {
                int32_t root = t.P[run_start(t, r, TW - 1)];
                atomicOr(&t.A[root >> 5], 1u << (root & 31));
            }
        }
    }
    // edge buffers
    if (top || bot) {
        for (int c = tid; c < 2 * TW; c += kThreads) {
            int side = c / TW, cc = c % TW;
            if ((side == 0 && !top) || (side == 1 && !bot))
                continue;
            int x = x0 + cc;
            if (x >= im.W)
                continue;
            int r = side ? TH - 1 : 0;
            uint16_t v = kNone;
            if ((t.M[r * NW + (cc >> 5)] >> (cc & 31)) & 1u)
                v = (uint16_t)t.P[run_start(t, r, cc)];
            im.he[((int64_t)ty * 2 + side) * im.W + x] = v;
        }
    }
    if (left || right) {
        for (int q = tid; q < 2 * TH; q += kThreads) {
            int side = q / TH, r = q % TH;
            if ((side == 0 && !left) || (side == 1 && !right))
                continue;
            int y = y0 + r;
            if (y >= im.H)
                continue;
            uint16_t v = kNone;
            if (side == 0) {
                if (t.M[r * NW] & 1u)
                    v = (uint16_t)t.P[r * TW];
            } else {
                if (t.M[r * NW + NW - 1] >> 31)
                    v = (uint16_t)t.P[run_start(t, r, TW - 1)];
            }
            im.ve[((int64_t)tx * 2 + side) * im.H + y] = v;
        }
    }
    __syncthreads();

    // classify the tile's components (one per local root)
#pragma unroll
    for (int k = 0; k < G::UPT; k++) {
        int u = tid + k * kThreads;
        if (u < G::NU) {
            int r = u / NW, w = u % NW;
            uint32_t bits = t.S[u];
            while (bits) {
                int bb = __ffs(bits) - 1;
                bits &= bits - 1u;
                int32_t s = r * TW + (w << 5) + bb;
                if (t.P[s] != s)
                    continue;
                if ((t.A[u] >> bb) & 1u) {
                    int j = atomicAdd(&t.nlist, 1);
                    t.list[j] = s;
                    int32_t g = gidx<TH, TW>(im, ty, tx, s);
                    im.labels[g] = g;
                } else {
                    atomicOr(&t.B[u], 1u << bb);
                    atomicAdd(&t.rowv[r], 1);
                }
            }
        }
    }
    __syncthreads();

    const int n = t.nlist;
    int32_t *bidx = im.bl_idx + (int64_t)ti * G::CAP;
    int32_t *bval = im.bl_val + (int64_t)ti * G::CAP;
    for (int j = tid; j < n; j += kThreads) {
        int32_t s = t.list[j];
        int r = s / TW, c = s % TW;
        bidx[j] = s;
        bval[j] = popc_before(&t.B[r * NW], c);
    }
    for (int r = tid; r < TH; r += kThreads)
        if (y0 + r < im.H)
            im.seg[(int64_t)(y0 + r) * im.NTX + tx] = t.rowv[r];
    if (tid == 0)
        im.bl_cnt[ti] = n;
}

// ------------------------------------------------------------------------
// K2: boundary merge (Algorithm 7's boundary loop, Algorithm 8's merger).
// One item per pixel of every interior tile edge.  8-connectivity: unite
// with the pixel straight across if it is foreground, else with the two
// diagonal ones (a foreground pixel straight across already joins its
// diagonal neighbours, through its own tile or the perpendicular edge).
// ------------------------------------------------------------------------
template <int TH, int TW>
__global__ __launch_bounds__(kThreads) void k_merge(Batch b) {
    const int32_t item = blockIdx.x * kThreads + threadIdx.x;
    const Img &im = find_img(b, item, kEdge);
    int32_t e = item - im.edge0;
    const int32_t nH = (im.NTY - 1) * im.W;
    const int32_t nV = (im.NTX - 1) * im.H;
    if (e < 0 || e >= nH + nV)
        return;
    int32_t *P = im.labels;
    if (e < nH) {
        const int ty = 1 + e / im.W, x = e % im.W;
        const uint16_t *lo = im.he + ((int64_t)ty * 2 + 0) * im.W;       // first row of tile row ty
        const uint16_t *hi = im.he + ((int64_t)(ty - 1) * 2 + 1) * im.W; // last row of tile row ty-1
        uint16_t l = lo[x];
        if (l == kNone)
            return;
        const int32_t ge = gidx<TH, TW>(im, ty, x / TW, l);
        uint16_t h = hi[x];
        if (h != kNone) {
            if ((x % TW) != 0 && lo[x - 1] == l && hi[x - 1] == h)
                return;  // same pair as the previous column
            rem_union<__HIP_MEMORY_SCOPE_AGENT>(P, ge, gidx<TH, TW>(im, ty - 1, x / TW, h));
        } else if (im.conn == 8) {
            if (x > 0 && hi[x - 1] != kNone)
                rem_union<__HIP_MEMORY_SCOPE_AGENT>(P, ge, gidx<TH, TW>(im, ty - 1, (x - 1) / TW, hi[x - 1]));
            if (x + 1 < im.W && hi[x + 1] != kNone)
                rem_union<__HIP_MEMORY_SCOPE_AGENT>(P, ge, gidx<TH, TW>(im, ty - 1, (x + 1) / TW, hi[x + 1]));
        }
    } else {
        e -= nH;
        const int tx = 1 + e / im.H, y = e % im.H;
        const uint16_t *rc = im.ve + ((int64_t)tx * 2 + 0) * im.H;       // first column of tile column tx
        const uint16_t *lc = im.ve + ((int64_t)(tx - 1) * 2 + 1) * im.H; // last column of tile column tx-1
        uint16_t rv = rc[y];
        if (rv == kNone)
            return;
        const int32_t ge = gidx<TH, TW>(im, y / TH, tx, rv);
        uint16_t lv = lc[y];
        if (lv != kNone) {
            if ((y % TH) != 0 && rc[y - 1] == rv && lc[y - 1] == lv)
                return;
            rem_union<__HIP_MEMORY_SCOPE_AGENT>(P, ge, gidx<TH, TW>(im, y / TH, tx - 1, lv));
        } else if (im.conn == 8) {
            if (y > 0 && lc[y - 1] != kNone)
                rem_union<__HIP_MEMORY_SCOPE_AGENT>(P, ge, gidx<TH, TW>(im, (y - 1) / TH, tx - 1, lc[y - 1]));
            if (y + 1 < im.H && lc[y + 1] != kNone)
                rem_union<__HIP_MEMORY_SCOPE_AGENT>(P, ge, gidx<TH, TW>(im, (y + 1) / TH, tx - 1, lc[y + 1]));
        }
    }
}

// ------------------------------------------------------------------------
// K3a: flatten the boundary roots of one tile; a boundary root that is its
// own global root is the first pixel of its component.  Adds those roots to
// the segment counts and stores their offset inside their row segment.
// ------------------------------------------------------------------------
template <int TH, int TW>
__global__ __launch_bounds__(kThreads) void k_flatten(Batch b) {
    using G = Geo<TH, TW>;
    constexpr int NW = G::NW;
    __shared__ uint32_t R[G::NU];
    __shared__ int32_t rowv[TH];
    __shared__ uint8_t isr[G::CAP];
    const Img &im = find_img(b, blockIdx.x, kTile);
    const int ti = blockIdx.x - im.tile0;
    const int n = im.bl_cnt[ti];
    if (n == 0)
        return;
    const int ty = ti / im.NTX, tx = ti % im.NTX;
    const int y0 = ty * TH;
    const int tid = threadIdx.x;
    for (int u = tid; u < G::NU; u += kThreads)
        R[u] = 0u;
    for (int r = tid; r < TH; r += kThreads)
        rowv[r] = 0;
    __syncthreads();
    int32_t *bidx = im.bl_idx + (int64_t)ti * G::CAP;
    int32_t *bval = im.bl_val + (int64_t)ti * G::CAP;
    for (int j = tid; j < n; j += kThreads) {
        int32_t s = bidx[j] & kLocalMask;
        int32_t g = gidx<TH, TW>(im, ty, tx, s);
        int32_t root = find_compress<__HIP_MEMORY_SCOPE_AGENT>(im.labels, g);
        bool is = root == g;
        isr[j] = is;
        if (is) {
            atomicOr(&R[s >> 5], 1u << (s & 31));
            atomicAdd(&rowv[s / TW], 1);
        }
    }
    __syncthreads();
    for (int j = tid; j < n; j += kThreads) {
        if (isr[j]) {
            int32_t s = bidx[j] & kLocalMask;
            int r = s / TW, c = s % TW;
            bval[j] += popc_before(&R[r * NW], c);
            bidx[j] = s | kRootFlag;
        }
    }
    for (int r = tid; r < TH; r += kThreads)
        if (rowv[r] && y0 + r < im.H)
            im.seg[(int64_t)(y0 + r) * im.NTX + tx] += rowv[r];
}

// ------------------------------------------------------------------------
// K4a / K4b: exclusive scan of the segment counts in raster order.
// K4a scans blocks of kScanChunk entries in place and stores block totals;
// K4b (one workgroup per image) scans the block totals and stores K.
// ------------------------------------------------------------------------
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t *total) {
    __shared__ int32_t wsum[kThreads / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int32_t o = __shfl_up(incl, d, 64);
        if (lane >= d)
            incl += o;
    }
    if (lane == 63)
        wsum[wv] = incl;
    __syncthreads();
    int32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kThreads / 64; k++) {
        int32_t s = wsum[k];
        before += (k < wv) ? s : 0;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + incl - v;
}

__global__ __launch_bounds__(kThreads) void k_scan_blocks(Batch b) {
    const Img &im = find_img(b, blockIdx.x, kScan);
    const int c = blockIdx.x - im.scan0;
    const int64_t L = (int64_t)im.H * im.NTX;
    const int64_t base = (int64_t)c * kScanChunk + threadIdx.x * 16;
    int32_t v[16];
    int32_t sum = 0;
#pragma unroll
    for (int i = 0; i < 16; i++) {
        v[i] = (base + i < L) ? im.seg[base + i] : 0;
        sum += v[i];
    }
    int32_t total;
    int32_t run = block_exclusive_scan(sum, &total);
#pragma unroll
    for (int i = 0; i < 16; i++) {
        if (base + i < L)
            im.seg[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0)
        im.blk[c] = total;
}

__global__ __launch_bounds__(kThreads) void k_scan_top(Batch b) {
    const Img &im = (b.n == 1) ? b.one : b.tab[blockIdx.x];
    int32_t carry = 0;
    for (int base = 0; base < im.nblk; base += kThreads) {
        int i = base + threadIdx.x;
        int32_t v = i < im.nblk ? im.blk[i] : 0;
        int32_t total;
        int32_t ex = block_exclusive_scan(v, &total);
        if (i < im.nblk)
            im.blk[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0 && im.ncomp)
        *im.ncomp = carry;
}

// ------------------------------------------------------------------------
// K3b: final label of every boundary root: 1 + roots before its segment +
// roots before it inside the segment.  Written to the boundary list and to
// labels[g] (read by other tiles' non-root boundary components in K5).
// ------------------------------------------------------------------------
template <int TH, int TW>
__global__ __launch_bounds__(kThreads) void k_publish(Batch b) {
    using G = Geo<TH, TW>;
    const Img &im = find_img(b, blockIdx.x, kTile);
    const int ti = blockIdx.x - im.tile0;
    const int n = im.bl_cnt[ti];
    const int ty = ti / im.NTX, tx = ti % im.NTX;
    int32_t *bidx = im.bl_idx + (int64_t)ti * G::CAP;
    int32_t *bval = im.bl_val + (int64_t)ti * G::CAP;
    for (int j = threadIdx.x; j < n; j += kThreads) {
        int32_t v = bidx[j];
        if (!(v & kRootFlag))
            continue;
        int32_t s = v & kLocalMask;
        int64_t sg = (int64_t)(ty * TH + s / TW) * im.NTX + tx;
        int32_t F = 1 + im.seg[sg] + im.blk[sg / kScanChunk] + bval[j];
        bval[j] = F;
        im.labels[gidx<TH, TW>(im, ty, tx, s)] = F;
    }
}

// ------------------------------------------------------------------------
// K5: labeling pass.  Rebuild the tile labeling, give every local component
// its final label, write all pixels with 16-byte stores.
// ------------------------------------------------------------------------
template <int TH, int TW>
__global__ __launch_bounds__(kThreads) void k_relabel(Batch b) {
    using G = Geo<TH, TW>;
    constexpr int NW = G::NW;
    __shared__ TileLds<TH, TW> t;
    __shared__ int32_t rowbase[TH];
    const Img &im = find_img(b, blockIdx.x, kTile);
    const int ti = blockIdx.x - im.tile0;
    const int ty = ti / im.NTX, tx = ti % im.NTX;
    const int y0 = ty * TH, x0 = tx * TW;
    const int tid = threadIdx.x;
    for (int r = tid; r < TH; r += kThreads) {
        int32_t v = 0;
        if (y0 + r < im.H) {
            int64_t sg = (int64_t)(y0 + r) * im.NTX + tx;
            v = im.seg[sg] + im.blk[sg / kScanChunk];
        }
        rowbase[r] = v;
    }
    tile_label<TH, TW>(t, im, y0, x0);

    // boundary components: final label from the boundary list (own roots)
    // or from the global root's published label
    const int n = im.bl_cnt[ti];
    const int32_t *bidx = im.bl_idx + (int64_t)ti * G::CAP;
    const int32_t *bval = im.bl_val + (int64_t)ti * G::CAP;
    for (int j = tid; j < n; j += kThreads) {
        int32_t v = bidx[j];
        int32_t s = v & kLocalMask;
        int32_t F;
        if (v & kRootFlag) {
            F = bval[j];
            atomicOr(&t.A[s >> 5], 1u << (s & 31));
        } else {
            int32_t root = im.labels[gidx<TH, TW>(im, ty, tx, s)];
            F = im.labels[root];
        }
        t.P[s] = -F - 1;
    }
    __syncthreads();
    // interior roots join the root mask
#pragma unroll
    for (int k = 0; k < G::UPT; k++) {
        int u = tid + k * kThreads;
        if (u < G::NU) {
            int r = u / NW, w = u % NW;
            uint32_t bits = t.S[u];
            while (bits) {
                int bb = __ffs(bits) - 1;
                bits &= bits - 1u;
                int32_t s = r * TW + (w << 5) + bb;
                if (t.P[s] == s)
                    atomicOr(&t.A[u], 1u << bb);
            }
        }
    }
    __syncthreads();
    // interior roots: rank inside their row segment
#pragma unroll
    for (int k = 0; k < G::UPT; k++) {
        int u = tid + k * kThreads;
        if (u < G::NU) {
            int r = u / NW, w = u % NW;
            uint32_t bits = t.S[u];
            while (bits) {
                int bb = __ffs(bits) - 1;
                bits &= bits - 1u;
                int32_t s = r * TW + (w << 5) + bb;
                if (t.P[s] == s) {
                    int32_t F = 1 + rowbase[r] + popc_before(&t.A[r * NW], (w << 5) + bb);
                    t.P[s] = -F - 1;
                }
            }
        }
    }
    __syncthreads();
    // other run starts take their root's final label
#pragma unroll
    for (int k = 0; k < G::UPT; k++) {
        int u = tid + k * kThreads;
        if (u < G::NU) {
            int r = u / NW, w = u % NW;
            uint32_t bits = t.S[u];
            while (bits) {
                int bb = __ffs(bits) - 1;
                bits &= bits - 1u;
                int32_t s = r * TW + (w << 5) + bb;
                int32_t p = t.P[s];
                if (p >= 0)
                    t.P[s] = t.P[p];
            }
        }
    }
    __syncthreads();

    // write: one tile row per wave instruction, 4 pixels (16 bytes) per lane
    const int wave = tid >> 6, lane = tid & 63;
    const bool vec_ok = ((im.W & 3) == 0) && ((reinterpret_cast<uintptr_t>(im.labels) & 15u) == 0);
    for (int r = wave; r < TH; r += kThreads / 64) {
        const int y = y0 + r;
        if (y >= im.H)
            break;
        for (int q = lane; q < TW / 4; q += 64) {
            const int c0 = q * 4, x = x0 + c0;
            if (x >= im.W)
                continue;
            const int w = c0 >> 5, b0 = c0 & 31;
            uint32_t m = t.M[r * NW + w] >> b0;
            uint32_t st = t.S[r * NW + w] >> b0;
            int32_t cur = 0;
            i32x4 o;
            if (m & 1u)
                cur = -t.P[run_start(t, r, c0)] - 1;
            o.x = (m & 1u) ? cur : 0;
            if (m & 2u) {
                if (st & 2u)
                    cur = -t.P[r * TW + c0 + 1] - 1;
                o.y = cur;
            } else {
                o.y = 0;
            }
            if (m & 4u) {
                if (st & 4u)
                    cur = -t.P[r * TW + c0 + 2] - 1;
                o.z = cur;
            } else {
                o.z = 0;
            }
            if (m & 8u) {
                if (st & 8u)
                    cur = -t.P[r * TW + c0 + 3] - 1;
                o.w = cur;
            } else {
                o.w = 0;
            }
            int32_t *dst = im.labels + (int64_t)y * im.W + x;
            if (vec_ok && x + 4 <= im.W) {
                __builtin_nontemporal_store(o, reinterpret_cast<i32x4 *>(dst));
            } else {
                int nn = im.W - x < 4 ? im.W - x : 4;
                dst[0] = o.x;
                if (nn > 1)
                    dst[1] = o.y;
                if (nn > 2)
                    dst[2] = o.z;
                if (nn > 3)
                    dst[3] = o.w;
            }
        }
    }
}

}  // namespace ccl
