// Fused Sobel + binarize + edge compaction for gfx950.
//
// What is computed (Sec. 2.1 Eq. (1), Sec. 2.2, zero padding Sec. 3.1/4.1):
//   gx = [1 2 1]^T x [-1 0 1] correlation, gy its transpose, pixels outside
//   the frame read as 0; edge = 255 iff |gx| + |gy| > threshold, else 0;
//   mag = min(|gx| + |gy|, 255).
//
// Work decomposition: one wave walks a strip of 32 rows x 1024 columns; each
// lane owns 16 adjacent columns, read with one 128-bit load per row, so a
// wave moves 1 KB per row in a single coalesced instruction.  The 3x3
// stencil is split into a horizontal pass per row ([1 2 1] smooth and
// [-1 0 1] difference, using the two neighbour bytes taken from the adjacent
// lanes) and a vertical pass over three rows held in registers, rotated
// without copies.  No LDS is needed and nothing is re-read except the two
// halo rows of the strip.
//
// Compaction (the vote reads a list of edge coordinates, Sec. 4.3): after
// every 8 rows each lane holds the 64-bit edge masks of its two 8x8 tiles.
// Tile counts are prefix-summed across the wave; then, tile by tile, the
// tile's mask is broadcast to the wave, every lane whose pixel is an edge
// takes its rank among the set bits (mbcnt of the mask) and the wave writes
// the tile's coordinates as one coalesced store.
#include "lane_internal.h"

namespace lane {

enum { kModeSobel = 0, kModeFromEdges = 1 };

// Loads the 16 pixels of one row owned by this lane plus the left and right
// neighbour; pixels outside the frame (or past W) are 0.
template <bool FAST>
__device__ __forceinline__ void load_row(const uint8_t* __restrict__ img, int W, int H, int pitch,
                                         int y, int x0, bool active, int lane, uint32_t (&p)[4],
                                         int& left, int& right) {
    const bool yin = (y >= 0) && (y < H);
    if (FAST) {
        u32x4 v = {0u, 0u, 0u, 0u};
        if (active && yin) v = gld4(img + (size_t)y * pitch + x0);
        p[0] = v.x; p[1] = v.y; p[2] = v.z; p[3] = v.w;
        uint32_t up = __shfl((int)v.w, lane > 0 ? lane - 1 : 0);
        uint32_t dn = __shfl((int)v.x, lane < kWave - 1 ? lane + 1 : kWave - 1);
        left = (int)(up >> 24);
        right = (int)(dn & 0xFFu);
        if (lane == 0) left = (yin && x0 > 0 && x0 - 1 < W) ? gld(img + (size_t)y * pitch + x0 - 1) : 0;
        if (lane == kWave - 1) right = (yin && x0 + 16 < W) ? gld(img + (size_t)y * pitch + x0 + 16) : 0;
    } else {
#pragma unroll
        for (int w = 0; w < 4; ++w) p[w] = 0;
        left = right = 0;
        if (active && yin) {
            const uint8_t* row = img + (size_t)y * pitch;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                int x = x0 + i;
                uint32_t b = (x < W) ? row[x] : 0u;
                p[i >> 2] |= b << ((i & 3) * 8);
            }
            left = (x0 > 0) ? row[x0 - 1] : 0;
            right = (x0 + 16 < W) ? row[x0 + 16] : 0;
        }
    }
}

// Horizontal pass of one row: hs = [1 2 1] smooth, hd = [-1 0 1] difference.
template <bool FAST>
__device__ __forceinline__ void row_filter(const SobelDesc& d, int y, int x0, bool active,
                                           int lane, int (&hs)[16], int (&hd)[16]) {
    uint32_t p[4];
    int left, right;
    load_row<FAST>(d.img, d.W, d.H, d.pitch, y, x0, active, lane, p, left, right);
    int a[18];
    a[0] = left;
    a[17] = right;
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i + 1] = (int)((p[i >> 2] >> ((i & 3) * 8)) & 0xFFu);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        hs[i] = a[i] + 2 * a[i + 1] + a[i + 2];
        hd[i] = a[i + 2] - a[i];
    }
}

// Edge bits of one row of an existing edge map (pixel == 255).
template <bool FAST>
__device__ __forceinline__ uint32_t row_edge_bits(const SobelDesc& d, int y, int x0, bool active,
                                                  int lane) {
    uint32_t p[4];
    int left, right;
    load_row<FAST>(d.img, d.W, d.H, d.pitch, y, x0, active, lane, p, left, right);
    uint32_t bits = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        uint32_t b = (p[i >> 2] >> ((i & 3) * 8)) & 0xFFu;
        bits |= (uint32_t)(b == 255u && x0 + i < d.W) << i;
    }
    return bits;
}

// Writes one tile row (8 rows x this wave's 1024 columns) into the list.
__device__ __forceinline__ void compact_tile_row(const SobelDesc& d, const ListLayout& L, int chunk,
                                                 int ty, uint64_t m0, uint64_t m1, int lane) {
    const uint32_t ca = (uint32_t)__popcll(m0);
    const uint32_t cb = (uint32_t)__popcll(m1);
    const uint32_t tot = ca + cb;
    uint32_t incl = tot;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t t = (uint32_t)__shfl_up((int)incl, o);
        if (lane >= o) incl += t;
    }
    const uint32_t off = incl - tot;
    const uint32_t total = (uint32_t)__shfl((int)incl, kWave - 1);
    const int seg = ty * L.nchunk + chunk;
    uint32_t* list = d.list;
    if (lane == 0) gst(list + seg, total);
    uint32_t* info = list + L.off_info + (size_t)ty * L.tw;
    const int txa = chunk * kTilesPerChunk + 2 * lane;
    if (txa < L.tw) gst(info + txa, (ca << 16) | off);
    if (txa + 1 < L.tw) gst(info + txa + 1, (cb << 16) | (off + ca));
    if (total == 0) return;
    uint32_t* ents = list + L.off_ent + (size_t)seg * kSegCap;
    const int ntiles = min(kTilesPerChunk, L.tw - chunk * kTilesPerChunk);
    const uint32_t ybase = (uint32_t)(ty * kTile + (lane >> 3)) << 16;
    const int npairs = (ntiles + 1) >> 1;
    for (int src = 0; src < npairs; ++src) {
        const uint32_t src_tot = (uint32_t)__builtin_amdgcn_readlane((int)tot, src);
        if (src_tot == 0) continue;
        const uint32_t src_off = (uint32_t)__builtin_amdgcn_readlane((int)off, src);
        const uint32_t src_ca = (uint32_t)__builtin_amdgcn_readlane((int)ca, src);
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const uint64_t mm = half ? m1 : m0;
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)mm, src);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(mm >> 32), src);
            if ((lo | hi) == 0) continue;
            const uint32_t start = src_off + (half ? src_ca : 0u);
            const uint64_t m = ((uint64_t)hi << 32) | lo;
            if ((m >> lane) & 1ull) {
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
                const uint32_t x = (uint32_t)((chunk * kTilesPerChunk + 2 * src + half) * kTile + (lane & 7));
                gst(ents + start + rank, ybase | x);
            }
        }
    }
}

template <bool FAST>
__device__ __forceinline__ void sobel_row_out(const SobelDesc& d, int y, int x0, bool active,
                                              const int (&hsU)[16], const int (&hdU)[16],
                                              const int (&hdM)[16], const int (&hsD)[16],
                                              const int (&hdD)[16], uint32_t& bits) {
    uint32_t eb[4] = {0, 0, 0, 0}, mb[4] = {0, 0, 0, 0};
    bits = 0;
    const bool ring_row = (d.border_mode == 1) && (y == 0 || y == d.H - 1);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int gx = hdU[i] + 2 * hdM[i] + hdD[i];
        const int gy = hsD[i] - hsU[i];
        const int g = abs(gx) + abs(gy);
        const int x = x0 + i;
        bool e = (g > d.threshold) && (x < d.W);
        if (d.border_mode == 1 && (ring_row || x == 0 || x == d.W - 1)) e = false;
        bits |= (uint32_t)e << i;
        eb[i >> 2] |= (e ? 0xFFu : 0u) << ((i & 3) * 8);
        mb[i >> 2] |= (uint32_t)min(g, 255) << ((i & 3) * 8);
    }
    if (!active) return;
    const size_t o = (size_t)y * d.W + x0;
    if (FAST) {
        gst4(d.edges + o, u32x4{eb[0], eb[1], eb[2], eb[3]});
        if (d.mag) gst4(d.mag + o, u32x4{mb[0], mb[1], mb[2], mb[3]});
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (x0 + i < d.W) {
                d.edges[o + i] = (uint8_t)(eb[i >> 2] >> ((i & 3) * 8));
                if (d.mag) d.mag[o + i] = (uint8_t)(mb[i >> 2] >> ((i & 3) * 8));
            }
        }
    }
}

template <bool FAST, int MODE>
__device__ void sobel_item(const SobelDesc& d, int item) {
    const int lane = threadIdx.x & (kWave - 1);
    const ListLayout L = list_layout(d.W, d.H);
    const int chunk = item % L.nchunk;
    const int strip = item / L.nchunk;
    const int x0 = chunk * kChunkPx + lane * 16;
    const bool active = x0 < d.W;
    const int y_begin = strip * kStripRows;
    const int y_end = min(y_begin + kStripRows, d.H);
    uint64_t m0 = 0, m1 = 0;
    uint32_t nedge = 0;

    auto account = [&](int y, uint32_t bits) {
        nedge += (uint32_t)__popc(bits);
        const int ly = y & (kTile - 1);
        m0 |= (uint64_t)(bits & 0xFFu) << (ly * 8);
        m1 |= (uint64_t)((bits >> 8) & 0xFFu) << (ly * 8);
        if (ly == kTile - 1 || y == y_end - 1) {
            if (d.list) compact_tile_row(d, L, chunk, y >> 3, m0, m1, lane);
            m0 = 0;
            m1 = 0;
        }
    };

    if (MODE == kModeFromEdges) {
        for (int y = y_begin; y < y_end; ++y) account(y, row_edge_bits<FAST>(d, y, x0, active, lane));
    } else {
        int hsA[16], hdA[16], hsB[16], hdB[16], hsC[16], hdC[16];
        row_filter<FAST>(d, y_begin - 1, x0, active, lane, hsA, hdA);
        row_filter<FAST>(d, y_begin, x0, active, lane, hsB, hdB);
        // rows rotate A -> B -> C without register copies
        for (int y = y_begin; y < y_end; y += 3) {
            uint32_t bits;
            row_filter<FAST>(d, y + 1, x0, active, lane, hsC, hdC);
            sobel_row_out<FAST>(d, y, x0, active, hsA, hdA, hdB, hsC, hdC, bits);
            account(y, bits);
            if (y + 1 >= y_end) break;
            row_filter<FAST>(d, y + 2, x0, active, lane, hsA, hdA);
            sobel_row_out<FAST>(d, y + 1, x0, active, hsB, hdB, hdC, hsA, hdA, bits);
            account(y + 1, bits);
            if (y + 2 >= y_end) break;
            row_filter<FAST>(d, y + 3, x0, active, lane, hsB, hdB);
            sobel_row_out<FAST>(d, y + 2, x0, active, hsC, hdC, hdA, hsB, hdB, bits);
            account(y + 2, bits);
        }
    }
    if (d.edge_count) {
        uint32_t s = nedge;
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) s += (uint32_t)__shfl_xor((int)s, o);
        if (lane == 0 && s) atomicAdd(d.edge_count, s);
    }
}

template <bool FAST, int MODE>
__global__ void __launch_bounds__(kWave * kSobelWaves) k_sobel(SobelDesc d, int n_items) {
    const int item = blockIdx.x * kSobelWaves + (threadIdx.x >> 6);
    if (item >= n_items) return;  // whole wave leaves; no barriers in this kernel
    sobel_item<FAST, MODE>(d, item);
}

// Batched, persistent: each wave walks the (frame, item) table with a grid
// stride.  Frames of any size and alignment mix in one launch; the aligned
// fast path is chosen per frame.
__global__ void __launch_bounds__(kWave * kSobelWaves)
    k_sobel_batch(const SobelDesc* __restrict__ descs, const int2* __restrict__ items, int n_items) {
    const int wave = threadIdx.x >> 6;
    for (int it = blockIdx.x * kSobelWaves + wave; it < n_items; it += gridDim.x * kSobelWaves) {
        const int2 w = items[it];
        if (w.x < 0) continue;
        const SobelDesc d = descs[w.x];
        if (d.fast) sobel_item<true, kModeSobel>(d, w.y);
        else sobel_item<false, kModeSobel>(d, w.y);
    }
}

__global__ void k_fill_u32(uint32_t* p, size_t n, uint32_t v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace lane

using namespace lane;

// Host-side launchers (called by the C ABI after validation).
extern "C" LANE_INTERNAL hipError_t lane_launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

extern "C" LANE_INTERNAL int lane_sobel_items(int W, int H) {
    const ListLayout L = list_layout(W, H);
    return L.nchunk * ((H + kStripRows - 1) / kStripRows);
}

extern "C" LANE_INTERNAL int lane_sobel_fast_ok(const SobelDesc* dp, int mode) {
    const SobelDesc& d = *dp;
    return ((uintptr_t)d.img % 16 == 0) && (d.pitch % 16 == 0) && (d.W % 16 == 0) &&
           (mode == kModeFromEdges ||
            (((uintptr_t)d.edges % 16 == 0) && ((uintptr_t)d.mag % 16 == 0)));
}

extern "C" LANE_INTERNAL hipError_t lane_launch_sobel_batch(const SobelDesc* descs, const int2* items, int n_items,
                                              int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_sobel_batch, dim3(grid), dim3(kWave * kSobelWaves), 0, s, descs, items,
                       n_items);
    return hipGetLastError();
}

extern "C" LANE_INTERNAL int lane_sobel_batch_occupancy() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_sobel_batch, kWave * kSobelWaves, 0) !=
        hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

extern "C" LANE_INTERNAL hipError_t lane_launch_sobel(const SobelDesc* dp, int mode, hipStream_t s) {
    const SobelDesc& d = *dp;
    const int n_items = lane_sobel_items(d.W, d.H);
    const unsigned blocks = (unsigned)((n_items + kSobelWaves - 1) / kSobelWaves);
    const bool fast = ((uintptr_t)d.img % 16 == 0) && (d.pitch % 16 == 0) && (d.W % 16 == 0) &&
                      (mode == kModeFromEdges ||
                       (((uintptr_t)d.edges % 16 == 0) && ((uintptr_t)d.mag % 16 == 0)));
    const dim3 grid(blocks), block(kWave * kSobelWaves);
    if (mode == kModeSobel) {
        if (fast) hipLaunchKernelGGL((k_sobel<true, kModeSobel>), grid, block, 0, s, d, n_items);
        else hipLaunchKernelGGL((k_sobel<false, kModeSobel>), grid, block, 0, s, d, n_items);
    } else {
        if (fast) hipLaunchKernelGGL((k_sobel<true, kModeFromEdges>), grid, block, 0, s, d, n_items);
        else hipLaunchKernelGGL((k_sobel<false, kModeFromEdges>), grid, block, 0, s, d, n_items);
    }
    return hipGetLastError();
}
