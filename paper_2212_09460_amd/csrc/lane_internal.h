// Internal descriptors and helpers shared by the HIP kernels and the C ABI.
// gfx950 (CDNA4) only: wave64, 160 KB LDS per workgroup.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#define LANE_INTERNAL __attribute__((visibility("hidden")))

// Global-memory accessors.  Pointers read out of descriptor tables are
// generic to the compiler, which then emits flat instructions; flat loads
// share the LDS wait counter, so every wait on them would also drain the
// vote's LDS atomics.  These casts make the accesses global_load/store.
#define LANE_GLOBAL __attribute__((address_space(1)))
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

namespace lane {

template <class T>
__device__ __forceinline__ T gld(const T* p) { return *(const LANE_GLOBAL T*)p; }
template <class T>
__device__ __forceinline__ void gst(T* p, T v) { *(LANE_GLOBAL T*)p = v; }
__device__ __forceinline__ u32x4 gld4(const void* p) { return *(const LANE_GLOBAL u32x4*)p; }
__device__ __forceinline__ void gst4(void* p, u32x4 v) { *(LANE_GLOBAL u32x4*)p = v; }

// Raw buffer loads: an offset past the buffer's size returns zero (used for
// reads outside a frame without branches).
constexpr uint32_t kBufOutside = 0x80000000u;
constexpr int kBufConfig = 0x00020000;  // raw buffer, 32-bit format (gfx9 family)

constexpr int kWave = 64;
constexpr int kTile = 8;                 // edge tiles are 8x8 pixels
constexpr int kChunkPx = 1024;           // one wave covers 64 lanes x 16 px
constexpr int kTilesPerChunk = kChunkPx / kTile;
constexpr int kSegCap = kTile * kChunkPx;  // entries a segment can hold
constexpr int kStripRows = 32;           // default rows one Sobel wave walks down (multiple of 8)
constexpr int kSobelWaves = 4;           // waves per Sobel workgroup
constexpr int kVoteThreads = 1024;       // 16 waves per vote workgroup
constexpr int kVoteLdsWords = 40704;     // accumulator dwords in LDS (159 KB): 1 workgroup/CU
constexpr int kVoteLdsWordsHalf = 20224; // 79 KB: 2 workgroups/CU
constexpr int kMaxT = 64;                // theta rows per vote workgroup (max)

// Layout of the compacted edge list of one frame (offsets in uint32 words).
struct ListLayout {
    int th, tw, nchunk, nseg;
    size_t off_info, off_ent, words;
};

__host__ __device__ inline ListLayout list_layout(int W, int H) {
    ListLayout L;
    L.th = (H + kTile - 1) / kTile;
    L.tw = (W + kTile - 1) / kTile;
    L.nchunk = (W + kChunkPx - 1) / kChunkPx;
    L.nseg = L.th * L.nchunk;
    L.off_info = (size_t)L.nseg;
    L.off_ent = ((L.off_info + (size_t)L.th * L.tw) + 3) & ~(size_t)3;
    L.words = L.off_ent + (size_t)L.nseg * kSegCap;
    return L;
}

// One frame for the Sobel + binarize + compaction pass.
struct SobelDesc {
    const uint8_t* img;
    int W, H, pitch;
    int threshold, border_mode;
    uint8_t* edges;      // [H][W]
    uint8_t* mag;        // [H][W] or null
    uint32_t* list;      // edge list or null
    uint32_t* edge_count;  // device scalar or null (zeroed beforehand)
    int fast;            // 16-byte aligned rows: vector loads/stores (batched path)
    int strip_rows;      // rows per work item, a multiple of 8
    const uint8_t* active;  // batched path: the frame runs iff *active != 0 (null = always)
};

// One frame for the vote.
struct VoteDesc {
    const uint32_t* list;
    int W, H;
    const int16_t* cos_q14;
    const int16_t* sin_q14;
    int n_theta, r_offset, n_r;
    const uint8_t* tile_mask;  // [th][tw] or null
    int32_t* acc;              // [n_theta][n_r]
    uint32_t* dropped;         // device scalar or null (zeroed beforehand)
    int T;                     // theta rows per workgroup (power of two <= 64)
    int log2T;
    int n_slices;
    unsigned long long* keys;  // or null: peak-search block keys written with the rows
    int key_log2;              // cells per key block = 1 << key_log2
    int nbr;                   // key blocks per row
    const uint8_t* active;     // batched path: the frame runs iff *active != 0 (null = always)
    int E;                     // edge split: workgroups per slice, each a 1/E share of the segments,
                               // adding into acc (cleared beforehand); keys must then be null
    int pruned;                // list is a pruned list (PruneDesc) of a frame with tile_mask
};

// One frame for the peak search.
struct PeaksDesc {
    const int32_t* acc;
    int n_theta, n_r, r_offset;
    int k, h_theta, h_r, min_votes;
    int32_t* theta_idx;
    int32_t* r_idx;
    int32_t* votes;
    int32_t* count;
    unsigned long long* keys;  // workspace: one key per block
    int block_log2;            // a block is 1 << block_log2 cells of one row
    int nbr;                   // blocks per row, ceil(n_r / block size)
    int n_blocks;              // n_theta * nbr
    int active_index;          // host bookkeeping: the frame this descriptor belongs to
    const uint8_t* active;     // batched path: the frame runs iff *active != 0 (null = always)
};

// One frame for the coarse-to-fine Hough transform.
struct ProgDesc {
    const uint32_t* list;  // edge list of a W x H frame
    int W, H;
    const int16_t* cos_q14;
    const int16_t* sin_q14;
    int n_theta, D;            // fine accumulator: n_r = 2 D + 1
    int f, w, q, kc, mt, mr;   // theta step, odd r width, (w - 1) / 2, coarse peaks, margins
    int k, ht, hr, min_votes;  // final selection
    int n_c, n_rc, Dc, R, Wc;  // coarse rows / columns / offset, window rows / columns
    float inv_w;               // float(1 / w)
    int T;                     // coarse rows per workgroup (1, 2 or 4)
    int n_slices, n_chunks, groups_per_chunk;  // coarse grid
    int r_chunks, r_parts, wpg, n_wgroups;     // refine grid: edge chunks x window groups;
                                               // a segment is cut into r_parts parts
    int32_t* coarse_acc;  // [n_c][n_rc]
    int32_t* cpk;         // coarse peaks: theta[kc], r[kc], votes[kc], count
    int32_t* windows;     // [kc][R][Wc]
    int32_t* cand;        // [kc][3]: fine theta, fine r_idx, count (-1: none)
    int32_t* theta_idx;   // [k]
    int32_t* r_idx;       // [k]
    int32_t* votes;       // [k]
    int32_t* count;       // scalar
};

// LDS bytes of a refine workgroup holding wpg windows of R x Wc cells:
// the cells, two words per (window, row), five per window.
inline size_t lane_prog_refine_lds(int wpg, int R, int Wc) {
    return ((size_t)wpg * R * Wc + 2 * (size_t)wpg * R + 5 * (size_t)wpg) * sizeof(int32_t);
}
constexpr int kProgRefineLdsMax = 65536;  // bytes
constexpr int kProgTargetGroups = 2048;    // coarse workgroups a launch aims at (8 per CU)
constexpr int kProgRefineGroups = 512;     // refine workgroups a launch aims at
constexpr int kProgCoarseLdsMax = 98304;  // bytes

// One frame of a split vote with a tile mask: the pruned copy of its edge
// list (same size and layout; word seg holds the count of segment seg's
// entries from tiles that vote every row, word off_info + seg the count of
// its band-restricted entries, which sit at the end of the segment's slot).
struct PruneDesc {
    const uint32_t* list;      // the frame's edge list
    uint32_t* pruned;          // the pruned list
    const uint8_t* tile_mask;  // [ceil(H/8)][ceil(W/8)] band bits
    int W, H;
    int vote;                  // index of the frame's VoteDesc in the plan
    const uint8_t* active;     // the frame runs iff *active != 0 (null = always)
};

// Band bits of theta row k: bit b is set when k lies in band b, the
// quarter turn of rows starting at row b * n_theta / 8 (cyclically).
__device__ __forceinline__ int band_bits_dev(int n_theta, int k) {
    int bits = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const int start = (b * n_theta) / 8;
        int dd = (k - start) % n_theta;
        if (dd < 0) dd += n_theta;
        if (dd < n_theta / 4) bits |= 1 << b;
    }
    return bits;
}

// Most frame pixels (x, y) in [0, W) x [0, H) that two neighbouring r cells
// of one theta row with table entries (C, S) can collect.  Cells u and u + 1
// hold the pixels with x*C + y*S in one half-open interval of width 2^15:
// on one image row y that is a run of at most ceil(2^15 / |C|) columns (all
// W when C = 0), and only rows y with y*S inside an interval of width
// 2^15 + (W - 1)|C| meet it, at most ceil((2^15 + (W - 1)|C|) / |S|) of them
// (all H when S = 0).  The same holds with x and y exchanged; the smaller
// product bounds the count.  For a rotation row (max(|C|, |S|) >= 2^14/sqrt 2)
// this is at most 3 max(W, H).
__host__ __device__ inline long long vote_pair_bound(int W, int H, int C, int S) {
    const long long ac = C < 0 ? -(long long)C : C, as = S < 0 ? -(long long)S : S;
    const long long w = W, h = H;
    long long ym = as ? (32768 + (w - 1) * ac + as - 1) / as : h;
    ym = ym < h ? ym : h;
    long long per_y = ac ? (32768 + ac - 1) / ac : w;
    ym *= per_y < w ? per_y : w;
    long long xm = ac ? (32768 + (h - 1) * as + ac - 1) / ac : w;
    xm = xm < w ? xm : w;
    long long per_x = as ? (32768 + as - 1) / as : h;
    xm *= per_x < h ? per_x : h;
    return ym < xm ? ym : xm;
}

// The paired LDS counters keep the sum of a cell pair in 14 bits.
constexpr long long kPairCountMax = 16383;

// One frame for the line segments along its peaks.
struct LinesDesc {
    const uint8_t* edges;  // [H][W], 255 = edge
    int W, H;
    const int16_t* cos_q14;
    const int16_t* sin_q14;
    int n_theta, r_offset;
    const int32_t* theta_idx;  // [k]
    const int32_t* r_idx;      // [k]
    const int32_t* count;      // device scalar or null: peaks j >= *count are empty
    int k;
    int fill_gap, min_length, max_seg;
    int32_t* segs;       // [k][max_seg][4]
    int32_t* seg_count;  // [k]
    int32_t* npts;       // [k] or null
    const uint8_t* active;  // batched path: the frame runs iff *active != 0 (null = always)
};

// LDS of one line workgroup: points (4 B) and segment starts (2 B) for up to
// two points per step of the frame's longer side.
inline size_t lines_lds_bytes(int W, int H) { return (size_t)6 * 2 * (size_t)(W > H ? W : H); }

// Peak-search key of a cell: one unsigned max picks the largest count and,
// among equal counts, the smallest theta-major index.
__device__ __forceinline__ unsigned long long make_key(int v, uint32_t idx) {
    return ((unsigned long long)((uint32_t)v ^ 0x80000000u) << 32) |
           (unsigned long long)(0xFFFFFFFFu - idx);
}

// One step of a wave reduction: the larger of v and the value DPP control
// CTRL brings from another lane (lanes outside ROW_MASK keep v).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned long long max_dpp_u64(unsigned long long v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)v, (int)(uint32_t)v, CTRL,
                                                              ROW_MASK, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(v >> 32), (int)(uint32_t)(v >> 32),
                                                              CTRL, ROW_MASK, 0xF, false);
    const unsigned long long w = ((unsigned long long)hi << 32) | lo;
    return w > v ? w : v;
}

// Maximum over each DPP row of 16 lanes, returned to every lane of the row.
__device__ __forceinline__ unsigned long long row_max_u64(unsigned long long v) {
    v = max_dpp_u64<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v = max_dpp_u64<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v = max_dpp_u64<0x141, 0xF>(v);  // row_half_mirror
    return max_dpp_u64<0x140, 0xF>(v);  // row_mirror
}

// Maximum over the 64 lanes, returned to every lane.  Data movement by DPP
// (VALU), not by LDS permutes, which would queue behind a vote's LDS
// atomics: swaps within quads, then mirrors within half-rows and rows of 16
// make every row uniform, two row broadcasts carry the rows' maxima to lane
// 63, and a readlane hands that to the wave.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
    v = row_max_u64(v);
    v = max_dpp_u64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v = max_dpp_u64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

constexpr int kPeaksMaxBlocksLds = 8192;

// A frame switched off in a batched launch keeps its previous outputs.
__device__ __forceinline__ bool frame_on(const uint8_t* active) { return !active || gld(active) != 0; }  // keys held in LDS by the select pass

inline int ilog2_floor(unsigned v) { int r = -1; while (v) { v >>= 1; ++r; } return r; }

}  // namespace lane
