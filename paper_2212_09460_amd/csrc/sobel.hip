// Fused Sobel + binarize + edge compaction for gfx950.
//
// What is computed (Sec. 2.1 Eq. (1), Sec. 2.2, zero padding Sec. 3.1/4.1):
//   gx = [1 2 1]^T x [-1 0 1] correlation, gy its transpose, pixels outside
//   the frame read as 0; edge = 255 iff |gx| + |gy| > threshold, else 0;
//   mag = min(|gx| + |gy|, 255).
//
// Work decomposition: one wave walks a strip of 32 rows x 1024 columns; each
// lane owns 16 adjacent columns, read with one 128-bit load per row, so a
// wave moves 1 KB per row in a single coalesced instruction.  Loads run six
// rows ahead of the arithmetic (a ring of raw rows in registers) so enough
// bytes are in flight to cover HBM latency.  The 3x3 stencil is split into a
// horizontal pass per row ([1 2 1] smooth, [-1 0 1] difference, the two
// neighbour bytes come from the adjacent lanes) and a vertical pass over
// three rows held in registers.  All of it runs on packed pairs (v_pk_*
// instructions, two pixels per operation), exact (below).
//
// Compaction (the vote reads a list of edge coordinates, Sec. 4.3): after
// every 8 rows each lane holds the 64-bit edge masks of its two 8x8 tiles.
// Tile counts are prefix-summed across the wave (the segment offsets); each
// lane places the coordinates of its two tiles' edge pixels in the wave's
// LDS stage, and the wave writes the stage out with coalesced stores.
#include "lane_entry.h"

namespace lane {

enum { kModeSobel = 0, kModeFromEdges = 1 };

// Stencil arithmetic runs on packed half-precision pairs holding the integer
// values scaled by 2^-24: a pixel byte b in the low byte of a 16-bit half IS
// the half-precision number b * 2^-24 (a subnormal), and every intermediate
// (|values| <= 2040, integers) is an integer multiple of 2^-24 below 2^-13,
// so each addition, doubling and difference is exact.  Packed half
// instructions give fused 2a + b and an absolute value in one operation each,
// which the 16-bit integer ones do not.
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

// 16 pixels of one row for one lane, plus the neighbours the lane cannot get
// from its own wave (lane 0's left, lane 63's right; others come by shuffle)
struct RawRow {
    u32x4 v;
    uint32_t l, r;  // left and right neighbour bytes, kept as loaded (no
                    // arithmetic on a load result here: that would make the
                    // wave wait for every load in flight)
};

// Rows of a frame whose rows are 16-byte aligned are read with raw buffer
// loads over the whole image (base, pitch x H bytes): a lane or row outside
// the frame passes an offset past the end and the hardware returns zeros.
// No branch and no merge of loaded and zero values, so the loads kept in
// flight across the row loop never force a wait for all of them.

template <bool FAST>
__device__ __forceinline__ RawRow load_raw(const uint8_t* __restrict__ img, __amdgpu_buffer_rsrc_t rsrc,
                                           int W, int H, int pitch, int y, int x0, bool active,
                                           int lane) {
    RawRow o;
    const bool yin = (y >= 0) && (y < H);
    if (FAST) {
        const bool ok = active && yin;
        const uint32_t off = ok ? (uint32_t)(y * pitch + x0) : kBufOutside;
        o.v = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, off, 0, 0));
        o.l = __builtin_amdgcn_raw_buffer_load_b8(rsrc, (ok && lane == 0 && x0 > 0) ? off - 1u : kBufOutside,
                                                  0, 0);
        o.r = __builtin_amdgcn_raw_buffer_load_b8(
            rsrc, (ok && lane == kWave - 1 && x0 + 16 < W) ? off + 16u : kBufOutside, 0, 0);
        return o;
    }
    o.v = u32x4{0u, 0u, 0u, 0u};
    o.l = 0;
    o.r = 0;
    if (!(active && yin)) return o;
    const uint8_t* row = img + (size_t)y * pitch;
    uint32_t p[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int x = x0 + i;
        const uint32_t b = (x < W) ? (uint32_t)gld(row + x) : 0u;
        p[i >> 2] |= b << ((i & 3) * 8);
    }
    o.v = u32x4{p[0], p[1], p[2], p[3]};
    o.l = (x0 > 0) ? gld(row + x0 - 1) : 0u;
    o.r = (x0 + 16 < W) ? gld(row + x0 + 16) : 0u;
    return o;
}

// DPP controls: every lane takes the value of lane - 1 / lane + 1
constexpr int kDppWaveShr1 = 0x138;
constexpr int kDppWaveShl1 = 0x130;

// Horizontal pass on packed pairs: pixel pair k = (a[2k], a[2k+1]).
struct HRow {
    h2 hs[8];  // [1 2 1] smooth
    h2 hd[8];  // [-1 0 1] difference
};

template <bool FAST>
__device__ __forceinline__ void hfilter(const RawRow& r, int lane, HRow& h) {
    int left = (int)r.l, right = (int)r.r;
    if (FAST) {
        // neighbours from the adjacent lanes by whole-wave DPP shifts by one
        // lane (lane 0 / 63 loaded theirs)
        const uint32_t up = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)r.v.w, kDppWaveShr1, 0xF, 0xF, false);
        const uint32_t dn = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)r.v.x, kDppWaveShl1, 0xF, 0xF, false);
        if (lane > 0) left = (int)(up >> 24);
        if (lane < kWave - 1) right = (int)(dn & 0xFFu);
    }
    const uint32_t dw[4] = {r.v.x, r.v.y, r.v.z, r.v.w};
    h2 P[8], S[9];
    // P[k] = (a[2k], a[2k+1]);  S[k] = (a[2k-1], a[2k]) with a[-1] = left, a[16] = right
#pragma unroll
    for (int k = 0; k < 8; ++k)
        P[k] = __builtin_bit_cast(h2, __builtin_amdgcn_perm(0u, dw[k >> 1], (k & 1) ? 0x0c030c02u : 0x0c010c00u));
    S[0] = __builtin_bit_cast(h2, __builtin_amdgcn_perm(dw[0], (uint32_t)left, 0x0c040c00u));
#pragma unroll
    for (int k = 1; k < 8; ++k) {
        if (k & 1) S[k] = __builtin_bit_cast(h2, __builtin_amdgcn_perm(0u, dw[k >> 1], 0x0c020c01u));
        else S[k] = __builtin_bit_cast(h2, __builtin_amdgcn_perm(dw[k >> 1], dw[(k >> 1) - 1], 0x0c040c03u));
    }
    S[8] = __builtin_bit_cast(h2, __builtin_amdgcn_perm((uint32_t)right, dw[3], 0x0c040c03u));
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        h.hs[k] = (S[k] + S[k + 1]) + P[k] * (_Float16)2;
        h.hd[k] = S[k + 1] - S[k];
    }
}

// Per-lane constants of the output masking: which of the lane's 16 columns
// may be edges (inside the frame; not on the ring in border mode 1).
struct ColMask {
    uint32_t bits;   // bit i: column x0 + i may be an edge
    uint32_t sel[4]; // byte selectors of the edge-map dwords (below): sign of the pixel's half, or 0
};

__device__ __forceinline__ ColMask col_mask(const SobelDesc& d, int x0) {
    ColMask c;
    c.bits = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int x = x0 + i;
        const bool ok = (x < d.W) && !(d.border_mode == 1 && (x == 0 || x == d.W - 1));
        c.bits |= (uint32_t)ok << i;
    }
    // v_perm_b32 selectors 8..11 give 0xFF or 0x00 by bit 15 / 31 of the
    // second and first source; 12 gives 0x00
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        uint32_t b = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) b |= (((c.bits >> (4 * w + i)) & 1u) ? (uint32_t)(8 + i) : 0x0Cu) << (8 * i);
        c.sel[w] = b;
    }
    return c;
}

// Vertical pass and output of row y.  X = hd(y-1) + 2 hd(y) and
// HU = hs(y-1) were kept from earlier rows; D is row y+1.  Returns the row's
// 16 edge bits.
template <bool FAST>
__device__ __forceinline__ uint32_t vout(const SobelDesc& d, int y, int x0, bool active,
                                         const ColMask& cm, const h2 (&X)[8],
                                         const h2 (&HU)[8], const HRow& D) {
    const h2 TT = __builtin_bit_cast(h2, (uint32_t)d.threshold * 0x00010001u);
    h2 g[8], ef[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const h2 gx = X[k] + D.hd[k];
        const h2 gy = D.hs[k] - HU[k];
        g[k] = __builtin_elementwise_abs(gx) + __builtin_elementwise_abs(gy);
        // threshold - g is negative exactly when g > threshold, so the sign
        // (bit 15 of each half) is the pixel's edge flag
        ef[k] = TT - g[k];
    }
    const bool ring_row = (d.border_mode == 1) && (y == 0 || y == d.H - 1);
    uint32_t eb[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        // pixels 4w .. 4w+3 are the halves of pairs 2w, 2w+1: one byte
        // permute turns their flag bits into 0xFF / 0x00 and zeroes the
        // columns that may not be edges
        eb[w] = ring_row ? 0u
                         : __builtin_amdgcn_perm(__builtin_bit_cast(uint32_t, ef[2 * w + 1]),
                                                 __builtin_bit_cast(uint32_t, ef[2 * w]), cm.sel[w]);
    }
    // 16 edge bits: each byte's low bit weighted 1, 2, 4, 8 (16 .. 128 for
    // the next dword) by unsigned byte dot products
    const uint32_t lo = __builtin_amdgcn_udot4(eb[1] & 0x01010101u, 0x80402010u,
                                               __builtin_amdgcn_udot4(eb[0] & 0x01010101u, 0x08040201u, 0u, false),
                                               false);
    const uint32_t hi = __builtin_amdgcn_udot4(eb[3] & 0x01010101u, 0x80402010u,
                                               __builtin_amdgcn_udot4(eb[2] & 0x01010101u, 0x08040201u, 0u, false),
                                               false);
    const uint32_t bits = lo | (hi << 8);
    if (active) {
        const size_t o = (size_t)y * d.W + x0;
        uint32_t mb[4] = {0u, 0u, 0u, 0u};
        if (d.mag) {
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                // min(g, 255): for values up to 255 the half's low byte is the value
                const h2 c255 = __builtin_bit_cast(h2, 0x00FF00FFu);
                const h2 m0 = __builtin_elementwise_min(g[2 * w], c255);
                const h2 m1 = __builtin_elementwise_min(g[2 * w + 1], c255);
                mb[w] = __builtin_amdgcn_perm(__builtin_bit_cast(uint32_t, m1),
                                              __builtin_bit_cast(uint32_t, m0), 0x06040200u);
            }
        }
        if (FAST) {
            // written once and not read again by the pass: streaming store
            __builtin_nontemporal_store(u32x4{eb[0], eb[1], eb[2], eb[3]},
                                        (LANE_GLOBAL u32x4*)(d.edges + o));
            if (d.mag) gst4(d.mag + o, u32x4{mb[0], mb[1], mb[2], mb[3]});
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                if (x0 + i < d.W) {
                    gst(d.edges + o + i, (uint8_t)(eb[i >> 2] >> ((i & 3) * 8)));
                    if (d.mag) gst(d.mag + o + i, (uint8_t)(mb[i >> 2] >> ((i & 3) * 8)));
                }
            }
        }
    }
    return bits;
}

// Edge bits of one row of an existing edge map (pixel == 255).
__device__ __forceinline__ uint32_t raw_edge_bits(const RawRow& r, int x0, int W) {
    const uint32_t dw[4] = {r.v.x, r.v.y, r.v.z, r.v.w};
    uint32_t bits = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint32_t b = (dw[i >> 2] >> ((i & 3) * 8)) & 0xFFu;
        bits |= (uint32_t)(b == 255u && x0 + i < W) << i;
    }
    return bits;
}

// Writes one tile row (8 rows x this wave's 1024 columns) into the list.
// Each lane first places its two tiles' coordinates in the wave's LDS
// stage (at their final offsets), then the wave copies the stage out with
// 128-bit stores, so every store instruction writes 1 KB of consecutive
// entries instead of 64 scattered words.  A tile row with more than CAP
// edges goes out in several passes of CAP entries: in each, the lanes whose
// runs lie inside the pass write them the fast way, the one or two lanes
// whose runs cross its bounds entry by entry.  Two stage sizes: 2048 entries
// (8 KB per wave) keeps enough Sobel workgroups per CU for a pass over many
// frames; 4096 (16 KB per wave, two workgroups per CU) puts nearly every
// tile row of a road frame in one pass, which shortens the slowest wave of a
// pass over one or a few frames (a 720p frame 22 -> 14 us).
constexpr int kStageCap = 2048;
constexpr int kStageCapLatency = 4096;

static_assert(kWave * kSobelWaves == 256, "one table entry per thread");

// lut[b]: the columns of the set bits of row byte b, in order, one per byte
__device__ __forceinline__ uint2 row_byte_columns(uint32_t b) {
    uint64_t v = 0;
    int n = 0;
    for (int c = 0; c < 8; ++c) {
        if ((b >> c) & 1u) {
            v |= (uint64_t)c << (8 * n);
            ++n;
        }
    }
    return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
}

template <int CAP>
__device__ __forceinline__ void compact_tile_row(const SobelDesc& d, const ListLayout& L, int chunk,
                                                 int ty, uint64_t m0, uint64_t m1, int lane,
                                                 uint32_t* __restrict__ stage,
                                                 const uint2* __restrict__ lut) {
    const uint32_t ca = (uint32_t)__popcll(m0);
    const uint32_t cb = (uint32_t)__popcll(m1);
    const uint32_t tot = ca + cb;
    uint32_t incl = tot;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)incl, o);
        if (lane >= o) incl += t;
    }
    const uint32_t off = incl - tot;
    const uint32_t total = (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)incl, kWave - 1));
    const int seg = ty * L.nchunk + chunk;
    uint32_t* list = d.list;
    if (lane == 0) gst(list + seg, total);
    uint32_t* info = list + L.off_info + (size_t)ty * L.tw;
    const int txa = chunk * kTilesPerChunk + 2 * lane;
    if (txa < L.tw) gst(info + txa, (ca << 16) | off);
    if (txa + 1 < L.tw) gst(info + txa + 1, (cb << 16) | (off + ca));
    if (total == 0) return;
    uint32_t* dst = list + L.off_ent + (size_t)seg * kSegCap;
    const uint32_t xa = (uint32_t)(txa * kTile);
    const uint32_t y0 = (uint32_t)(ty * kTile) << 16;
    const uint32_t end = off + tot;
    for (uint32_t p0 = 0; p0 < total; p0 += CAP) {
        if (off >= p0 && end <= p0 + (uint32_t)CAP) {
            // The run inside this pass.  The lane's 16 row bytes (tile a
            // rows 0-7, tile b rows 0-7) in order: each writes its entries
            // as a block of 8 (the row's columns from the table; the slots
            // past its count hold junk that the next row byte overwrites),
            // as long as the block ends inside the lane's run.  The row
            // bytes after that (their entries are the run's last seven or
            // fewer) go one entry at a time.
            uint32_t p = off - p0, nfull = 0;  // stage positions: entry p0 + i at stage[i]
            const uint32_t end_s = end - p0;
#pragma unroll 1  // (unrolled, the table reads of all 16 hoist and spill)
            for (int g = 0; g < 4; ++g) {  // four row bytes at a time: their table reads go out together
                const uint32_t w = (uint32_t)((g < 2 ? m0 : m1) >> (32 * (g & 1)));
                uint2 cols[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) cols[i] = lut[(w >> (8 * i)) & 0xFFu];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int j = 4 * g + i;
                    const uint32_t rb = y0 + ((uint32_t)(j & 7) << 16) + xa + (j < 8 ? 0u : (uint32_t)kTile);
                    if (p + 8u <= end_s) {
                        uint32_t* q = stage + p;
#pragma unroll
                        for (int c = 0; c < 4; ++c) q[c] = rb + ((cols[i].x >> (8 * c)) & 0xFFu);
#pragma unroll
                        for (int c = 0; c < 4; ++c) q[4 + c] = rb + ((cols[i].y >> (8 * c)) & 0xFFu);
                        ++nfull;
                    }
                    p += (uint32_t)__popc((w >> (8 * i)) & 0xFFu);
                }
            }
            // row bytes nfull .. 15
            uint64_t t0 = nfull >= 8 ? 0ull : (m0 >> (8 * nfull)) << (8 * nfull);
            uint64_t t1 = nfull <= 8 ? m1 : nfull >= 16 ? 0ull : (m1 >> (8 * (nfull - 8))) << (8 * (nfull - 8));
            uint32_t e = end_s - (uint32_t)(__popcll(t0) + __popcll(t1));
            while (t0 | t1) {
                const bool in_a = t0 != 0;
                const uint64_t m = in_a ? t0 : t1;
                const uint32_t bit = (uint32_t)__builtin_ctzll(m);
                stage[e++] = y0 + ((bit >> 3) << 16) + xa + (in_a ? 0u : (uint32_t)kTile) + (bit & 7u);
                if (in_a) t0 &= t0 - 1ull;
                else t1 &= t1 - 1ull;
            }
        } else if (off < p0 + (uint32_t)CAP && end > p0) {
            // a run crossing the pass's bounds: tile a then tile b,
            // row-major in a tile; only the entries of this pass land in the
            // stage
            uint32_t e = off - p0;  // wraps for runs before the pass: then >= CAP
#pragma unroll
            for (int q = 0; q < 4; ++q) {  // (tile a, rows 0-3), (a, 4-7), (b, 0-3), (b, 4-7)
                uint32_t m = (uint32_t)(((q < 2) ? m0 : m1) >> ((q & 1) * 32));
                const uint32_t base = y0 + ((uint32_t)((q & 1) * 4) << 16) + xa + (uint32_t)((q >> 1) * kTile);
                while (m) {
                    const uint32_t bit = (uint32_t)__builtin_ctz(m);
                    m &= m - 1u;
                    if (e < (uint32_t)CAP) stage[e] = base + ((bit >> 3) << 16) + (bit & 7u);
                    ++e;
                }
            }
        }
        // the stage is read by other lanes of the same wave: order the LDS
        // writes before the reads (one wave, so no workgroup barrier)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t n = min(total - p0, (uint32_t)CAP);
        // whole 16-byte groups; the last may carry up to three stale words
        // past the segment's count, inside the segment's capacity
        for (uint32_t g = (uint32_t)lane * 4u; g < n; g += 4u * kWave)
            // streaming store too: a launch over many frames reads the list
            // back only after the whole pass, long after any cache held it
            __builtin_nontemporal_store(*reinterpret_cast<const u32x4*>(stage + g),
                                        (LANE_GLOBAL u32x4*)(dst + p0 + g));
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

template <bool FAST, int MODE, int CAP>
__device__ void sobel_item(const SobelDesc& d, int item, uint32_t* __restrict__ stage,
                           const uint2* __restrict__ lut) {
    const int lane = threadIdx.x & (kWave - 1);
    const ListLayout L = list_layout(d.W, d.H);
    const int chunk = item % L.nchunk;
    const int strip = item / L.nchunk;
    const int x0 = chunk * kChunkPx + lane * 16;
    const bool active = x0 < d.W;
    const int y_begin = strip * d.strip_rows;
    const int y_end = min(y_begin + d.strip_rows, d.H);
    const int y_load_end = min(y_end + 1, d.H);  // rows this strip reads: [y_begin - 1, y_end]
    uint64_t m0 = 0, m1 = 0;
    uint32_t nedge = 0;

    auto account = [&](int y, uint32_t bits) {
        nedge += (uint32_t)__popc(bits);
        const int ly = y & (kTile - 1);
        m0 |= (uint64_t)(bits & 0xFFu) << (ly * 8);
        m1 |= (uint64_t)((bits >> 8) & 0xFFu) << (ly * 8);
    };
    auto flush = [&](int ty) {
        if (d.list) compact_tile_row<CAP>(d, L, chunk, ty, m0, m1, lane, stage, lut);
        m0 = 0;
        m1 = 0;
    };
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)d.img, (short)0, (int)((uint32_t)d.pitch * (uint32_t)d.H), kBufConfig);
    auto load = [&](int y) {
        return load_raw<FAST>(d.img, rsrc, d.W, d.H, d.pitch, y, x0, active && y < y_load_end, lane);
    };

    if (MODE == kModeFromEdges) {
        for (int y = y_begin; y < y_end; ++y) {
            account(y, raw_edge_bits(load(y), x0, d.W));
            if ((y & (kTile - 1)) == kTile - 1 || y == y_end - 1) flush(y >> 3);
        }
    } else {
        const ColMask cm = col_mask(d, x0);
        // raw rows y+1 .. y+4 in flight; Q0/Q1 alternate as "row y" and
        // "row y+1"; X = hd(y-1) + 2 hd(y) and HU = hs(y-1) carry over
        // (the two rows needed first are issued first)
        const RawRow Rm = load(y_begin - 1), Rc = load(y_begin);
        RawRow R0 = load(y_begin + 1), R1 = load(y_begin + 2);
        RawRow R2 = load(y_begin + 3), R3 = load(y_begin + 4);
        __builtin_amdgcn_sched_barrier(0);  // all six rows go out before the first one is used
        HRow Q0, Q1;
        h2 X[8];
        h2 HU[8];
        hfilter<FAST>(Rm, lane, Q1);
        hfilter<FAST>(Rc, lane, Q0);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            X[k] = Q1.hd[k] + Q0.hd[k] * (_Float16)2;
            HU[k] = Q1.hs[k];
        }
    // Every step runs (rows past the strip's end are computed and dropped:
    // no store, no bits), so no branch surrounds the loads and the waits
    // for rows in flight stay partial.
#define LANE_SOBEL_STEP(QC, QN, R_, dy, B_)                                       \
    {                                                                             \
        const int yy = y + (dy);                                                  \
        const bool row_in = yy < y_end;                                           \
        hfilter<FAST>(R_, lane, QN);                                              \
        R_ = load(yy + 5);                                                        \
        B_ = vout<FAST>(d, yy, x0, active && row_in, cm, X, HU, QN);              \
        B_ = row_in ? B_ : 0u;                                                    \
        _Pragma("unroll") for (int k = 0; k < 8; ++k) {                           \
            X[k] = QC.hd[k] + QN.hd[k] * (_Float16)2;                             \
            HU[k] = QC.hs[k];                                                     \
        }                                                                         \
    }
        // strips start on a tile row, so each group of 4 rows is rows 0-3 or
        // 4-7 of its tile row
        for (int y = y_begin; y < y_end; y += 4) {
            uint32_t b0, b1, b2, b3;
            LANE_SOBEL_STEP(Q0, Q1, R0, 0, b0)
            LANE_SOBEL_STEP(Q1, Q0, R1, 1, b1)
            LANE_SOBEL_STEP(Q0, Q1, R2, 2, b2)
            LANE_SOBEL_STEP(Q1, Q0, R3, 3, b3)
            // row r's bits: byte 0 tile a, byte 1 tile b; gather each tile's
            // four row bytes into one dword (row r in byte r)
            const uint32_t t01 = __builtin_amdgcn_perm(b1, b0, 0x05010400u);
            const uint32_t t23 = __builtin_amdgcn_perm(b3, b2, 0x05010400u);
            const uint32_t qa = __builtin_amdgcn_perm(t23, t01, 0x05040100u);
            const uint32_t qb = __builtin_amdgcn_perm(t23, t01, 0x07060302u);
            nedge += (uint32_t)__popc(qa) + (uint32_t)__popc(qb);
            if (y & 4) {
                m0 |= (uint64_t)qa << 32;
                m1 |= (uint64_t)qb << 32;
            } else {
                m0 = qa;
                m1 = qb;
            }
            if (((y + 4) & (kTile - 1)) == 0 || y + 4 >= y_end) flush(y >> 3);
        }
#undef LANE_SOBEL_STEP
    }
    if (d.edge_count) {
        uint32_t s = nedge;
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) s += (uint32_t)__shfl_xor((int)s, o);
        if (lane == 0 && s) atomicAdd(d.edge_count, s);
    }
}

// (one frame: the latency stage)
template <bool FAST, int MODE>
__global__ void __launch_bounds__(kWave * kSobelWaves) __attribute__((amdgpu_waves_per_eu(4)))
    k_sobel(SobelDesc d, int n_items) {
    __shared__ __align__(16) uint32_t s_stage[kSobelWaves * kStageCapLatency];
    __shared__ uint2 s_lut[256];
    s_lut[threadIdx.x] = row_byte_columns(threadIdx.x);  // 256 threads
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int item = blockIdx.x * kSobelWaves + wave;
    if (item >= n_items) return;  // whole wave leaves; no barriers after this
    sobel_item<FAST, MODE, kStageCapLatency>(d, item, s_stage + wave * kStageCapLatency, s_lut);
}

// Batched: each wave walks the (frame, item) table with a grid stride (one
// item per wave when the grid covers the table, the default; several with a
// persistent grid).  Frames of any size mix in one launch; frames whose rows
// are 16-byte aligned go to the vector-load instance, the rest to the byte
// one.
template <bool FAST, int CAP>
__global__ void __launch_bounds__(kWave * kSobelWaves) __attribute__((amdgpu_waves_per_eu(4)))
    k_sobel_batch(const SobelDesc* __restrict__ descs, const int2* __restrict__ items,
                  const int* __restrict__ counts, int group) {
    // items of group 0 (aligned frames) come first, then group 1; the counts
    // live in device memory so a launch can run any selection of frames
    const int first = group == 0 ? 0 : gld(counts);
    const int n_items = gld(counts + group);
    items += first;
    __shared__ __align__(16) uint32_t s_stage[kSobelWaves * CAP];
    __shared__ uint2 s_lut[256];
    s_lut[threadIdx.x] = row_byte_columns(threadIdx.x);  // 256 threads
    __syncthreads();
    // wave-uniform indices, so the table and descriptor loads are scalar
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    for (int it = blockIdx.x * kSobelWaves + wave; it < n_items; it += gridDim.x * kSobelWaves) {
        const int2 w = items[it];
        if (w.x < 0) continue;
        const SobelDesc d = descs[w.x];
        if (!frame_on(d.active)) continue;
        sobel_item<FAST, kModeSobel, CAP>(d, w.y, s_stage + wave * CAP, s_lut);
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

extern "C" LANE_INTERNAL int lane_sobel_items(int W, int H, int strip_rows) {
    const ListLayout L = list_layout(W, H);
    return L.nchunk * ((H + strip_rows - 1) / strip_rows);
}

// The 128-bit path reads the frame as one raw buffer of pitch x H bytes
// (32-bit offsets, out-of-frame reads past its end), so it needs aligned
// rows and a frame below 2^31 bytes.
extern "C" LANE_INTERNAL int lane_sobel_fast_ok(const SobelDesc* dp, int mode) {
    const SobelDesc& d = *dp;
    return ((uintptr_t)d.img % 16 == 0) && (d.pitch % 16 == 0) && (d.W % 16 == 0) &&
           ((int64_t)d.pitch * d.H <= 0x7FFFFFFFll) &&
           (mode == kModeFromEdges ||
            (((uintptr_t)d.edges % 16 == 0) && ((uintptr_t)d.mag % 16 == 0)));
}

extern "C" LANE_INTERNAL hipError_t lane_launch_sobel_batch(const SobelDesc* descs, const int2* items,
                                                            const int* counts, int fast, int latency,
                                                            int grid, hipStream_t s) {
    const dim3 g(grid), blk(kWave * kSobelWaves);
    if (fast && latency)
        hipLaunchKernelGGL((k_sobel_batch<true, kStageCapLatency>), g, blk, 0, s, descs, items, counts, 0);
    else if (fast)
        hipLaunchKernelGGL((k_sobel_batch<true, kStageCap>), g, blk, 0, s, descs, items, counts, 0);
    else if (latency)
        hipLaunchKernelGGL((k_sobel_batch<false, kStageCapLatency>), g, blk, 0, s, descs, items, counts, 1);
    else
        hipLaunchKernelGGL((k_sobel_batch<false, kStageCap>), g, blk, 0, s, descs, items, counts, 1);
    return hipGetLastError();
}

extern "C" LANE_INTERNAL hipError_t lane_launch_sobel(const SobelDesc* dp, int mode, hipStream_t s) {
    const SobelDesc& d = *dp;
    const int n_items = lane_sobel_items(d.W, d.H, d.strip_rows);
    const unsigned blocks = (unsigned)((n_items + kSobelWaves - 1) / kSobelWaves);
    const bool fast = lane_sobel_fast_ok(&d, mode) != 0;
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
