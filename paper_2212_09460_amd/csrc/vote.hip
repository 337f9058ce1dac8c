// Hough vote for gfx950: theta-slice accumulators in LDS.
//
// What is computed (Sec. 2.3 Eq. (3)): every edge pixel (x, y) votes in
// every theta row k at r_idx = floor((x*C[k] + y*S[k] + 2^13) / 2^14) +
// r_offset of an int32 accumulator [n_theta][n_r]; votes outside [0, n_r)
// are dropped and counted.
//
// Design.  As in the per-angle partition of Sec. 4.3, a workgroup owns a
// slice of T theta rows and keeps them in LDS while it streams the whole
// compacted edge list.  On gfx950 the slice is sized to the 160 KB LDS
// rather than one row per block: each row only stores the r range its angle
// can reach inside the frame (found from the four corners, where the
// monotone r is extreme), so T = 16 rows of a 1080p frame fit.  A wave's 64
// lanes are split into 64/T edge slots x T theta rows; each lane loads four
// packed (y << 16 | x) entries with one 128-bit load and, per entry, does
//     v   = dot2(x|y, C|S) + K        one v_dot2_i32_i16
//     adr = (v >> 12) & ~3            the r cell's LDS byte address
//     ds_add_u32 [adr], 1
// where K folds in the rounding bias 2^13 and the row's LDS base, so the
// vote costs three VALU instructions and one LDS atomic (no MFMA: there is
// no dense contraction here).  A row whose corner range leaves [0, n_r), or
// a slice that does not fit in LDS (possible only with an unusual table),
// is handled by an exact fallback that adds into global memory with
// range checks and counts dropped votes.
#include "lane_entry.h"

namespace lane {

__device__ __forceinline__ int dot2_i16(int a, int b, int c) {
    // d = a.lo*b.lo + a.hi*b.hi + c, signed 16-bit halves, 32-bit sum
    int d;
    asm("v_dot2_i32_i16 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// Workgroup state.  The accumulator array is declared per LDS-size variant
// (kVoteLdsWords: one workgroup per CU; kVoteLdsWordsHalf: two).
template <int LDSW>
struct VoteLds {
    int32_t acc[LDSW];
    int lo[kMaxT], win[kMaxT], base[kMaxT];
    int fast, item;
    int il, lo_min, span;  // layout (0 rows back to back, 1 interleaved, 2 interleaved pairs),
                           // lowest r_idx of the slice, its r span
    uint32_t dropped;
};

template <int LDSW>
__device__ __forceinline__ void lds_vote(VoteLds<LDSW>& L, uint32_t v) {
    const uint32_t adr = (v >> 12) & 0x3FFFCu;  // 4 * floor(v / 2^14)
    __hip_atomic_fetch_add(reinterpret_cast<int32_t*>(
                               __builtin_assume_aligned(reinterpret_cast<char*>(L.acc) + adr, 4)),
                           1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Interleaved layout: cell u = r_idx - lo_min of row j sits in word u*T + j,
// so within one pixel's T lanes (T rows) the banks differ (j + T u mod 32
// with j < T); with back-to-back rows the banks of a wave's 64 votes are
// effectively random.  The word's byte address is ((v >> 14) << (2 +
// log2 T)) | 4j with v the biased dot product (floor(v / 2^14) = u): the
// same three instructions per vote as the back-to-back layout.  It needs
// T x (the slice's r span) words, used whenever that fits.
template <int LDSW>
__device__ __forceinline__ void lds_vote_il(VoteLds<LDSW>& L, uint32_t v, uint32_t jb, int sh) {
    const uint32_t adr = ((v >> 14) << sh) | jb;
    __hip_atomic_fetch_add(reinterpret_cast<int32_t*>(
                               __builtin_assume_aligned(reinterpret_cast<char*>(L.acc) + adr, 4)),
                           1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Interleaved pairs: cells u = 2m and 2m + 1 of row j share word m*T + j;
// a vote adds 1 to the word's low 14 bits and, for odd u, also 1 << 14, so
// the low field counts both cells and the high field the odd one (even =
// low - high).  Half the words of the interleaved layout for one more
// instruction ((v & 2^14) | 1 is one v_and_or); with T = 32 rows every lane
// of a pixel owns bank j and the wave's two pixels meet at most pairwise,
// the fewest bank cycles a 64-lane atomic can take.  Exact while no cell
// pair collects more than 2^14 - 1 votes: a slice takes this layout only
// when every row's table entries bound its pairs below that
// (vote_pair_bound), which holds for rotation tables on the frames the
// paired slice sizes are planned for and fails for tables with small entries.
template <int LDSW>
__device__ __forceinline__ void lds_vote_il2(VoteLds<LDSW>& L, uint32_t v, uint32_t jb, int sh) {
    const uint32_t adr = ((v >> 15) << sh) | jb;
    const uint32_t inc = (v & 0x4000u) | 1u;
    __hip_atomic_fetch_add(reinterpret_cast<uint32_t*>(
                               __builtin_assume_aligned(reinterpret_cast<char*>(L.acc) + adr, 4)),
                           inc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int M>
struct Mode {
    static constexpr int value = M;
};

// slots of one wave that share a segment when the slice has few rows
constexpr int kSlotsPerSegment = 8;

template <int LDSW>
__device__ void vote_item(VoteLds<LDSW>& sm, const VoteDesc& d, int code) {
    // code = slice * E + part: with an edge split, E workgroups share a
    // slice, each voting a contiguous 1/E share of the segments into its own
    // LDS rows and adding them into the accumulator, which the caller clears
    // before the launch (global atomic adds: no partial buffers, no arrival
    // protocol, no device-scope fences)
    const int E = d.E > 1 ? d.E : 1;
    const int slice = code / E, part = code - slice * E;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid >> 6;
    const int nwaves = blockDim.x >> 6;
    const int own_from = slice * d.T;  // rows below this belong to the previous slice
    // where the slice height d.T does not divide the angle count, the last
    // slice takes only the rows it owns, rounded up to a power of two (360
    // angles in slices of 16: the last votes 8 rows, not 16)
    int lg = d.log2T;
    while (lg > 0 && (1 << (lg - 1)) >= d.n_theta - own_from) --lg;
    const int T = 1 << lg;
    const int j = lane & (T - 1);
    const int g = lane >> lg;
    const int G = kWave >> lg;
    const int k0 = min(own_from, d.n_theta - T);
    const ListLayout L = list_layout(d.W, d.H);
    const uint32_t* __restrict__ list = d.list;

    // Set-up, one barrier: every thread clears the LDS counters (the
    // previous item's rows were read out before the caller's barrier) and
    // loads its own row's table entries, while wave 0 finds the slice's
    // layout: each lane q < T the r window its row can reach (the four
    // corners, where the monotone r is extreme), then a prefix sum of the
    // windows and the slice's extent across the lanes.
    for (int c = tid; c < LDSW; c += blockDim.x) sm.acc[c] = 0;
    const int kk = k0 + j;
    const int C = gld(d.cos_q14 + kk), S = gld(d.sin_q14 + kk);
    if (wave == 0) {
        int lo = 0x7FFFFFFF, hi = -1, win = 0;
        bool fast_ok = true, pair_ok = true;
        if (lane < T) {
            const int xs[4] = {0, d.W - 1, 0, d.W - 1};
            const int ys[4] = {0, 0, d.H - 1, d.H - 1};
            int rmin = 0x7FFFFFFF, rmax = -0x7FFFFFFF;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int r = (xs[c] * C + ys[c] * S + 8192) >> 14;  // arithmetic shift = floor
                rmin = min(rmin, r);
                rmax = max(rmax, r);
            }
            lo = rmin + d.r_offset;
            hi = rmax + d.r_offset;
            win = hi - lo + 1;
            fast_ok = lo >= 0 && hi < d.n_r;
            pair_ok = vote_pair_bound(d.W, d.H, C, S) <= kPairCountMax;
        }
        int incl = win;  // inclusive prefix sum of the windows over lanes < T
        for (int o = 1; o < T; o <<= 1) {
            const int t = __shfl_up(incl, o);
            if (lane >= o) incl += t;
        }
        int lo_min = lo, hi_max = hi;
        for (int o = 32; o > 0; o >>= 1) {
            lo_min = min(lo_min, __shfl_xor(lo_min, o));
            hi_max = max(hi_max, __shfl_xor(hi_max, o));
        }
        const bool all_fast = __ballot(!fast_ok) == 0;
        const bool all_pair = __ballot(!pair_ok) == 0;
        const int b2b_words = __shfl(incl, T - 1);
        if (lane < T) {
            sm.lo[lane] = lo;
            sm.win[lane] = win;
            sm.base[lane] = incl - win;
        }
        if (lane == 0) {
            // layout: pairs when 32 or more rows make them conflict-free, else
            // interleaved, else pairs to fit, else rows back to back.  The
            // slice's lowest cell is taken even, so that a pair never
            // straddles a key block (blocks start at multiples of 64)
            lo_min &= ~1;
            const int span = hi_max - lo_min + 1;
            auto fits = [&](int w) { return w <= LDSW; };
            const int il_words = span * T, il2_words = ((span + 1) >> 1) * T;
            // paired counters only where no row's cell pair can reach 2^14 votes
            const bool il2_ok = all_pair && fits(il2_words);
            const int mode = (T >= 32 && il2_ok) ? 2 : fits(il_words) ? 1 : il2_ok ? 2 : 0;
            sm.il = mode;
            sm.lo_min = lo_min;
            sm.span = span;
            sm.fast = all_fast && (mode != 0 || fits(b2b_words)) ? 1 : 0;
            sm.dropped = 0;
        }
    }
    __syncthreads();
    const bool fast = sm.fast != 0;
    const int layout = sm.il;
    const bool il = layout != 0;
    // the exact fallback runs unsplit, in part 0 (the same decision in every part)
    if (!fast && part != 0) return;
    const int seg_lo = fast ? (int)(((long long)L.nseg * part) / E) : 0;
    const int seg_hi = fast ? (int)(((long long)L.nseg * (part + 1)) / E) : L.nseg;
    // pruned: the list holds, per segment, the entries of tiles that vote
    // every row (streamed like an unmasked list) and, at the end of the
    // segment's slot, those of band-restricted tiles, tested entry by entry
    const bool pruned = d.pruned != 0;
    const bool masked = d.tile_mask != nullptr && !pruned;
    const int bb = (masked || pruned) ? band_bits_dev(d.n_theta, kk) : 0xFF;
    int slice_bits = 0;
    if (masked) {
        for (int q = 0; q < T; ++q) slice_bits |= band_bits_dev(d.n_theta, k0 + q);
    }

    if (fast) {
        const int lo = sm.lo[j], base = sm.base[j];
        const int K = il ? 8192 + (d.r_offset - sm.lo_min) * 16384
                         : 8192 + (base - lo + d.r_offset) * 16384;
        const int CS = (int)(((uint32_t)(uint16_t)S << 16) | (uint32_t)(uint16_t)C);
        const uint32_t jb = 4u * (uint32_t)j;
        const int sh = 2 + lg;
        auto body = [&](auto mode) {
        constexpr int kIL = decltype(mode)::value;
        auto vote1 = [&](uint32_t xy) {
            const uint32_t v = (uint32_t)dot2_i16((int)xy, CS, K);
            if constexpr (kIL == 2) lds_vote_il2(sm, v, jb, sh);
            else if constexpr (kIL == 1) lds_vote_il(sm, v, jb, sh);
            else lds_vote(sm, v);
        };
        auto voteV = [&](uint32_t v) {
            if constexpr (kIL == 2) lds_vote_il2(sm, v, jb, sh);
            else if constexpr (kIL == 1) lds_vote_il(sm, v, jb, sh);
            else lds_vote(sm, v);
        };
        // four entries: the four dot products first, so no address waits on
        // the product just issued
        auto vote4 = [&](u32x4 q) {
            const uint32_t v0 = (uint32_t)dot2_i16((int)q.x, CS, K);
            const uint32_t v1 = (uint32_t)dot2_i16((int)q.y, CS, K);
            const uint32_t v2 = (uint32_t)dot2_i16((int)q.z, CS, K);
            const uint32_t v3 = (uint32_t)dot2_i16((int)q.w, CS, K);
            voteV(v0);
            voteV(v1);
            voteV(v2);
            voteV(v3);
        };
        if (!masked) {
            // One segment's entries split over Gs slots (slot gs): each slot
            // takes its own part of the segment (a different stretch of
            // columns), so slots voting for the same theta rarely hit the
            // same r cell at once.
            auto run_segment = [&](const uint32_t* __restrict__ ents, int n, int Gs, int gs) {
                const int part = (n / (4 * Gs)) * 4;  // entries per slot, multiple of 4
                const int nfull = part / 4;
                const uint32_t* p = ents + gs * part;
                // software pipeline: U 128-bit loads per lane stay in flight
                // while the previous U are voted; two register sets take
                // turns, so no copies between them
                constexpr int U = 4;
                int it = 0;
                if (nfull >= U) {
                    u32x4 a[U], b[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) a[u] = gld4(p + 4 * u);
                    // (the scheduling barriers keep the compiler from hoisting
                    // the other set's first votes above its wait)
                    for (it = U; it + 2 * U <= nfull; it += 2 * U) {
#pragma unroll
                        for (int u = 0; u < U; ++u) b[u] = gld4(p + 4 * (it + u));
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int u = 0; u < U; ++u) vote4(a[u]);
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int u = 0; u < U; ++u) a[u] = gld4(p + 4 * (it + U + u));
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int u = 0; u < U; ++u) vote4(b[u]);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    // a holds entries [it - U, it); fewer than 2U groups remain
                    if (it + U <= nfull) {
#pragma unroll
                        for (int u = 0; u < U; ++u) b[u] = gld4(p + 4 * (it + u));
#pragma unroll
                        for (int u = 0; u < U; ++u) vote4(a[u]);
#pragma unroll
                        for (int u = 0; u < U; ++u) vote4(b[u]);
                        it += U;
                    } else {
#pragma unroll
                        for (int u = 0; u < U; ++u) vote4(a[u]);
                    }
                }
                for (; it < nfull; ++it) vote4(gld4(p + 4 * it));
                // remainder (fewer than 4 Gs entries), shared by all slots
                const int i0 = Gs * part + 4 * gs;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (i0 + q < n) vote1(gld(ents + i0 + q));
                }
            };
            if (G <= kSlotsPerSegment) {
                // the entry counts of the wave's next 64 segments in one load,
                // so a segment never waits for its count
                for (int seg0 = seg_lo + wave; seg0 < seg_hi; seg0 += nwaves * kWave) {
                    const int sj = seg0 + lane * nwaves;
                    const int cnt = sj < seg_hi ? min((int)gld(list + sj), kSegCap) : 0;
                    const int nk = min(kWave, (seg_hi - seg0 + nwaves - 1) / nwaves);
                    for (int k = 0; k < nk; ++k) {
                        const int seg = seg0 + k * nwaves;
                        run_segment(list + L.off_ent + (size_t)seg * kSegCap,
                                    __builtin_amdgcn_readlane(cnt, k), G, g);
                    }
                }
            } else {
                // few theta rows, many slots: a wave works on G / 8 segments at
                // once, 8 slots each, so every slot has a long run of loads to
                // pipeline instead of a few per segment
                const int P = G / kSlotsPerSegment;
                const int sub = g / kSlotsPerSegment, gs = g - sub * kSlotsPerSegment;
                for (int seg0 = seg_lo + wave * P; seg0 < seg_hi; seg0 += nwaves * P) {
                    const int seg = seg0 + sub;
                    const int n = seg < seg_hi ? min((int)gld(list + seg), kSegCap) : 0;
                    run_segment(list + L.off_ent + (size_t)min(seg, seg_hi - 1) * kSegCap, n,
                                kSlotsPerSegment, gs);
                }
            }
        } else {
            // Masked vote.  A segment's 128 tiles are scanned at once (tiles
            // l and l + 64 per lane); tiles with edges whose band bits meet
            // this slice's angles form runs of equal mask byte, and a run's
            // entries are contiguous in the segment, so each run is voted
            // like the unmasked stream, with the lane predicate "this lane's
            // angle lies in a band of the run's mask".
            for (int seg = seg_lo + wave; seg < seg_hi; seg += nwaves) {
                const int ty = seg / L.nchunk, chunk = seg - ty * L.nchunk;
                const int n = min((int)gld(list + seg), kSegCap);
                if (n == 0) continue;
                const uint32_t* __restrict__ ents = list + L.off_ent + (size_t)seg * kSegCap;
                const int tx0 = chunk * kTilesPerChunk;
                const int ntx = min(L.tw - tx0, kTilesPerChunk);
                const uint32_t* info = list + L.off_info + (size_t)ty * L.tw + tx0;
                const uint8_t* mrow = d.tile_mask + (size_t)ty * L.tw + tx0;
                uint32_t inf[2];
                int mk[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {  // clamped, so the four loads go out together
                    const int t = min(h * kWave + lane, ntx - 1);
                    inf[h] = gld(info + t);
                    mk[h] = (int)gld(mrow + t);
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (h * kWave + lane >= ntx) {
                        inf[h] = 0u;
                        mk[h] = 0;
                    }
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const bool rel = (inf[h] >> 16) != 0 && (mk[h] & slice_bits) != 0;
                    const int mprev = __shfl_up(mk[h], 1);
                    const uint32_t iprev = (uint32_t)__shfl_up((int)inf[h], 1);
                    const bool relprev = lane > 0 && (iprev >> 16) != 0 && (mprev & slice_bits) != 0;
                    const bool brk = rel && (!relprev || mprev != mk[h]);
                    const uint64_t relm = __ballot(rel);
                    uint64_t brkm = __ballot(brk);
                    while (brkm) {
                        const int a = __builtin_ctzll(brkm);
                        brkm &= brkm - 1;
                        const uint64_t stop = (~relm | brkm) & ~((2ull << a) - 1ull);
                        const int b = stop ? __builtin_ctzll(stop) : kWave;
                        const uint32_t ia = (uint32_t)__builtin_amdgcn_readlane((int)inf[h], a);
                        const uint32_t iz = (uint32_t)__builtin_amdgcn_readlane((int)inf[h], b - 1);
                        const int mr = __builtin_amdgcn_readlane(mk[h], a);
                        const int start = (int)(ia & 0xFFFFu);
                        const int end = min((int)(iz & 0xFFFFu) + (int)(iz >> 16), n);
                        if ((mr & bb) == 0 || start >= end) continue;
                        // full quads [qa, qz), then up to 3 loose entries at
                        // each end
                        const int qa = (start + 3) >> 2, qz = end >> 2;
                        int q = qa + g;
                        if (q < qz) {
                            u32x4 cur = gld4(ents + 4 * q);
                            for (q += G; q < qz; q += G) {
                                const u32x4 nxt = gld4(ents + 4 * q);
                                vote4(cur);
                                cur = nxt;
                            }
                            vote4(cur);
                        }
                        const int h1 = min(4 * qa, end);
                        const int nh = h1 - start;
                        const int t0 = max(4 * qz, 4 * qa);
                        const int nl = nh + max(0, end - t0);
                        for (int t = g; t < nl; t += G) {
                            const int e = t < nh ? start + t : t0 + (t - nh);
                            vote1(gld(ents + e));
                        }
                    }
                }
            }
        }
        if (pruned) {
            // band-restricted entries of this wave's segments: the counts of
            // 64 segments at once, then each segment that has any, its
            // entries spread over the slots, each voting in this lane's row
            // if its tile's mask meets the row's bands
            for (int s0 = seg_lo + wave; s0 < seg_hi; s0 += nwaves * kWave) {
                const int sj = s0 + lane * nwaves;
                const int R = sj < seg_hi ? min((int)gld(list + L.off_info + sj), kSegCap) : 0;
                unsigned long long mk = __ballot(R > 0);
                while (mk) {
                    const int l = __builtin_ctzll(mk);
                    mk &= mk - 1ull;
                    const int seg = s0 + l * nwaves;
                    const int Rs = __builtin_amdgcn_readlane(R, l);
                    const uint32_t* __restrict__ ents = list + L.off_ent + (size_t)seg * kSegCap + (kSegCap - Rs);
                    for (int e = g; e < Rs; e += G) {
                        const uint32_t xy = gld(ents + e);
                        const int x = (int)(xy & 0xFFFFu), y = (int)(xy >> 16);
                        if (x >= d.W || y >= d.H) continue;
                        if (gld(d.tile_mask + (size_t)(y >> 3) * L.tw + (x >> 3)) & bb) vote1(xy);
                    }
                }
            }
        }
        };
        if (layout == 2) body(Mode<2>{});
        else if (layout == 1) body(Mode<1>{});
        else body(Mode<0>{});
        __syncthreads();
        const int q0 = own_from - k0;  // first owned row of the slice
        const int lo_min = sm.lo_min, span = sm.span;
        auto cell = [&](int q, int rlo, int rwin, int rbase, int i) -> int {
            if (layout == 1) {
                const int u = i - lo_min;
                return (u >= 0 && u < span) ? sm.acc[u * T + q] : 0;
            }
            if (layout == 2) {
                const int u = i - lo_min;
                if (u < 0 || u >= span) return 0;
                const uint32_t w = (uint32_t)sm.acc[(u >> 1) * T + q];
                const uint32_t odd = w >> 14;
                return (int)((u & 1) ? odd : (w & 0x3FFFu) - odd);
            }
            const int o = i - rlo;
            return (o >= 0 && o < rwin) ? sm.acc[rbase + o] : 0;
        };
        if (E > 1) {
            // this part's share of the owned rows, over each row's window
            // (cells outside it are zero); the peak keys come from a later pass
            for (int q = q0; q < T; ++q) {
                const int row = k0 + q;
                const int rlo = sm.lo[q], rwin = sm.win[q], rbase = sm.base[q];
                int32_t* out = d.acc + (size_t)row * d.n_r;
                for (int o = tid; o < rwin; o += blockDim.x) {
                    const int v = cell(q, rlo, rwin, rbase, rlo + o);
                    if (v != 0) atomicAdd(out + rlo + o, v);
                }
            }
        } else if (layout != 0 && T >= 4) {
            // Write the owned rows and, block by block, the peak-search keys,
            // four rows at a time: lane (r, c) = (lane / 16, lane % 16) takes
            // LDS words c, c + 16, ... of row 4 grp + r within the block, so
            // a read touches 16 words of each of 4 rows (at most 4 to a bank,
            // where 64 cells of one row would put 8 or more there) and the
            // stores of a row cover 128 contiguous bytes.  Each lane keeps
            // the first largest of its cells; the 16 lanes of a row, one DPP
            // row, merge them once per block.
            const int cpw = layout == 2 ? 2 : 1;                   // cells per LDS word
            const int npw = layout == 2 ? (span + 1) >> 1 : span;  // LDS words per row
            const int B = d.keys ? 1 << d.key_log2 : 256;
            const int nbr = d.keys ? d.nbr : (d.n_r + 255) >> 8;
            const int r = lane >> 4, c = lane & 15;
            const int g_lo = q0 >> 2;  // first group with an owned row
            const int ntask = ((T >> 2) - g_lo) * nbr;
            for (int task = wave; task < ntask; task += nwaves) {
                const int grp = g_lo + task / nbr, jb = task % nbr;
                const int q = 4 * grp + r;
                const bool own = q >= q0;
                const int row = k0 + q;
                int32_t* out = d.acc + (size_t)row * d.n_r;
                const uint32_t rowc = (uint32_t)row * (uint32_t)d.n_r;
                const int b0 = jb * B, b1 = min(d.n_r, b0 + B);
                const int w0 = (b0 - lo_min) / cpw;  // exact: both even when paired
                const int nw = (b1 - b0 + cpw - 1) / cpw;
                int bv = -1, bi = 0;
                for (int w = c; w < nw; w += 16) {
                    const int m = w0 + w;
                    const uint32_t x = (m >= 0 && m < npw) ? (uint32_t)sm.acc[m * T + q] : 0u;
                    const int i = b0 + w * cpw;
                    if (layout == 2) {
                        const int odd = (int)(x >> 14), even = (int)(x & 0x3FFFu) - odd;
                        if (own) gst(out + i, even);
                        if (even > bv) {
                            bv = even;
                            bi = i;
                        }
                        if (i + 1 < b1) {
                            if (own) gst(out + i + 1, odd);
                            if (odd > bv) {
                                bv = odd;
                                bi = i + 1;
                            }
                        }
                    } else {
                        if (own) gst(out + i, (int)x);
                        if ((int)x > bv) {
                            bv = (int)x;
                            bi = i;
                        }
                    }
                }
                if (d.keys) {
                    unsigned long long key = bv >= 0 ? make_key(bv, rowc + (uint32_t)bi) : 0ull;
                    key = row_max_u64(key);
                    if (own && c == 0) gst(d.keys + (size_t)row * d.nbr + jb, key);
                }
            }
        } else if (d.keys) {
            // write the rows and, block by block, the peak-search keys
            const int B = 1 << d.key_log2;
            const int ntask = (T - q0) * d.nbr;
            for (int task = wave; task < ntask; task += nwaves) {
                const int q = q0 + task / d.nbr, jb = task % d.nbr;
                const int row = k0 + q;
                const int rlo = sm.lo[q], rwin = sm.win[q], rbase = sm.base[q];
                int32_t* out = d.acc + (size_t)row * d.n_r;
                const uint32_t rowc = (uint32_t)row * (uint32_t)d.n_r;
                const int i0 = jb * B, i1 = min(d.n_r, i0 + B);
                unsigned long long best = 0;
                for (int i = i0 + lane; i < i1; i += kWave) {
                    const int v = cell(q, rlo, rwin, rbase, i);
                    gst(out + i, v);
                    const unsigned long long kk = make_key(v, rowc + (uint32_t)i);
                    best = kk > best ? kk : best;
                }
                best = wave_max_u64(best);
                if (lane == 0) gst(d.keys + (size_t)row * d.nbr + jb, best);
            }
        } else {
            for (int q = q0; q < T; ++q) {
                const int row = k0 + q;
                const int rlo = sm.lo[q], rwin = sm.win[q], rbase = sm.base[q];
                int32_t* out = d.acc + (size_t)row * d.n_r;
                for (int i = tid; i < d.n_r; i += blockDim.x) gst(out + i, cell(q, rlo, rwin, rbase, i));
            }
        }
    } else {
        // exact fallback: zero the owned rows, then add into global memory
        for (int q = 0; q < T; ++q) {
            const int row = k0 + q;
            if (row < own_from) continue;
            int32_t* out = d.acc + (size_t)row * d.n_r;
            for (int i = tid; i < d.n_r; i += blockDim.x) out[i] = 0;
        }
        __threadfence();
        __syncthreads();
        const bool own = kk >= own_from;
        int32_t* out = d.acc + (size_t)kk * d.n_r;
        uint32_t drop = 0;
        for (int seg = wave; seg < L.nseg; seg += nwaves) {
            const int n = min((int)list[seg], kSegCap);
            // a pruned list's band-restricted entries follow, from the slot's end
            const int R = pruned ? min((int)list[L.off_info + seg], kSegCap - n) : 0;
            const uint32_t* ents = list + L.off_ent + (size_t)seg * kSegCap;
            for (int e = g; e < n + R; e += G) {
                const bool res = e >= n;
                const uint32_t xy = ents[res ? kSegCap - R + (e - n) : e];
                const int x = (int)(xy & 0xFFFFu), y = (int)(xy >> 16);
                if (!own || x >= d.W || y >= d.H) continue;
                if (masked || res) {
                    const int m = d.tile_mask[(size_t)(y >> 3) * L.tw + (x >> 3)];
                    if ((m & bb) == 0) continue;
                }
                const int r = (x * C + y * S + 8192) >> 14;
                const int i = r + d.r_offset;
                if (i >= 0 && i < d.n_r) atomicAdd(out + i, 1);
                else ++drop;
            }
        }
        if (drop) atomicAdd(&sm.dropped, drop);
        __threadfence();
        __syncthreads();
        if (tid == 0 && d.dropped && sm.dropped) atomicAdd(d.dropped, sm.dropped);
        if (d.keys) {
            // keys from the finished rows, read back at device scope
            const int B = 1 << d.key_log2;
            const int q0 = own_from - k0;
            const int ntask = (T - q0) * d.nbr;
            for (int task = wave; task < ntask; task += nwaves) {
                const int q = q0 + task / d.nbr, jb = task % d.nbr;
                const int row = k0 + q;
                int32_t* rowp = d.acc + (size_t)row * d.n_r;
                const uint32_t rowc = (uint32_t)row * (uint32_t)d.n_r;
                const int i0 = jb * B, i1 = min(d.n_r, i0 + B);
                unsigned long long best = 0;
                for (int i = i0 + lane; i < i1; i += kWave) {
                    const int v = __hip_atomic_load(rowp + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const unsigned long long kk = make_key(v, rowc + (uint32_t)i);
                    best = kk > best ? kk : best;
                }
                best = wave_max_u64(best);
                if (lane == 0) gst(d.keys + (size_t)row * d.nbr + jb, best);
            }
        }
    }
}

__global__ void __launch_bounds__(kVoteThreads) k_vote(VoteDesc d) {
    __shared__ VoteLds<kVoteLdsWords> sm;
    vote_item(sm, d, blockIdx.x);
}

// Batched, persistent.  queue == null: static grid stride over the item
// table (the table is laid out so that a frame's slices land on one XCD and
// share its L2).  queue != null, xends == null: items are taken in table
// order from one atomic ticket (longest items first balances mixed sizes).
// queue and xends != null: the table holds one run of items per XCD (the
// frames given to that XCD, each frame's slices together), xends[x] the end
// of run x; a workgroup takes tickets from its own XCD's run (workgroups
// are dispatched to the XCDs in turn), so the slices running at once on an
// XCD share the frames whose lists its L2 holds, and when that run is used
// up it takes from the others in turn.
template <int LDSW>
__global__ void __launch_bounds__(kVoteThreads)
    __attribute__((amdgpu_waves_per_eu(LDSW == kVoteLdsWordsHalf ? 8 : 4)))
    k_vote_batch(const VoteDesc* __restrict__ descs, const int2* __restrict__ items,
                 const int* __restrict__ n_items_ptr, uint32_t* queue, const int* __restrict__ xends) {
    const int n_items = gld(n_items_ptr);  // in device memory: any selection of frames
    __shared__ VoteLds<LDSW> sm;
    int it = blockIdx.x;
    int k = 0;  // XCD runs this workgroup has found used up (own first)
    const int home = (int)(blockIdx.x & 7u);
    for (;;) {
        if (queue) {
            if (threadIdx.x == 0) {
                int item = n_items;
                if (xends) {
                    for (; k < 8; ++k) {
                        const int x = (home + k) & 7;
                        const int lo = x ? gld(xends + x - 1) : 0, hi = gld(xends + x);
                        if (lo >= hi) continue;
                        const int t = (int)atomicAdd(queue + x, 1u);
                        if (lo + t < hi) {
                            item = lo + t;
                            break;
                        }
                    }
                } else {
                    item = (int)atomicAdd(queue, 1u);
                }
                sm.item = item;
            }
            __syncthreads();
            it = __builtin_amdgcn_readfirstlane(sm.item);
        }
        if (it >= n_items) break;
        const int2 w = items[it];
        if (w.x >= 0) {
            const VoteDesc d = descs[w.x];
            if (frame_on(d.active)) vote_item(sm, d, w.y);
        }
        __syncthreads();
        if (!queue) it += gridDim.x;
    }
}

}  // namespace lane

using namespace lane;

extern "C" LANE_INTERNAL hipError_t lane_launch_vote(const VoteDesc* dp, hipStream_t s) {
    hipLaunchKernelGGL(k_vote, dim3(dp->n_slices), dim3(kVoteThreads), 0, s, *dp);
    return hipGetLastError();
}

extern "C" LANE_INTERNAL hipError_t lane_launch_vote_batch(const VoteDesc* descs, const int2* items,
                                                           const int* n_items, uint32_t* queue,
                                                           const int* xends, int half_lds, int grid,
                                                           hipStream_t s) {
    if (half_lds)
        hipLaunchKernelGGL(k_vote_batch<kVoteLdsWordsHalf>, dim3(grid), dim3(kVoteThreads), 0, s,
                           descs, items, n_items, queue, xends);
    else
        hipLaunchKernelGGL(k_vote_batch<kVoteLdsWords>, dim3(grid), dim3(kVoteThreads), 0, s, descs,
                           items, n_items, queue, xends);
    return hipGetLastError();
}
