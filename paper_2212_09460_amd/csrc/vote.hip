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
#include "lane_internal.h"

namespace lane {

__device__ __forceinline__ int dot2_i16(int a, int b, int c) {
    // d = a.lo*b.lo + a.hi*b.hi + c, signed 16-bit halves, 32-bit sum
    int d;
    asm("v_dot2_i32_i16 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

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

__shared__ int32_t s_acc[kVoteLdsWords];
__shared__ int s_lo[kMaxT], s_win[kMaxT], s_base[kMaxT];
__shared__ int s_fast, s_total;
__shared__ uint32_t s_dropped;

__device__ __forceinline__ void lds_vote(uint32_t v) {
    const uint32_t adr = (v >> 12) & 0x3FFFCu;
    __hip_atomic_fetch_add(reinterpret_cast<int32_t*>(
                               __builtin_assume_aligned(reinterpret_cast<char*>(s_acc) + adr, 4)),
                           1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ void vote_item(const VoteDesc& d, int slice) {
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid >> 6;
    const int nwaves = blockDim.x >> 6;
    const int T = d.T;
    const int j = lane & (T - 1);
    const int g = lane >> d.log2T;
    const int G = kWave >> d.log2T;
    const int k0 = min(slice * T, d.n_theta - T);
    const int own_from = slice * T;  // rows below this belong to the previous slice
    const ListLayout L = list_layout(d.W, d.H);
    const uint32_t* __restrict__ list = d.list;

    if (tid == 0) {
        s_fast = 1;
        s_dropped = 0;
    }
    __syncthreads();
    if (tid < T) {
        const int k = k0 + tid;
        const int C = gld(d.cos_q14 + k), S = gld(d.sin_q14 + k);
        const int xs[4] = {0, d.W - 1, 0, d.W - 1};
        const int ys[4] = {0, 0, d.H - 1, d.H - 1};
        int rmin = 0x7FFFFFFF, rmax = -0x7FFFFFFF;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int r = (xs[c] * C + ys[c] * S + 8192) >> 14;  // arithmetic shift = floor
            rmin = min(rmin, r);
            rmax = max(rmax, r);
        }
        const int lo = rmin + d.r_offset, hi = rmax + d.r_offset;
        s_lo[tid] = lo;
        s_win[tid] = hi - lo + 1;
        if (lo < 0 || hi >= d.n_r) s_fast = 0;
    }
    __syncthreads();
    if (tid == 0) {
        int base = 0;
        for (int q = 0; q < T; ++q) {
            s_base[q] = base;
            base += s_win[q];
        }
        s_total = base;
        if (base > kVoteLdsWords) s_fast = 0;
    }
    __syncthreads();
    const bool fast = s_fast != 0;
    const int kk = k0 + j;
    const int C = gld(d.cos_q14 + kk), S = gld(d.sin_q14 + kk);
    const bool masked = d.tile_mask != nullptr;
    const int bb = masked ? band_bits_dev(d.n_theta, kk) : 0xFF;
    int slice_bits = 0;
    if (masked) {
        for (int q = 0; q < T; ++q) slice_bits |= band_bits_dev(d.n_theta, k0 + q);
    }

    if (fast) {
        const int total = s_total;
        for (int c = tid; c < total; c += blockDim.x) s_acc[c] = 0;
        const int lo = s_lo[j], base = s_base[j];
        const int K = 8192 + (base - lo + d.r_offset) * 16384;
        const int CS = (int)(((uint32_t)(uint16_t)S << 16) | (uint32_t)(uint16_t)C);
        __syncthreads();
        if (!masked) {
            auto vote4 = [&](u32x4 q) {
                lds_vote((uint32_t)dot2_i16((int)q.x, CS, K));
                lds_vote((uint32_t)dot2_i16((int)q.y, CS, K));
                lds_vote((uint32_t)dot2_i16((int)q.z, CS, K));
                lds_vote((uint32_t)dot2_i16((int)q.w, CS, K));
            };
            for (int seg = wave; seg < L.nseg; seg += nwaves) {
                const int n = min((int)gld(list + seg), kSegCap);
                const uint32_t* __restrict__ ents = list + L.off_ent + (size_t)seg * kSegCap;
                const int step = 4 * G;        // entries one wave-iteration covers
                const int nfull = n / step;
                const uint32_t* p = ents + 4 * g;
                // software pipeline: U 128-bit loads per lane stay in flight
                // while the previous U are voted
                constexpr int U = 4;
                int it = 0;
                if (nfull >= U) {
                    u32x4 cur[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) cur[u] = gld4(p + u * step);
                    for (it = U; it + U <= nfull; it += U) {
                        u32x4 nxt[U];
#pragma unroll
                        for (int u = 0; u < U; ++u) nxt[u] = gld4(p + (it + u) * step);
#pragma unroll
                        for (int u = 0; u < U; ++u) vote4(cur[u]);
#pragma unroll
                        for (int u = 0; u < U; ++u) cur[u] = nxt[u];
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) vote4(cur[u]);
                }
                for (; it < nfull; ++it) vote4(gld4(p + it * step));
                const int i0 = nfull * step + 4 * g;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (i0 + q < n) lds_vote((uint32_t)dot2_i16((int)gld(ents + i0 + q), CS, K));
                }
            }
        } else {
            for (int seg = wave; seg < L.nseg; seg += nwaves) {
                const int ty = seg / L.nchunk, chunk = seg - ty * L.nchunk;
                const uint32_t* __restrict__ ents = list + L.off_ent + (size_t)seg * kSegCap;
                const int tx0 = chunk * kTilesPerChunk;
                const int tx1 = min(L.tw, tx0 + kTilesPerChunk);
                const uint32_t* info = list + L.off_info + (size_t)ty * L.tw;
                const uint8_t* mrow = d.tile_mask + (size_t)ty * L.tw;
                for (int tx = tx0; tx < tx1; ++tx) {
                    const uint32_t inf = gld(info + tx);
                    const int cnt = min((int)(inf >> 16), kTile * kTile);
                    if (cnt == 0 || (int)(inf & 0xFFFFu) > kSegCap - cnt) continue;
                    const int m = gld(mrow + tx);
                    if ((m & slice_bits) == 0) continue;
                    if ((m & bb) == 0) continue;  // this lane's angle is pruned in this tile
                    const uint32_t* te = ents + (inf & 0xFFFFu);
                    for (int e = g; e < cnt; e += G) lds_vote((uint32_t)dot2_i16((int)gld(te + e), CS, K));
                }
            }
        }
        __syncthreads();
        for (int q = 0; q < T; ++q) {
            const int row = k0 + q;
            if (row < own_from) continue;
            const int rlo = s_lo[q], rwin = s_win[q], rbase = s_base[q];
            int32_t* out = d.acc + (size_t)row * d.n_r;
            for (int i = tid; i < d.n_r; i += blockDim.x) {
                const int o = i - rlo;
                gst(out + i, (o >= 0 && o < rwin) ? s_acc[rbase + o] : 0);
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
            const uint32_t* ents = list + L.off_ent + (size_t)seg * kSegCap;
            for (int e = g; e < n; e += G) {
                const uint32_t xy = ents[e];
                const int x = (int)(xy & 0xFFFFu), y = (int)(xy >> 16);
                if (!own || x >= d.W || y >= d.H) continue;
                if (masked) {
                    const int m = d.tile_mask[(size_t)(y >> 3) * L.tw + (x >> 3)];
                    if ((m & bb) == 0) continue;
                }
                const int r = (x * C + y * S + 8192) >> 14;
                const int i = r + d.r_offset;
                if (i >= 0 && i < d.n_r) atomicAdd(out + i, 1);
                else ++drop;
            }
        }
        if (drop) atomicAdd(&s_dropped, drop);
        __syncthreads();
        if (tid == 0 && d.dropped && s_dropped) atomicAdd(d.dropped, s_dropped);
    }
}

__global__ void __launch_bounds__(kVoteThreads) k_vote(VoteDesc d) { vote_item(d, blockIdx.x); }

__shared__ int s_item;

// Batched, persistent.  queue == null: static grid stride over the item
// table (the table is laid out so that a frame's slices land on one XCD and
// share its L2).  queue != null: items are taken in table order from an
// atomic ticket (longest items first balances mixed sizes).
__global__ void __launch_bounds__(kVoteThreads)
    k_vote_batch(const VoteDesc* __restrict__ descs, const int2* __restrict__ items, int n_items,
                 uint32_t* queue) {
    int it = blockIdx.x;
    for (;;) {
        if (queue) {
            if (threadIdx.x == 0) s_item = (int)atomicAdd(queue, 1u);
            __syncthreads();
            it = s_item;
        }
        if (it >= n_items) break;
        const int2 w = items[it];
        if (w.x >= 0) {
            const VoteDesc d = descs[w.x];
            vote_item(d, w.y);
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

extern "C" LANE_INTERNAL hipError_t lane_launch_vote_batch(const VoteDesc* descs, const int2* items, int n_items,
                                             uint32_t* queue, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_vote_batch, dim3(grid), dim3(kVoteThreads), 0, s, descs, items, n_items,
                       queue);
    return hipGetLastError();
}
