// Hough vote with the angle pairing of the FPGA design (Sec. 3.3 Eq. (4)-(5)).
//
// What is computed: the accumulator of lane_hough_vote (Sec. 2.3 Eq. (3)),
// r_idx = floor((x*C[k] + y*S[k] + 2^13) / 2^14) + r_offset, votes outside
// [0, n_r) counted as dropped.  The pairing: theta_{n-k} = 180deg - theta_k,
// so with a symmetric table (C[n-k] = -C[k], S[n-k] = S[k]) both rows follow
// from the same two products u = x*C[k] and w = y*S[k]:
//     r_k = floor((w + u + 2^13) / 2^14),  r_{n-k} = floor((w - u + 2^13) / 2^14),
// which is what the FPGA's 180 processing elements share.  A pair whose
// table rows are not symmetric is voted row by row, so the result is exact
// for any table.
//
// Design.  One workgroup per row pair {k, n-k} (row 0 and, for even n, row
// n/2 stand alone), both rows in LDS over the r range the angle reaches in
// the frame (from the four corners, where the monotone r is extreme), the
// whole edge list streamed 16 segments at a time, each thread on its own part
// of a segment (so that the lanes of one LDS atomic come from pixels far
// apart) with eight 128-bit loads in flight.
// `pairing` selects the shared products (24-bit multiplies, then an add and
// a subtract) or one packed dot product per row, on the same kernel, so the
// two differ only in the arithmetic of a vote.  A pair whose rows do not fit
// in LDS (possible only with an unusual table on a large frame) adds into
// global memory instead.
#include "lane_entry.h"

namespace lane {

constexpr int kPairThreads = 1024;
constexpr int kPairLdsWords = 40704;  // 159 KB

__device__ __forceinline__ int pair_dot2(int a, int b, int c) {
    // a.lo*b.lo + a.hi*b.hi + c on signed 16-bit halves
    int d;
    asm("v_dot2_i32_i16 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

__device__ __forceinline__ long long r_of(long long x, long long y, int C, int S) {
    const long long v = x * C + y * S + 8192;
    return v >= 0 ? v / 16384 : -((-v + 16383) / 16384);  // floor
}

struct PairRow {
    int row, lo, span, base;  // r_idx range [lo, lo + span) at LDS word base
};

__global__ void __launch_bounds__(kPairThreads) k_vote_pair(VoteDesc d, int pairing) {
    __shared__ int32_t s_acc[kPairLdsWords];
    __shared__ PairRow s_row[2];
    __shared__ int s_mode;  // 0: LDS rows, 1: global fallback
    __shared__ uint32_t s_drop;
    const int tid = threadIdx.x;
    const int n = d.n_theta, g = blockIdx.x;
    const int a = g, b = (g == 0 || 2 * g == n) ? -1 : n - g;  // b = -1: row a alone
    const int Ca = gld(d.cos_q14 + a), Sa = gld(d.sin_q14 + a);
    const int Cb = b >= 0 ? gld(d.cos_q14 + b) : 0, Sb = b >= 0 ? gld(d.sin_q14 + b) : 0;
    const bool sym = pairing != 0 && b >= 0 && Cb == -Ca && Sb == Sa;
    if (tid == 0) {
        int base = 0;
        for (int q = 0; q < 2; ++q) {
            const int row = q == 0 ? a : b;
            PairRow pr{row, 0, 0, base};
            if (row >= 0) {
                const int C = q == 0 ? Ca : Cb, S = q == 0 ? Sa : Sb;
                long long lo = 0, hi = 0;
                for (int c = 0; c < 4; ++c) {
                    const long long r = r_of((c & 1) ? d.W - 1 : 0, (c & 2) ? d.H - 1 : 0, C, S);
                    lo = c == 0 || r < lo ? r : lo;
                    hi = c == 0 || r > hi ? r : hi;
                }
                pr.lo = (int)(lo + d.r_offset);
                pr.span = (int)(hi - lo + 1);
                base += pr.span;
            }
            s_row[q] = pr;
        }
        s_mode = base <= kPairLdsWords ? 0 : 1;
        s_drop = 0;
    }
    __syncthreads();
    const PairRow ra = s_row[0], rb = s_row[1];
    const int mode = s_mode;
    if (mode == 0) {
        for (int i = tid; i < ra.span + rb.span; i += kPairThreads) s_acc[i] = 0;
    } else {
        for (int i = tid; i < d.n_r; i += kPairThreads) {
            gst(d.acc + (size_t)a * d.n_r + i, 0);
            if (b >= 0) gst(d.acc + (size_t)b * d.n_r + i, 0);
        }
        __threadfence();  // the cleared rows are in place before any wave adds into them
    }
    __syncthreads();

    // LDS word of a vote = floor((value + K) / 2^14), K folding in the
    // rounding bias and the row's window (r_idx - lo + base)
    const int Ka = 8192 + (d.r_offset - ra.lo + ra.base) * 16384;
    const int Kb = 8192 + (d.r_offset - rb.lo + rb.base) * 16384;
    const int CSa = (int)(((uint32_t)(uint16_t)Sa << 16) | (uint32_t)(uint16_t)Ca);
    const int CSb = (int)(((uint32_t)(uint16_t)Sb << 16) | (uint32_t)(uint16_t)Cb);
    uint32_t drop = 0;
    auto vote_global = [&](int row, int C, int S, int x, int y) {
        const long long i = r_of(x, y, C, S) + d.r_offset;
        if (i >= 0 && i < d.n_r) atomicAdd(d.acc + (size_t)row * d.n_r + i, 1);
        else ++drop;
    };
    auto vote = [&](uint32_t xy) {
        if (mode == 0) {
            if (sym) {
                const int x = (int)(xy & 0xFFFFu), y = (int)(xy >> 16);
                const int u = __mul24(x, Ca);
                const int wa = __mul24(y, Sa) + Ka, wb = __mul24(y, Sa) + Kb;
                atomicAdd(s_acc + ((wa + u) >> 14), 1);
                atomicAdd(s_acc + ((wb - u) >> 14), 1);
            } else {
                atomicAdd(s_acc + (pair_dot2((int)xy, CSa, Ka) >> 14), 1);
                if (b >= 0) atomicAdd(s_acc + (pair_dot2((int)xy, CSb, Kb) >> 14), 1);
            }
        } else {
            const int x = (int)(xy & 0xFFFFu), y = (int)(xy >> 16);
            vote_global(a, Ca, Sa, x, y);
            if (b >= 0) vote_global(b, Cb, Sb, x, y);
        }
    };

    // 16 segments at a time, each cut into 64 parts: thread (g, p) votes
    // part p of segment g of the group, from its own phase, with two sets
    // of four 128-bit loads taking turns
    const ListLayout L = list_layout(d.W, d.H);
    const uint32_t* ents = d.list + L.off_ent;
    constexpr int kGroup = 16, kParts = kPairThreads / kGroup;
    const int gsel = tid % kGroup, part = tid / kGroup;
    for (int s0 = 0; s0 < L.nseg; s0 += kGroup) {
        const int sg = s0 + gsel;
        const int cnt = sg < L.nseg ? (int)gld(d.list + sg) : 0;
        const int nq = (cnt + 3) >> 2;
        const int pq = (nq + kParts - 1) / kParts;
        const int q0 = min(part * pq, nq), q1 = min(q0 + pq, nq);
        const int len = q1 - q0;
        const int phase = (gsel * len) / kGroup;
        const uint32_t* base = ents + (size_t)sg * kSegCap;
        u32x4 va[4], vb[4];
        int xa[4], xb[4];
        auto load = [&](u32x4* v, int* xs, int i0) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + u;
                int x = q0 + i + phase;
                x = x >= q1 ? x - len : x;
                xs[u] = i < len ? x : -1;
                v[u] = i < len ? gld4(base + 4 * x) : u32x4{0u, 0u, 0u, 0u};
            }
        };
        auto vote4 = [&](const u32x4* v, const int* xs) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (xs[u] < 0) continue;
                const int e0 = 4 * xs[u];
                vote(v[u].x);
                if (e0 + 1 < cnt) vote(v[u].y);
                if (e0 + 2 < cnt) vote(v[u].z);
                if (e0 + 3 < cnt) vote(v[u].w);
            }
        };
        load(va, xa, 0);
        for (int i = 0; i < len; i += 8) {
            load(vb, xb, i + 4);
            vote4(va, xa);
            load(va, xa, i + 8);
            vote4(vb, xb);
        }
    }
    __syncthreads();
    if (mode == 0) {
        for (int q = 0; q < 2; ++q) {
            const PairRow pr = q == 0 ? ra : rb;
            if (pr.row < 0) continue;
            int32_t* out = d.acc + (size_t)pr.row * d.n_r;
            for (int i = tid; i < d.n_r; i += kPairThreads) {
                const int w = i - pr.lo;
                gst(out + i, (w >= 0 && w < pr.span) ? s_acc[pr.base + w] : 0);
            }
            // LDS cells whose r_idx lies outside [0, n_r) hold dropped votes
            for (int w = tid; w < pr.span; w += kPairThreads) {
                const int i = pr.lo + w;
                if (i < 0 || i >= d.n_r) drop += (uint32_t)s_acc[pr.base + w];
            }
        }
    }
    if (d.dropped) {
        if (drop) atomicAdd(&s_drop, drop);
        __syncthreads();
        if (tid == 0 && s_drop) atomicAdd(d.dropped, s_drop);
    }
}

}  // namespace lane

using namespace lane;

extern "C" LANE_INTERNAL hipError_t lane_launch_vote_pair(const VoteDesc* dp, int pairing, hipStream_t s) {
    const VoteDesc& d = *dp;
    // workgroup g in [0, floor(n/2)]: row g with row n - g (g = 0 and g = n/2 alone)
    hipLaunchKernelGGL(k_vote_pair, dim3(d.n_theta / 2 + 1), dim3(kPairThreads), 0, s, d, pairing);
    return hipGetLastError();
}
