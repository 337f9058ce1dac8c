// Coarse-to-fine Hough transform.  The paper bases its GPU vote (Sec. 4.3)
// on a multiresolution progressive Hough method (its reference [9]) and
// gives no algorithm; this library defines it as:
//
//   coarse vote   coarse row c samples the fine row c*f + f/2; the r axis is
//                 cut into odd bins of w cells centred on r = 0, bin
//                 floor((r + q) / w) at column bin + Dc (q = (w - 1) / 2);
//   coarse peaks  the greedy peaks of lane_hough_peaks on that accumulator;
//   windows       each coarse peak opens R = f + 2 m_t unfolded fine rows by
//                 Wc = w + 2 m_r cells around its bin and counts them exactly
//                 (a row past 0 or 180 degrees reads the mirrored r, since
//                 the line (r, theta + 180) is (-r, theta));
//   final peaks   each window's largest count (first in window order) is a
//                 candidate; greedy selection among the candidates.
//
// Kernels.  k_prog_coarse: a workgroup holds T coarse rows in LDS (cell b of
// row j at word b*T + j) and votes the edges of a chunk of segments; its
// 256/T slots walk 16 segments at once, each in its own part and from its
// own phase, so the lanes of one LDS atomic come from pixels far apart
// (coarse bins are wide: neighbours would hit one cell); chunk partial rows
// go to the accumulator with global atomics.  The bin needs a division by
// w: (n + 0.5) * float(1/w) truncated is floor(n / w) exactly for
// 0 <= n < 2^22 (the float error stays below the distance 0.5/w to the next
// integer).  k_prog_refine: a workgroup holds a group of windows in LDS and
// votes a chunk of edges; an edge is tested against a window's middle row
// first and skips the window when the other rows cannot reach it (a bound
// from the table differences); the pairs that pass queue up per wave and are
// counted 64 at a time, each lane starting at its own row (the pairs of a
// line are queued together and would add into one cell at once).  The edges
// are cut into parts of segments to fill the GPU.  k_prog_cand: one
// workgroup per window takes the maximum.
// k_prog_final: one wave, greedy selection over <= 64 candidates.
#include "lane_entry.h"


namespace lane {

constexpr int kProgThreads = 256;
constexpr int kProgGroup = 16;  // segments a coarse workgroup walks at once
constexpr int kQueue = 128;     // per-wave ring of refine work (two 64-pair batches)

// LDS written by some lanes of a wave, then read by others of the same wave
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int prog_dot2(int a, int b, int c) {
    // a.lo*b.lo + a.hi*b.hi + c on signed 16-bit halves
    int d;
    asm("v_dot2_i32_i16 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

__device__ __forceinline__ int pack_cs(int C, int S) {
    return (int)(((uint32_t)(uint16_t)S << 16) | (uint32_t)(uint16_t)C);
}

__device__ __forceinline__ int floor_div_p(int a, int b) {  // b > 0
    const int q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}

template <int T>
__global__ void __launch_bounds__(kProgThreads) k_prog_coarse(ProgDesc d) {
    extern __shared__ __align__(16) int32_t s_acc[];  // (n_rc + 1) * T words; cell n_rc is a sink
    constexpr int kSlots = kProgThreads / T;
    constexpr int kParts = kSlots / kProgGroup;
    const int tid = threadIdx.x;
    const int words = (d.n_rc + 1) * T;
    for (int i = tid; i < words; i += kProgThreads) s_acc[i] = 0;

    const int c0 = blockIdx.x * T;
    const int j = tid & (T - 1);
    const int slot = tid / T;
    const int g = slot % kProgGroup, p = slot / kProgGroup;
    const int c = c0 + j;
    const bool row_ok = c < d.n_c;
    const int t = (row_ok ? c : d.n_c - 1) * d.f + d.f / 2;
    const int CS = pack_cs(gld(d.cos_q14 + t), gld(d.sin_q14 + t));
    // nn = r + q + w Dc, in [0, 2 D + 2 q] exactly when r is in [-D, D]
    const int K = 8192 + (d.q + d.w * d.Dc) * 16384;
    const uint32_t lo = (uint32_t)(d.q + d.w * d.Dc - d.D);
    const uint32_t span = 2u * (uint32_t)d.D;
    const float iw = d.inv_w, hiw = 0.5f * d.inv_w;
    const int sink = d.n_rc * T + j;
    __syncthreads();

    auto vote = [&](uint32_t xy, bool valid) {
        const int nn = prog_dot2((int)xy, CS, K) >> 14;
        const bool ok = valid && ((uint32_t)nn - lo) <= span;
        const int b = (int)__builtin_fmaf((float)nn, iw, hiw);
        atomicAdd(s_acc + (ok ? b * T + j : sink), 1);
    };

    const ListLayout L = list_layout(d.W, d.H);
    const uint32_t* ents = d.list + L.off_ent;
    const int n_groups = (L.nseg + kProgGroup - 1) / kProgGroup;
    const int gr0 = blockIdx.y * d.groups_per_chunk;
    const int gr1 = min(gr0 + d.groups_per_chunk, n_groups);
    if (row_ok) {
        for (int gr = gr0; gr < gr1; ++gr) {
            const int seg = gr * kProgGroup + g;
            const int n = seg < L.nseg ? (int)gld(d.list + seg) : 0;
            const int nq = (n + 3) >> 2;  // 4 entries per 128-bit load
            const int pq = (nq + kParts - 1) / kParts;
            const int q0 = min(p * pq, nq), q1 = min(q0 + pq, nq);
            const int len = q1 - q0;
            const int phase = (g * len) / kProgGroup;
            const uint32_t* base = ents + (size_t)seg * kSegCap;
            // two register sets take turns: one set of four 128-bit loads is
            // in flight while the other is voted
            u32x4 a[4], b[4];
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
                    const bool in = xs[u] >= 0;
                    const int e0 = 4 * xs[u];
                    vote(v[u].x, in && e0 + 0 < n);
                    vote(v[u].y, in && e0 + 1 < n);
                    vote(v[u].z, in && e0 + 2 < n);
                    vote(v[u].w, in && e0 + 3 < n);
                }
            };
            load(a, xa, 0);
            for (int i = 0; i < len; i += 8) {
                load(b, xb, i + 4);
                vote4(a, xa);
                load(a, xa, i + 8);
                vote4(b, xb);
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < d.n_rc * T; i += kProgThreads) {
        const int v = s_acc[i];
        const int cc = c0 + (i & (T - 1));
        if (v != 0 && cc < d.n_c) atomicAdd(d.coarse_acc + (size_t)cc * d.n_rc + (i / T), v);
    }
}

// Per-row constants of a window group: packed table row, mirror mask.
struct RefineRow {
    int cs, m;
};
struct RefineWin {
    int ok, rlo, cs_mid, m_mid, reach;  // reach: |e(row) - e(mid row)| bound
};

__global__ void __launch_bounds__(kProgThreads) k_prog_refine(ProgDesc d) {
    extern __shared__ __align__(16) int32_t s_dyn[];
    const int wpg = d.wpg, R = d.R, Wc = d.Wc;
    const int cells = wpg * R * Wc;
    int32_t* s_win = s_dyn;
    RefineRow* s_row = (RefineRow*)(s_dyn + cells);
    RefineWin* s_w = (RefineWin*)(s_row + wpg * R);
    const int tid = threadIdx.x;
    const int j0 = blockIdx.y * wpg;
    const int n_coarse = gld(d.cpk + 3 * d.kc);

    for (int i = tid; i < cells; i += kProgThreads) s_win[i] = 0;
    for (int i = tid; i < wpg * R; i += kProgThreads) {
        const int jj = i / R, a = i - jj * R, j = j0 + jj;
        int cs = 0, m = 0;
        if (j < d.kc && j < n_coarse) {
            const int u = gld(d.cpk + j) * d.f - d.mt + a;
            const int h = floor_div_p(u, d.n_theta);
            const int tt = u - h * d.n_theta;
            cs = pack_cs(gld(d.cos_q14 + tt), gld(d.sin_q14 + tt));
            m = (h & 1) ? -1 : 0;
        }
        s_row[i] = RefineRow{cs, m};
    }
    __syncthreads();
    if (tid < wpg) {
        const int j = j0 + tid;
        RefineWin W{0, 0, 0, 0, 0};
        if (j < d.kc && j < n_coarse) {
            W.ok = 1;
            W.rlo = (gld(d.cpk + d.kc + j) - d.Dc) * d.w - d.q - d.mr;
            const int am = R / 2;
            const RefineRow rm = s_row[tid * R + am];
            W.cs_mid = rm.cs;
            W.m_mid = rm.m;
            // |U_a - U_mid| <= (|dCu| (W-1) + |dSu| (H-1) + |s_a - s_mid| 2^13) / 2^14 + 2,
            // Cu, Su the table row with the unfolding sign applied
            const int sm = rm.m ? -1 : 1;
            const int cm = sm * (int)(int16_t)(rm.cs & 0xFFFF), snm = sm * (int)(int16_t)(rm.cs >> 16);
            long long worst = 0;
            for (int a = 0; a < R; ++a) {
                const RefineRow ra = s_row[tid * R + a];
                const int sa = ra.m ? -1 : 1;
                const long long dc = (long long)sa * (int16_t)(ra.cs & 0xFFFF) - cm;
                const long long ds = (long long)sa * (int16_t)(ra.cs >> 16) - snm;
                const long long b = (dc < 0 ? -dc : dc) * (d.W - 1) + (ds < 0 ? -ds : ds) * (d.H - 1) +
                                    (sa != sm ? 16384 : 0);
                worst = b > worst ? b : worst;
            }
            W.reach = (int)(worst >> 14) + 2;
        }
        s_w[tid] = W;
    }
    __syncthreads();

    // this workgroup's share of the edges: units u0 .. u1 - 1, unit u being
    // part u % P of segment u / P (P parts of equal quad counts)
    const ListLayout L = list_layout(d.W, d.H);
    const uint32_t* ents = d.list + L.off_ent;
    const int P = d.r_parts;
    const long units = (long)L.nseg * P;
    const int u0 = (int)((units * blockIdx.x) / d.r_chunks);
    const int u1 = (int)((units * (blockIdx.x + 1)) / d.r_chunks);
    const uint32_t span = 2u * (uint32_t)d.D;
    const int nw = min(wpg, max(0, min(d.kc, n_coarse) - j0));

    // Pairs (edge, window) that pass the reach test go to a per-wave ring in
    // LDS; every 64 of them are counted row by row with all lanes busy (a
    // wave would otherwise run a window's rows whenever one lane needs them).
    __shared__ uint32_t s_qxy[kProgThreads / kWave][kQueue];
    __shared__ int s_qj[kProgThreads / kWave][kQueue];
    const int lane = tid & (kWave - 1), wv = tid >> 6;
    uint32_t* qxy = s_qxy[wv];
    int* qj = s_qj[wv];
    int qt = 0, qn = 0;  // ring tail and fill, the same in every lane of the wave

    auto drain = [&](int nact) {
        wave_sync();
        if (lane < nact) {
            const int slot = (qt + lane) & (kQueue - 1);
            const uint32_t xy = qxy[slot];
            const int jj = qj[slot];
            const RefineRow* rows = s_row + jj * R;
            int32_t* win = s_win + jj * R * Wc;
            const int rlo = s_w[jj].rlo;
            // lanes start at different rows (the pairs of a line are queued
            // together and would add into one cell at once); the constants of
            // eight rows are read before any is used
            const int a0 = lane % R;
            for (int k0 = 0; k0 < R; k0 += 8) {
                RefineRow rr[8];
                int ar[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int k = k0 + u;
                    const int a = a0 + k < R ? a0 + k : a0 + k - R;
                    ar[u] = a;
                    rr[u] = rows[k < R ? a : 0];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int r = prog_dot2((int)xy, rr[u].cs, 8192) >> 14;
                    const int e = (r ^ rr[u].m) - rr[u].m - rlo;
                    if (k0 + u < R && (uint32_t)(r + d.D) <= span && (uint32_t)e < (uint32_t)Wc)
                        atomicAdd(win + ar[u] * Wc + e, 1);
                }
            }
        }
        wave_sync();
        qt = (qt + nact) & (kQueue - 1);
        qn -= nact;
    };

    auto offer = [&](uint32_t xy, bool valid) {
        for (int jb = 0; jb < nw; jb += 4) {
            // four windows' constants read together, then four tests
            RefineWin w4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) w4[u] = s_w[jb + u < nw ? jb + u : nw - 1];
            bool pass[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int rm = prog_dot2((int)xy, w4[u].cs_mid, 8192) >> 14;
                const int em = (rm ^ w4[u].m_mid) - w4[u].m_mid - w4[u].rlo;
                pass[u] = valid && jb + u < nw &&
                          (uint32_t)(em + w4[u].reach) <= (uint32_t)(Wc - 1 + 2 * w4[u].reach);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const unsigned long long m = __ballot(pass[u]);
                if (pass[u]) {
                    const int before = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    const int pos = (qt + qn + before) & (kQueue - 1);
                    qxy[pos] = xy;
                    qj[pos] = jb + u;
                }
                qn += __popcll(m);
                if (qn >= kWave) drain(kWave);
            }
        }
    };

    if (nw > 0) {
        for (int un = u0; un < u1; ++un) {
            const int sg = un / P, part = un - sg * P;
            const int n = (int)gld(d.list + sg);
            const uint32_t* base = ents + (size_t)sg * kSegCap;
            const int nq = (n + 3) >> 2;
            const int qa = (int)(((long)nq * part) / P), qb = (int)(((long)nq * (part + 1)) / P);
            for (int q0 = qa + wv * kWave; q0 < qb; q0 += kProgThreads) {  // the same trips in every lane
                const int qi = q0 + lane;
                const bool okq = qi < qb;
                const u32x4 e = okq ? gld4(base + 4 * qi) : u32x4{0u, 0u, 0u, 0u};
                const int e0 = 4 * qi;
                offer(e.x, okq);
                offer(e.y, okq && e0 + 1 < n);
                offer(e.z, okq && e0 + 2 < n);
                offer(e.w, okq && e0 + 3 < n);
            }
        }
        if (qn > 0) drain(qn);
    }
    __syncthreads();
    const int used = nw * R * Wc;
    int32_t* out = d.windows + (size_t)j0 * R * Wc;
    for (int i = tid; i < used; i += kProgThreads) {
        const int v = s_win[i];
        if (v != 0) atomicAdd(out + i, v);
    }
}

// Window j's largest count, first in (row, cell) order among cells whose
// r lies in [-D, D].
__global__ void __launch_bounds__(kProgThreads) k_prog_cand(ProgDesc d) {
    __shared__ unsigned long long s_best[kProgThreads / kWave];
    const int j = blockIdx.x, tid = threadIdx.x;
    const int n_coarse = gld(d.cpk + 3 * d.kc);
    if (j >= n_coarse) {
        if (tid < 3) gst(d.cand + 3 * j + tid, -1);
        return;
    }
    const int c = gld(d.cpk + j);
    const int rlo = (gld(d.cpk + d.kc + j) - d.Dc) * d.w - d.q - d.mr;
    const int cells = d.R * d.Wc;
    const int32_t* win = d.windows + (size_t)j * cells;
    unsigned long long best = 0;  // (count << 32) | ~index; 0 = none
    for (int i = tid; i < cells; i += kProgThreads) {
        const int a = i / d.Wc, e = i - a * d.Wc;
        const int v = gld(win + i);
        const int ru = rlo + e;
        if (ru < -d.D || ru > d.D) continue;
        const unsigned long long key = ((unsigned long long)(uint32_t)v << 32) | (uint32_t)~(uint32_t)i;
        best = key > best ? key : best;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long x = __shfl_xor(best, o);
        best = x > best ? x : best;
    }
    if ((tid & (kWave - 1)) == 0) s_best[tid >> 6] = best;
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < kProgThreads / kWave; ++w) best = s_best[w] > best ? s_best[w] : best;
        if (best == 0) {
            gst(d.cand + 3 * j, -1);
            gst(d.cand + 3 * j + 1, -1);
            gst(d.cand + 3 * j + 2, -1);
        } else {
            const int i = (int)~(uint32_t)(best & 0xFFFFFFFFull);
            const int a = i / d.Wc, e = i - a * d.Wc;
            const int u = c * d.f - d.mt + a;
            const int h = floor_div_p(u, d.n_theta);
            const int ru = rlo + e;
            gst(d.cand + 3 * j, u - h * d.n_theta);
            gst(d.cand + 3 * j + 1, ((h & 1) ? -ru : ru) + d.D);
            gst(d.cand + 3 * j + 2, (int)(best >> 32));
        }
    }
}

// Greedy selection among the candidates (one wave, lane l = candidate l):
// largest count first, ties to the smaller theta-major index; a selected
// line suppresses candidates within h_theta rows and h_r cells, a row past
// either end of the half turn read mirrored (h_theta < n_theta).
__global__ void __launch_bounds__(kWave) k_prog_final(ProgDesc d) {
    const int l = threadIdx.x;
    const int n_coarse = gld(d.cpk + 3 * d.kc);
    const int n_r = 2 * d.D + 1;
    int t = -1, col = -1, v = -1;
    if (l < d.kc && l < n_coarse) {
        t = gld(d.cand + 3 * l);
        col = gld(d.cand + 3 * l + 1);
        v = gld(d.cand + 3 * l + 2);
    }
    const int floor_votes = d.min_votes > 1 ? d.min_votes : 1;
    bool alive = t >= 0 && v >= floor_votes;
    int found = 0;
    for (int s = 0; s < d.k; ++s) {
        unsigned long long key =
            alive ? ((unsigned long long)(uint32_t)v << 32) | (uint32_t)~(uint32_t)(t * n_r + col) : 0ull;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long x = __shfl_xor(key, o);
            key = x > key ? x : key;
        }
        if (key == 0) break;  // uniform
        const int idx = (int)~(uint32_t)(key & 0xFFFFFFFFull);
        const int ts = idx / n_r, cs = idx - ts * n_r, vs = (int)(key >> 32);
        if (l == 0) {
            gst(d.theta_idx + s, ts);
            gst(d.r_idx + s, cs);
            gst(d.votes + s, vs);
        }
        ++found;
        if (alive) {
            const int dt = t - ts;
            const int dc = col - cs, dm = col - (2 * d.D - cs);
            const bool same = (dt <= d.ht && -dt <= d.ht) && (dc <= d.hr && -dc <= d.hr);
            const bool wrap = ((dt - d.n_theta <= d.ht && d.n_theta - dt <= d.ht) ||
                               (dt + d.n_theta <= d.ht && -dt - d.n_theta <= d.ht)) &&
                              (dm <= d.hr && -dm <= d.hr);
            if (same || wrap) alive = false;
        }
    }
    for (int s = found + l; s < d.k; s += kWave) {
        gst(d.theta_idx + s, -1);
        gst(d.r_idx + s, -1);
        gst(d.votes + s, -1);
    }
    if (l == 0) gst(d.count, found);
}

}  // namespace lane

using namespace lane;

// Coarse peaks run as lane_hough_peaks with the caller's descriptor `pk`
// (its accumulator is d.coarse_acc, its outputs the d.cpk arrays).
extern "C" LANE_INTERNAL hipError_t lane_launch_progressive(const ProgDesc* dp, const PeaksDesc* pk,
                                                            hipStream_t s) {
    const ProgDesc& d = *dp;
    hipError_t e = lane_launch_fill_u32((uint32_t*)d.coarse_acc, (size_t)d.n_c * d.n_rc, 0u, s);
    if (e != hipSuccess) return e;
    e = lane_launch_fill_u32((uint32_t*)d.windows, (size_t)d.kc * d.R * d.Wc, 0u, s);
    if (e != hipSuccess) return e;

    const size_t lds_c = (size_t)(d.n_rc + 1) * d.T * sizeof(int32_t);
    const dim3 gc(d.n_slices, d.n_chunks);
    if (d.T == 4)
        hipLaunchKernelGGL(k_prog_coarse<4>, gc, dim3(kProgThreads), lds_c, s, d);
    else if (d.T == 2)
        hipLaunchKernelGGL(k_prog_coarse<2>, gc, dim3(kProgThreads), lds_c, s, d);
    else
        hipLaunchKernelGGL(k_prog_coarse<1>, gc, dim3(kProgThreads), lds_c, s, d);
    e = hipGetLastError();
    if (e != hipSuccess) return e;

    e = lane_launch_peaks(pk, s);
    if (e != hipSuccess) return e;

    hipLaunchKernelGGL(k_prog_refine, dim3(d.r_chunks, d.n_wgroups), dim3(kProgThreads),
                       lane_prog_refine_lds(d.wpg, d.R, d.Wc), s, d);
    hipLaunchKernelGGL(k_prog_cand, dim3(d.kc), dim3(kProgThreads), 0, s, d);
    hipLaunchKernelGGL(k_prog_final, dim3(1), dim3(kWave), 0, s, d);
    return hipGetLastError();
}
