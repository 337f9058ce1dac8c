// Hough peaks for gfx950: exact greedy non-maximum suppression.
//
// What is computed (Sec. 2.3: the largest accumulator counts are the lines;
// the paper hands this step to MATLAB, the procedure here is the greedy
// suppression documented in lane.h): up to k times take the largest
// unsuppressed cell (ties to the smaller theta-major index), stop below
// max(1, min_votes), emit it and suppress its window, with theta wrapping
// and the r window mirrored for an odd number of wraps.
//
// Design.  Pass 1 (many workgroups, reads the accumulator once): one wave
// per block of B cells writes the block's best key, key = (count, -index)
// packed in 64 bits so that one unsigned max gives "largest count, then
// smallest index".  Pass 2 (one workgroup per frame) first tries a
// candidate set: a histogram of the block maxima gives the lowest count tau
// such that at most 256 blocks of at most 16384 cells in all (65536 for
// k > 16) reach it, the
// cells >= tau of those blocks (every cell >= tau in the frame) are loaded
// into LDS once, and the greedy rounds run over them alone, one barrier per
// round and no memory access.  A pick among the candidates is the frame's
// pick as long as one is left: every cell outside the set counts less than
// tau.  If the set runs out before k peaks while tau is above the vote
// floor (or does not fit), the frame is redone by the general search: the
// block keys sit in LDS with one group key per 32 blocks; each round every
// wave finds the maximum over the group keys by itself (a DPP reduction, no
// barrier), lists
// the earlier peaks whose windows can reach the new window's rows (one
// ballot), and only the blocks touched by the new window are rescanned
// (skipping every suppressed cell), the cells of all touched blocks spread
// over the whole workgroup with their loads issued together; the new block
// keys go to a scratch array (two buffers taking turns) and the touched
// groups are recomputed, so a round costs O(window), one memory round trip
// and two barriers.
#include "lane_entry.h"

namespace lane {

__device__ __forceinline__ int key_value(unsigned long long k) {
    return (int)((uint32_t)(k >> 32) ^ 0x80000000u);
}
__device__ __forceinline__ uint32_t key_index(unsigned long long k) {
    return 0xFFFFFFFFu - (uint32_t)k;
}


__device__ __forceinline__ int floor_div_i(int a, int b) {
    int q = a / b;
    if ((a % b != 0) && (a < 0)) --q;
    return q;
}

// true if cell (t, i) lies in the suppression window of peak (tp, ip)
__device__ __forceinline__ bool in_window(int t, int i, int tp, int ip, const PeaksDesc& d) {
    const int n = d.n_theta;
    const int qlo = -floor_div_i(t - (tp - d.h_theta), n);  // ceil((tp - h - t) / n)
    const int qhi = floor_div_i(tp + d.h_theta - t, n);
    for (int q = qlo; q <= qhi; ++q) {
        const int centre = (q & 1) ? 2 * d.r_offset - ip : ip;
        if (abs(i - centre) <= d.h_r) return true;
    }
    return false;
}

// key of block b = (row t, column chunk j): cells t*n_r + [j*B, min(n_r, (j+1)*B))
__device__ __forceinline__ void block_key(const PeaksDesc& d, int b, int lane) {
    const int t = b / d.nbr, j = b - t * d.nbr;
    const int B = 1 << d.block_log2;
    const int i0 = j * B, i1 = min(d.n_r, i0 + B);
    const uint32_t rowc = (uint32_t)t * (uint32_t)d.n_r;
    unsigned long long best = 0;
    for (int i = i0 + lane; i < i1; i += kWave) {
        const unsigned long long k = make_key(gld(d.acc + rowc + i), rowc + (uint32_t)i);
        best = k > best ? k : best;
    }
    best = wave_max_u64(best);
    if (lane == 0) gst(d.keys + b, best);
}

__global__ void __launch_bounds__(256) k_block_keys(PeaksDesc d) {
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= d.n_blocks) return;
    block_key(d, b, threadIdx.x & (kWave - 1));
}

// Batched: blockIdx.y = frame (a frame switched off leaves at once),
// workgroups of a frame stride over its blocks, one wave per block; blocks
// of up to 256 cells go four at a time, every load of the four issued
// before the first maximum (a wave walks many blocks: one memory round trip
// per four instead of one per block).
// Block keys of the frames in `list` (device: counts[3] frame indices,
// refreshed per selection), after a split vote: the grid is shared out
// evenly over those frames, so one frame alone gets all of it.
__global__ void __launch_bounds__(256) k_block_keys_batch(const PeaksDesc* __restrict__ descs,
                                                          const int* __restrict__ list,
                                                          const int* __restrict__ counts) {
    const int na = gld(counts + 3);
    if (na <= 0) return;
    const int per = max(1, (int)gridDim.x / na);  // workgroups per frame
    const int fi = (int)blockIdx.x / per;
    if (fi >= na) return;
    const PeaksDesc d = descs[gld(list + fi)];
    if (!frame_on(d.active)) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int stride = per * 4;
    int b = ((int)blockIdx.x - fi * per) * 4 + (threadIdx.x >> 6);
    if (d.block_log2 <= 8) {
        constexpr int U = 4, Q = 4;  // blocks per round, cells per lane and block
        const int B = 1 << d.block_log2;
        for (; b < d.n_blocks; b += U * stride) {
            int v[U][Q];
            uint32_t idx[U][Q];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int bb = min(b + u * stride, d.n_blocks - 1);
                const int t = bb / d.nbr, j = bb - t * d.nbr;
                const uint32_t rowc = (uint32_t)t * (uint32_t)d.n_r;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int i = j * B + q * kWave + lane;
                    const bool ok = q * kWave + lane < B && i < d.n_r;
                    idx[u][q] = ok ? rowc + (uint32_t)i : 0xFFFFFFFFu;
                    v[u][q] = gld(d.acc + (ok ? rowc + (uint32_t)i : rowc));
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                unsigned long long best = 0;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    if (idx[u][q] == 0xFFFFFFFFu) continue;
                    const unsigned long long k = make_key(v[u][q], idx[u][q]);
                    best = k > best ? k : best;
                }
                best = wave_max_u64(best);
                if (lane == 0 && b + u * stride < d.n_blocks) gst(d.keys + b + u * stride, best);
            }
        }
        return;
    }
    for (; b < d.n_blocks; b += stride) block_key(d, b, lane);
}

constexpr int kGroupLog2 = 5;                                  // 32 block keys per group key
constexpr int kMaxGroups = kPeaksMaxBlocksLds >> kGroupLog2;
constexpr int kTaskMax = 1024;                                 // rescan tasks of the two-buffer path
constexpr int kSelWavesMax = 16;
__shared__ unsigned long long s_keys[kPeaksMaxBlocksLds];
__shared__ unsigned long long s_gkey[kMaxGroups];
__shared__ unsigned long long s_new[2][kTaskMax];   // a round's rescanned block keys, by task
__shared__ int s_sel_t[1024], s_sel_i[1024];
__shared__ int s_rel[kSelWavesMax][kWave];          // per wave: earlier peaks that reach the rows
// candidate path
constexpr int kCandSlots = 4;                                  // candidates per thread (1024 threads)
constexpr int kCandMax = kCandSlots * 1024;
constexpr int kSelBlocksMax = 256;                             // blocks whose cells are gathered
constexpr int kGatherSmallK = 16384;   // cells gathered at most for k <= 16
constexpr int kGatherLargeK = 65536;   // and for larger k
__shared__ unsigned long long s_cand[kCandMax];
__shared__ uint32_t s_bbase[kSelBlocksMax];  // gathered blocks: first cell (theta-major index)
__shared__ int s_bcnt[kSelBlocksMax];        // and cell count
__shared__ uint32_t s_hist[256];
__shared__ unsigned long long s_wbest[2][kSelWavesMax];
__shared__ int s_wv[kSelWavesMax];
__shared__ int s_nsel, s_ncand;

// in_window without divisions for the usual h_theta < n_theta, where a
// cell's row can meet the window only unwrapped or wrapped once either way
// (both wraps mirror the r centre)
__device__ __forceinline__ bool in_window_fast(int t, int i, int tp, int ip, const PeaksDesc& d) {
    const int n = d.n_theta, h = d.h_theta;
    if (h >= n) return in_window(t, i, tp, ip, d);
    if (abs(t - tp) <= h && abs(i - ip) <= d.h_r) return true;
    const int mir = 2 * d.r_offset - ip;
    if ((t - n >= tp - h || t + n <= tp + h) && abs(i - mir) <= d.h_r) return true;
    return false;
}

__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Candidate search (see the top of the file).  Returns the number of peaks
// found, or -1 if the general search has to run.  Block keys are in s_keys,
// vmax >= floor_votes is the largest block count, s_hist and the counters
// are zero.
__device__ int peaks_candidates(const PeaksDesc& d, int floor_votes, int vmax) {
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid >> 6, nwaves = blockDim.x >> 6;
    const int nthreads = blockDim.x;
    const int lg = d.block_log2, B = 1 << lg;
    int found = 0;
    // histogram of the block maxima >= floor, 256 bins of 2^s counts
    const uint32_t span = (uint32_t)(vmax - floor_votes);
    const int s = max(0, (span ? 32 - __builtin_clz(span) : 0) - 8);
    for (int b = tid; b < d.n_blocks; b += nthreads) {
        const unsigned long long kb = s_keys[b];
        const int v = kb ? key_value(kb) : INT_MIN;
        if (v >= floor_votes) atomicAdd(&s_hist[(uint32_t)(v - floor_votes) >> s], 1u);
    }
    __syncthreads();
    // beta = the lowest bin such that at most NB blocks lie in it or
    // above (every wave works it out for itself): lane l holds bins
    // 4l .. 4l + 3, suffix sums over the lanes
    const int NB = min(kSelBlocksMax, max(1, (d.k <= 16 ? kGatherSmallK : kGatherLargeK) >> lg));
    uint32_t h[4], lsum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        h[q] = s_hist[4 * lane + q];
        lsum += h[q];
    }
    uint32_t suf = lsum;  // sum over lanes >= lane
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t t = (uint32_t)__shfl_down((int)suf, o);
        if (lane + o < kWave) suf += t;
    }
    int qmin = 4;
    uint32_t sq = suf;  // suffix from bin 4 lane + q
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (qmin == 4 && sq <= (uint32_t)NB) qmin = q;
        sq -= h[q];
    }
    const unsigned long long okm = __ballot(qmin < 4);
    // the suffix only falls with the bin, so the lowest lane that
    // qualifies holds beta; none: more than NB blocks in the top bin
    if (okm == 0ull) return -1;
    const int Lq = __builtin_ctzll(okm);
    const int beta = 4 * Lq + __shfl(qmin, Lq);
    const long long tau64 = (long long)floor_votes + ((long long)beta << s);
    // beta past the top bin: more than NB blocks share it
    if (tau64 > (long long)vmax) return -1;
    const int tau = (int)tau64;
    // the blocks that reach tau (at most NB)
    for (int b0 = wave * kWave; b0 < d.n_blocks; b0 += nthreads) {
        const int b = b0 + lane;
        const unsigned long long kb = b < d.n_blocks ? s_keys[b] : 0ull;
        const bool keep = kb != 0ull && key_value(kb) >= tau;
        const unsigned long long mk = __ballot(keep);
        if (mk == 0ull) continue;
        int base = 0;
        if (lane == 0) base = atomicAdd(&s_nsel, __popcll(mk));
        base = __shfl(base, 0);
        if (keep) {
            const int pos = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
            const int t = b / d.nbr, c0 = (b - t * d.nbr) << lg;
            s_bbase[pos] = (uint32_t)t * (uint32_t)d.n_r + (uint32_t)c0;
            s_bcnt[pos] = min(B, d.n_r - c0);
        }
    }
    __syncthreads();
    // their cells >= tau into the candidate array: batches of four loads
    // per lane, the next batch in flight while one is filtered, and one LDS
    // atomic per batch and wave for the positions
    const int nsel = s_nsel;
    const int ncells = nsel << lg;
    constexpr int U = 4;
    const int step = U * nthreads;
    auto load = [&](int c0, uint32_t* ii, int* vv) {  // ii = ~0u: no cell
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = c0 + u * nthreads + lane;
            const int q = min(c, ncells - 1) >> lg, w = c & (B - 1);
            ii[u] = (c < ncells && w < s_bcnt[q]) ? s_bbase[q] + (uint32_t)w : ~0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) vv[u] = gld(d.acc + (ii[u] != ~0u ? ii[u] : 0u));
    };
    auto take = [&](const uint32_t* ii, const int* vv) {
        unsigned long long mk[U];
        int tot = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            mk[u] = __ballot(ii[u] != ~0u && vv[u] >= tau);
            tot += __popcll(mk[u]);
        }
        if (tot == 0) return;
        int base = 0;
        if (lane == 0) base = atomicAdd(&s_ncand, tot);
        base = __shfl(base, 0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if ((mk[u] >> lane) & 1ull) {
                const int pos = base + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mk[u] >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)mk[u], 0u));
                if (pos < kCandMax) s_cand[pos] = make_key(vv[u], ii[u]);
            }
            base += __popcll(mk[u]);
        }
    };
    {
        uint32_t ia[U], ib[U];
        int va[U], vb[U];
        int c0 = wave * kWave;
        if (c0 < ncells) load(c0, ia, va);
        for (; c0 < ncells; c0 += 2 * step) {
            if (c0 + step < ncells) load(c0 + step, ib, vb);
            take(ia, va);
            if (c0 + step < ncells) {
                if (c0 + 2 * step < ncells) load(c0 + 2 * step, ia, va);
                take(ib, vb);
            }
        }
    }
    __syncthreads();
    const int nc = s_ncand;
    if (nc > kCandMax || nthreads * kCandSlots < kCandMax) return -1;
    unsigned long long ck[kCandSlots];
    int ct[kCandSlots], ci[kCandSlots];
#pragma unroll
    for (int m = 0; m < kCandSlots; ++m) {
        const int c = tid + m * nthreads;
        ck[m] = c < nc ? s_cand[c] : 0ull;
        const uint32_t idx = key_index(ck[m]);
        ct[m] = ck[m] ? (int)(idx / (uint32_t)d.n_r) : 0;
        ci[m] = ck[m] ? (int)(idx - (uint32_t)ct[m] * (uint32_t)d.n_r) : 0;
    }
    bool ran_out = false;
    for (int j = 0; j < d.k; ++j) {
        unsigned long long best = 0;
#pragma unroll
        for (int m = 0; m < kCandSlots; ++m) best = ck[m] > best ? ck[m] : best;
        best = wave_max_u64(best);
        if (lane == 0) s_wbest[j & 1][wave] = best;
        __syncthreads();
        const unsigned long long mx = wave_max_u64(lane < nwaves ? s_wbest[j & 1][lane] : 0ull);
        if (mx == 0ull) {
            ran_out = true;
            break;
        }
        const uint32_t idx = key_index(mx);
        const int t = (int)(idx / (uint32_t)d.n_r), i = (int)(idx % (uint32_t)d.n_r);
        if (tid == 0) {
            d.theta_idx[j] = t;
            d.r_idx[j] = i;
            d.votes[j] = key_value(mx);
        }
        found = j + 1;
#pragma unroll
        for (int m = 0; m < kCandSlots; ++m)
            if (ck[m] && in_window_fast(ct[m], ci[m], t, i, d)) ck[m] = 0ull;
    }
    // out of candidates: every cell left counts less than tau, so the
    // search is over if tau is the floor, else the general search redoes it
    if (!ran_out || tau == floor_votes) return found;
    return -1;
}

// General search (see the top of the file); block keys are in s_keys.
// Returns the number of peaks found.
__device__ int peaks_general(const PeaksDesc& d, int floor_votes) {
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid >> 6, nwaves = blockDim.x >> 6;
    const int nthreads = blockDim.x;
    const int lg = d.block_log2, B = 1 << lg;
    const int n_groups = (d.n_blocks + (1 << kGroupLog2) - 1) >> kGroupLog2;
    int found = 0;
    for (int q = tid; q < 2 * kTaskMax; q += nthreads) s_new[q / kTaskMax][q % kTaskMax] = 0;
    // group keys: the maximum of 32 consecutive block keys
    for (int g = wave; g < n_groups; g += nwaves) {
        const int b = (g << kGroupLog2) + (lane & 31);
        const unsigned long long v = (lane < 32 && b < d.n_blocks) ? s_keys[b] : 0ull;
        const unsigned long long m = wave_max_u64(v);
        if (lane == 0) s_gkey[g] = m;
    }
    __syncthreads();
    // blocks a window can touch: 2 h_theta + 1 rows (all blocks when the
    // rows would repeat), each a contiguous column range of at most nbw
    // blocks.  Few tasks: the rescanned keys go to s_new (two buffers taking
    // turns), so a round needs two barriers; otherwise the touched blocks
    // are cleared and rescanned in place (three).
    const bool all_rows = 2 * d.h_theta + 1 > d.n_theta;
    const int nbw = min(d.nbr, ((2 * d.h_r) >> lg) + 2);
    const int ntask = all_rows ? d.n_blocks : (2 * d.h_theta + 1) * nbw;
    const bool two_buf = !all_rows && ntask <= kTaskMax;
    for (int j = 0; j < d.k; ++j) {
        // every wave finds the largest key itself: no barrier to share it
        unsigned long long best = 0;
        for (int g = lane; g < n_groups; g += kWave) best = s_gkey[g] > best ? s_gkey[g] : best;
        const unsigned long long m = wave_max_u64(best);
        if (m == 0 || key_value(m) < floor_votes) break;  // the same decision in every wave
        const uint32_t idx = key_index(m);
        const int t = (int)(idx / (uint32_t)d.n_r), i = (int)(idx % (uint32_t)d.n_r);
        if (tid == 0) {
            d.theta_idx[j] = t;
            d.r_idx[j] = i;
            d.votes[j] = key_value(m);
            s_sel_t[j] = t;
            s_sel_i[j] = i;
        }
        found = j + 1;
        if (found == d.k) break;  // no further round reads the keys

        // task -> (row, block column) of the new window, -1 if none
        auto task_block = [&](int task, int& row) -> int {
            if (all_rows) {
                row = task / d.nbr;
                return task - row * d.nbr;
            }
            const int r = task / nbw, bi = task - r * nbw;
            const int traw = t - d.h_theta + r;
            const int q = floor_div_i(traw, d.n_theta);
            row = traw - q * d.n_theta;
            const int centre = (q & 1) ? 2 * d.r_offset - i : i;
            const int ca = max(0, centre - d.h_r), cb = min(d.n_r - 1, centre + d.h_r);
            return (ca > cb || (ca >> lg) + bi > (cb >> lg)) ? -1 : (ca >> lg) + bi;
        };
        // the task of block (row, jb) in this round, -1 if untouched (two-buffer path)
        auto block_task = [&](int row, int jb) -> int {
            int r = row - (t - d.h_theta);
            r %= d.n_theta;
            if (r < 0) r += d.n_theta;
            if (r > 2 * d.h_theta) return -1;
            const int traw = t - d.h_theta + r;
            const int q = floor_div_i(traw, d.n_theta);
            const int centre = (q & 1) ? 2 * d.r_offset - i : i;
            const int ca = max(0, centre - d.h_r), cb = min(d.n_r - 1, centre + d.h_r);
            if (ca > cb || jb < (ca >> lg) || jb > (cb >> lg)) return -1;
            return r * nbw + (jb - (ca >> lg));
        };

        // earlier peaks whose windows reach the new window's rows (cyclic
        // row distance <= 2 h_theta); each wave lists them for itself
        int nrel = 0;
        for (int p0 = 0; p0 < j; p0 += kWave) {
            const int p = p0 + lane;
            bool rel = false;
            if (p < j) {
                int dt = abs(t - s_sel_t[p]) % d.n_theta;
                dt = min(dt, d.n_theta - dt);
                rel = all_rows || dt <= 2 * d.h_theta;
            }
            const unsigned long long mk = __ballot(rel);
            if (rel) {
                const int pos = nrel + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
                if (pos < kWave) s_rel[wave][pos] = p;
            }
            nrel += __popcll(mk);
        }
        wave_lds_sync();
        const bool rel_all = nrel > kWave;  // too many to list: test every earlier peak
        auto suppressed = [&](int row, int cell) {
            if (in_window_fast(row, cell, t, i, d)) return true;
            if (rel_all) {
                for (int p = 0; p < j; ++p)
                    if (in_window_fast(row, cell, s_sel_t[p], s_sel_i[p], d)) return true;
                return false;
            }
            for (int q = 0; q < nrel; ++q) {
                const int p = s_rel[wave][q];
                if (in_window_fast(row, cell, s_sel_t[p], s_sel_i[p], d)) return true;
            }
            return false;
        };

        unsigned long long* snew = s_new[j & 1];
        if (two_buf) {
            // the other buffer was read in the previous round: clear it for the next
            for (int q = tid; q < ntask; q += nthreads) s_new[(j & 1) ^ 1][q] = 0;
        } else {
            for (int task = tid; task < ntask; task += nthreads) {
                int row;
                const int jb = task_block(task, row);
                if (jb >= 0) s_keys[row * d.nbr + jb] = 0;
            }
            __syncthreads();
        }
        // rescan: every thread takes cells of the touched blocks, all loads
        // of a group of eight first, then the suppression tests and an LDS max
        const int ncell = ntask << lg;
        for (int c0 = tid; c0 < ncell; c0 += 8 * nthreads) {
            int tk[8], rw[8], ce[8], ii[8], vv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int c = c0 + u * nthreads;
                int row = 0, jb = -1;
                if (c < ncell) jb = task_block(c >> lg, row);
                const int cell = (jb << lg) + (c & (B - 1));
                const bool ok = jb >= 0 && cell < d.n_r;
                tk[u] = ok ? (c >> lg) : -1;
                rw[u] = row;
                ce[u] = jb >= 0 ? jb : 0;
                ii[u] = ok ? row * d.n_r + cell : 0;  // theta-major index
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) vv[u] = gld(d.acc + ii[u]);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (tk[u] < 0) continue;
                const int cell = ii[u] - rw[u] * d.n_r;
                if (suppressed(rw[u], cell)) continue;
                unsigned long long* dst = two_buf ? &snew[tk[u]] : &s_keys[rw[u] * d.nbr + ce[u]];
                atomicMax(dst, make_key(vv[u], (uint32_t)ii[u]));
            }
        }
        __syncthreads();
        // group keys of the touched blocks (two-buffer path: a touched
        // block's new key is read from s_new and copied into s_keys)
        const int ngt = all_rows ? n_groups : ntask;
        for (int task = wave; task < ngt; task += nwaves) {
            int g;
            if (all_rows) {
                g = task;
            } else {
                int row;
                const int jb = task_block(task, row);
                if (jb < 0) continue;  // the same in every lane
                g = (row * d.nbr + jb) >> kGroupLog2;
            }
            const int b = (g << kGroupLog2) + (lane & 31);
            unsigned long long v = 0;
            int tb = -1;
            if (lane < 32 && b < d.n_blocks) {
                if (two_buf) {
                    const int brow = b / d.nbr;
                    tb = block_task(brow, b - brow * d.nbr);
                }
                v = tb >= 0 ? snew[tb] : s_keys[b];
            }
            const unsigned long long gm = wave_max_u64(v);
            if (lane == 0) s_gkey[g] = gm;
            if (tb >= 0) s_keys[b] = v;
        }
        __syncthreads();
    }
    return found;
}

__device__ void peaks_select(const PeaksDesc& d) {
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid >> 6, nwaves = blockDim.x >> 6;
    const int nthreads = blockDim.x;
    const int floor_votes = d.min_votes > 1 ? d.min_votes : 1;
    // block keys into LDS, eight loads in flight per thread (indices are
    // clamped so every load is in bounds and none waits on a branch), and
    // the largest block count
    int vmax = INT_MIN;
    for (int b0 = tid; b0 < d.n_blocks; b0 += 8 * nthreads) {
        unsigned long long v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = gld(d.keys + min(b0 + u * nthreads, d.n_blocks - 1));
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (b0 + u * nthreads < d.n_blocks) {
                s_keys[b0 + u * nthreads] = v[u];
                if (v[u] != 0ull) vmax = max(vmax, key_value(v[u]));
            }
        }
    }
    vmax = wave_max_i32(vmax);
    if (lane == 0) s_wv[wave] = vmax;
    for (int q = tid; q < 256; q += nthreads) s_hist[q] = 0;
    if (tid == 0) {
        s_nsel = 0;
        s_ncand = 0;
    }
    __syncthreads();
    vmax = wave_max_i32(lane < nwaves ? s_wv[lane] : INT_MIN);
    int found = 0;
    if (vmax >= floor_votes) {  // else no cell reaches the floor
        found = peaks_candidates(d, floor_votes, vmax);
        if (found < 0) found = peaks_general(d, floor_votes);
    }
    __syncthreads();
    for (int j = found + tid; j < d.k; j += nthreads) {
        d.theta_idx[j] = -1;
        d.r_idx[j] = -1;
        d.votes[j] = -1;
    }
    if (tid == 0) *d.count = found;
}

__global__ void __launch_bounds__(1024) k_peaks_select(PeaksDesc d) { peaks_select(d); }

__global__ void __launch_bounds__(1024) k_peaks_select_batch(const PeaksDesc* __restrict__ descs,
                                                             int n_frames) {
    for (int f = blockIdx.x; f < n_frames; f += gridDim.x) {
        const PeaksDesc d = descs[f];
        if (!frame_on(d.active)) continue;
        peaks_select(d);
        __syncthreads();
    }
}

}  // namespace lane

using namespace lane;

extern "C" LANE_INTERNAL hipError_t lane_launch_peaks(const PeaksDesc* dp, hipStream_t s) {
    const PeaksDesc& d = *dp;
    hipLaunchKernelGGL(k_block_keys, dim3((d.n_blocks + 3) / 4), dim3(256), 0, s, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_peaks_select, dim3(1), dim3(1024), 0, s, d);
    return hipGetLastError();
}

extern "C" LANE_INTERNAL hipError_t lane_launch_peaks_batch(const PeaksDesc* descs, const int* list,
                                                            const int* counts, int n_frames, int grid_keys,
                                                            int grid_select, hipStream_t s) {
    if (grid_keys > 0) {  // 0: the vote already wrote the keys
        hipLaunchKernelGGL(k_block_keys_batch, dim3(grid_keys), dim3(256), 0, s, descs, list, counts);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_peaks_select_batch, dim3(grid_select), dim3(1024), 0, s, descs, n_frames);
    return hipGetLastError();
}
