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
// smallest index".  Pass 2 (one workgroup per frame): the block keys sit in
// LDS; each round is one block-wide max, and only the blocks touched by the
// new window are rescanned (skipping every suppressed cell), the cells of
// all touched blocks spread over the whole workgroup with their loads
// issued together, so a round costs O(window) and one memory round trip
// instead of a pass over the accumulator.
#include "lane_internal.h"

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

// Batched: wave-granular grid stride over all blocks of all frames; the frame
// of a global block index is found by binary search in the prefix table.
__global__ void __launch_bounds__(256) k_block_keys_batch(const PeaksDesc* __restrict__ descs,
                                                          const int* __restrict__ prefix, int n_frames) {
    const int total = prefix[n_frames];
    for (int gb = blockIdx.x * 4 + (threadIdx.x >> 6); gb < total; gb += gridDim.x * 4) {
        int lo = 0, hi = n_frames - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= gb) lo = mid;
            else hi = mid - 1;
        }
        const PeaksDesc d = descs[lo];
        if (!frame_on(d.active)) continue;
        block_key(d, gb - prefix[lo], threadIdx.x & (kWave - 1));
    }
}

__shared__ unsigned long long s_keys[kPeaksMaxBlocksLds];
__shared__ int s_tb[kPeaksMaxBlocksLds];  // rescan task -> (row | block column << 13), -1 if none
constexpr int kIvTasks = 1024, kIvMax = 4;
__shared__ uint32_t s_iv[kIvTasks][kIvMax];  // suppressed column ranges of a task's row (lo | hi << 16)
__shared__ int s_niv[kIvTasks];
__shared__ int s_sel_t[1024], s_sel_i[1024];
__shared__ unsigned long long s_red[16];

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

__device__ void peaks_select(const PeaksDesc& d) {
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid >> 6, nwaves = blockDim.x >> 6;
    const int nthreads = blockDim.x;
    const int floor_votes = d.min_votes > 1 ? d.min_votes : 1;
    // block keys into LDS, eight loads in flight per thread (indices are
    // clamped so every load is in bounds and none waits on a branch)
    for (int b0 = tid; b0 < d.n_blocks; b0 += 8 * nthreads) {
        unsigned long long v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = gld(d.keys + min(b0 + u * nthreads, d.n_blocks - 1));
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (b0 + u * nthreads < d.n_blocks) s_keys[b0 + u * nthreads] = v[u];
    }
    __syncthreads();
    // blocks a window can touch: 2 h_theta + 1 rows (all blocks when the
    // rows would repeat), each a contiguous column range of at most nbw
    // blocks; at most n_blocks tasks either way
    const bool all_rows = 2 * d.h_theta + 1 > d.n_theta;
    const int nbw = min(d.nbr, ((2 * d.h_r) >> d.block_log2) + 2);
    const int ntask = all_rows ? d.n_blocks : (2 * d.h_theta + 1) * nbw;
    // per-row suppressed ranges replace the per-cell window tests when the
    // windows do not wrap more than once and the tasks are few
    const bool use_iv = !all_rows && ntask <= kIvTasks && d.n_r <= 0xFFFF;
    const int lg = d.block_log2, B = 1 << lg;
    int found = 0;
    for (int j = 0; j < d.k; ++j) {
        unsigned long long best = 0;
        for (int b = tid; b < d.n_blocks; b += nthreads) best = s_keys[b] > best ? s_keys[b] : best;
        best = wave_max_u64(best);
        if (lane == 0) s_red[wave] = best;
        __syncthreads();
        unsigned long long m = 0;
        for (int w = 0; w < nwaves; ++w) m = s_red[w] > m ? s_red[w] : m;
        if (m == 0 || key_value(m) < floor_votes) break;  // the same decision in every thread
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
        __syncthreads();
        // tasks -> blocks (the touched blocks restart from the empty key) and,
        // per task row, the column ranges every selected window suppresses
        for (int task = tid; task < ntask; task += nthreads) {
            int row, jb;
            if (all_rows) {
                row = task / d.nbr;
                jb = task - row * d.nbr;
            } else {
                const int r = task / nbw, bi = task - r * nbw;
                const int traw = t - d.h_theta + r;
                const int q = floor_div_i(traw, d.n_theta);
                row = traw - q * d.n_theta;
                const int centre = (q & 1) ? 2 * d.r_offset - i : i;
                const int ca = max(0, centre - d.h_r), cb = min(d.n_r - 1, centre + d.h_r);
                jb = (ca > cb || (ca >> lg) + bi > (cb >> lg)) ? -1 : (ca >> lg) + bi;
            }
            s_tb[task] = jb < 0 ? -1 : (row | (jb << 13));
            if (jb >= 0) s_keys[row * d.nbr + jb] = 0;
            if (use_iv) {
                int n = 0;
                for (int p = 0; p <= j && n <= kIvMax; ++p) {
                    const int tp = s_sel_t[p], ip = s_sel_i[p];
                    const int mir = 2 * d.r_offset - ip;
                    int cs[3], nc = 0;
                    if (abs(row - tp) <= d.h_theta) cs[nc++] = ip;
                    if (row - d.n_theta >= tp - d.h_theta) cs[nc++] = mir;
                    if (row + d.n_theta <= tp + d.h_theta) cs[nc++] = mir;
                    for (int c = 0; c < nc; ++c) {
                        const int lo = max(0, cs[c] - d.h_r), hi = min(d.n_r - 1, cs[c] + d.h_r);
                        if (lo > hi) continue;
                        if (n < kIvMax) s_iv[task][n] = (uint32_t)lo | ((uint32_t)hi << 16);
                        ++n;
                    }
                }
                s_niv[task] = n;  // more than kIvMax: the cells of this task use the full test
            }
        }
        __syncthreads();
        // rescan: every thread takes cells of the touched blocks, all loads
        // of a group of eight first, then the suppression tests and an LDS max
        const int ncell = ntask << lg;
        for (int c0 = tid; c0 < ncell; c0 += 8 * nthreads) {
            int tk[8], ii[8], vv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int c = c0 + u * nthreads;
                const int e = c < ncell ? s_tb[c >> lg] : -1;
                const int row = e & 0x1FFF, cell = ((e >> 13) << lg) + (c & (B - 1));
                const bool ok = e >= 0 && cell < d.n_r;
                tk[u] = ok ? (c >> lg) : -1;
                ii[u] = ok ? row * d.n_r + cell : 0;  // theta-major index
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) vv[u] = gld(d.acc + ii[u]);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (tk[u] < 0) continue;
                const int e = s_tb[tk[u]];
                const int row = e & 0x1FFF, cell = ((e >> 13) << lg) + ((c0 + u * nthreads) & (B - 1));
                bool sup = false;
                const int niv = use_iv ? s_niv[tk[u]] : kIvMax + 1;
                if (niv <= kIvMax) {
                    for (int q = 0; q < niv; ++q) {
                        const uint32_t iv = s_iv[tk[u]][q];
                        sup |= cell >= (int)(iv & 0xFFFFu) && cell <= (int)(iv >> 16);
                    }
                } else {
                    for (int p = 0; p <= j && !sup; ++p)
                        sup = in_window_fast(row, cell, s_sel_t[p], s_sel_i[p], d);
                }
                if (!sup) atomicMax(&s_keys[row * d.nbr + (e >> 13)], make_key(vv[u], (uint32_t)ii[u]));
            }
        }
        __syncthreads();
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

extern "C" LANE_INTERNAL hipError_t lane_launch_peaks_batch(const PeaksDesc* descs, const int* prefix, int n_frames,
                                              int total_blocks, int grid_keys, int grid_select,
                                              hipStream_t s) {
    if (grid_keys > 0) {  // 0: the vote already wrote the keys
        hipLaunchKernelGGL(k_block_keys_batch, dim3(grid_keys), dim3(256), 0, s, descs, prefix, n_frames);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_peaks_select_batch, dim3(grid_select), dim3(1024), 0, s, descs, n_frames);
    return hipGetLastError();
}
