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
// new window are rescanned (skipping every suppressed cell), so a round
// costs O(window) instead of a pass over the accumulator.
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
        block_key(d, gb - prefix[lo], threadIdx.x & (kWave - 1));
    }
}

__shared__ unsigned long long s_keys[kPeaksMaxBlocksLds];
__shared__ uint32_t s_mark[kPeaksMaxBlocksLds / 32];
__shared__ int s_list[kPeaksMaxBlocksLds];
__shared__ int s_nlist;
__shared__ int s_sel_t[1024], s_sel_i[1024];
__shared__ unsigned long long s_red[16];
__shared__ int s_found, s_stop;

__device__ void peaks_select(const PeaksDesc& d) {
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid >> 6, nwaves = blockDim.x >> 6;
    const int floor_votes = d.min_votes > 1 ? d.min_votes : 1;
    for (int b = tid; b < d.n_blocks; b += blockDim.x) s_keys[b] = gld(d.keys + b);
    if (tid == 0) {
        s_found = 0;
        s_stop = 0;
    }
    __syncthreads();
    for (int j = 0; j < d.k; ++j) {
        unsigned long long best = 0;
        for (int b = tid; b < d.n_blocks; b += blockDim.x) best = s_keys[b] > best ? s_keys[b] : best;
        best = wave_max_u64(best);
        if (lane == 0) s_red[wave] = best;
        __syncthreads();
        if (tid == 0) {
            unsigned long long m = 0;
            for (int w = 0; w < nwaves; ++w) m = s_red[w] > m ? s_red[w] : m;
            const int v = key_value(m);
            if (m == 0 || v < floor_votes) {
                s_stop = 1;
            } else {
                const uint32_t idx = key_index(m);
                const int t = (int)(idx / (uint32_t)d.n_r), i = (int)(idx % (uint32_t)d.n_r);
                d.theta_idx[j] = t;
                d.r_idx[j] = i;
                d.votes[j] = v;
                s_sel_t[j] = t;
                s_sel_i[j] = i;
                s_found = j + 1;
                // mark the blocks the new window touches
                for (int w = 0; w < (d.n_blocks + 31) / 32; ++w) s_mark[w] = 0;
                for (int dt = -d.h_theta; dt <= d.h_theta; ++dt) {
                    const int traw = t + dt;
                    const int q = floor_div_i(traw, d.n_theta);
                    const int row = traw - q * d.n_theta;
                    const int centre = (q & 1) ? 2 * d.r_offset - i : i;
                    const int ca = max(0, centre - d.h_r), cb = min(d.n_r - 1, centre + d.h_r);
                    if (ca > cb) continue;
                    for (int b = row * d.nbr + (ca >> d.block_log2); b <= row * d.nbr + (cb >> d.block_log2); ++b)
                        s_mark[b >> 5] |= 1u << (b & 31);
                }
                int n = 0;
                for (int w = 0; w < (d.n_blocks + 31) / 32; ++w) {
                    uint32_t bits = s_mark[w];
                    while (bits) {
                        const int bit = __ffs(bits) - 1;
                        bits &= bits - 1;
                        s_list[n++] = w * 32 + bit;
                    }
                }
                s_nlist = n;
            }
        }
        __syncthreads();
        if (s_stop) break;
        // rescan the touched blocks, skipping cells inside any selected window
        const int nsel = j + 1;
        for (int li = wave; li < s_nlist; li += nwaves) {
            const int b = s_list[li];
            const int t = b / d.nbr, jb = b - t * d.nbr;
            const int i0 = jb << d.block_log2, i1 = min(d.n_r, i0 + (1 << d.block_log2));
            const uint32_t rowc = (uint32_t)t * (uint32_t)d.n_r;
            unsigned long long bk = 0;
            for (int i = i0 + lane; i < i1; i += kWave) {
                bool sup = false;
                for (int p = 0; p < nsel && !sup; ++p) sup = in_window(t, i, s_sel_t[p], s_sel_i[p], d);
                if (!sup) {
                    const unsigned long long kk = make_key(gld(d.acc + rowc + i), rowc + (uint32_t)i);
                    bk = kk > bk ? kk : bk;
                }
            }
            bk = wave_max_u64(bk);
            if (lane == 0) s_keys[b] = bk;
        }
        __syncthreads();
    }
    __syncthreads();
    const int found = s_found;
    for (int j = found + tid; j < d.k; j += blockDim.x) {
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
