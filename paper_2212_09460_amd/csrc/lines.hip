// Line segments along Hough peaks (the lane lines drawn from the peaks:
// Sec. 1 step 4, Sec. 5 "Hough lines"; the paper leaves this step to MATLAB
// and gives no algorithm, so what is computed is this library's definition):
//
//   points of peak (t, i): the 255 pixels whose vote for bin t lands in cell
//     i, i.e. floor((x C[t] + y S[t] + 2^13) / 2^14) + r_offset == i;
//   order: by (y, x) when |C[t]| >= |S[t]| (the line is nearer the
//     vertical), else by (x, y);
//   split: consecutive points more than fill_gap apart start a new segment;
//   keep: segments whose end points are at least min_length apart.
//
// One workgroup per peak.  Instead of searching the edge list, the
// workgroup walks the line's main axis (rows when |C| >= |S|, else
// columns): for each step m, the cross coordinates o with the right cell
// satisfy o*A in [r*2^14 - 2^13 - m*B, r*2^14 + 2^13 - m*B), A the larger of
// |C|, |S| (>= 2^14 / sqrt(2)), so at most two integers, found by testing the
// few candidates around the interval with the exact integer formula and
// reading the edge map there.  Walking in order of m and ascending o yields
// the points already sorted; a workgroup prefix sum places them in LDS.  A
// second pass marks segment starts (squared gap > fill_gap^2), a third keeps
// the segments whose squared length reaches min_length^2, each compacted by
// prefix sums so the output order is the line order.
#include "lane_entry.h"

namespace lane {

constexpr int kLinesThreads = 256;
// A cell's voters: at most two per step of the walked axis (|A| >= 2^14/sqrt 2),
// so a frame with longer side L needs room for 2L points (lines_lds_bytes).

__device__ __forceinline__ int floor_div_i(int a, int b) {  // b != 0, any signs
    int q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
    return q;
}

// Exclusive prefix sum over the workgroup (256 threads = 4 waves); returns
// this thread's offset and writes the total to *total.
__device__ __forceinline__ int block_excl_scan(int v, int* s_wave, int* total) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int t = __shfl_up(incl, o);
        if (lane >= o) incl += t;
    }
    if (lane == kWave - 1) s_wave[wave] = incl;
    __syncthreads();
    int base = 0, sum = 0;
#pragma unroll
    for (int w = 0; w < kLinesThreads / kWave; ++w) {
        const int t = s_wave[w];
        base += w < wave ? t : 0;
        sum += t;
    }
    __syncthreads();  // s_wave is reused by the next scan
    *total = sum;
    return base + incl - v;
}

__device__ __forceinline__ long long dist2(uint32_t p, uint32_t q) {
    const long long dx = (long long)(int)(p & 0xFFFFu) - (long long)(int)(q & 0xFFFFu);
    const long long dy = (long long)(int)(p >> 16) - (long long)(int)(q >> 16);
    return dx * dx + dy * dy;
}

// Peak j of frame d; s_pts / s_start hold 2 * max(W, H) entries.
__device__ void lines_item(const LinesDesc& d, int j, uint32_t* s_pts, uint16_t* s_start, int* s_wave) {
    const int tid = threadIdx.x;
    int32_t* out = d.segs + (size_t)j * d.max_seg * 4;
    for (int s = tid; s < 4 * d.max_seg; s += kLinesThreads) gst(out + s, -1);

    const int t = gld(d.theta_idx + j);
    const int i = gld(d.r_idx + j);
    const int n_peaks = d.count ? gld(d.count) : d.k;
    const int n_r = 2 * d.r_offset + 1;
    if (j >= n_peaks || t < 0 || t >= d.n_theta || i < 0 || i >= n_r) {
        if (tid == 0) {
            gst(d.seg_count + j, 0);
            if (d.npts) gst(d.npts + j, 0);
        }
        return;  // whole workgroup leaves together
    }
    const int C = gld(d.cos_q14 + t), S = gld(d.sin_q14 + t);
    const int r = i - d.r_offset;
    const bool by_y = (C < 0 ? -C : C) >= (S < 0 ? -S : S);
    const int A = by_y ? C : S, B = by_y ? S : C;
    // a row of a rotation table has max(|C|, |S|) >= round(2^14 / sqrt 2);
    // any other row is refused (count -1).  |r| above 2^14 + 1 cannot be
    // reached from inside an 8192 x 8192 frame: no points.
    const bool table_ok = (A < 0 ? -A : A) >= 11585;
    if (!table_ok || r > 16385 || r < -16385) {
        if (tid == 0) {
            gst(d.seg_count + j, table_ok ? 0 : -1);
            if (d.npts) gst(d.npts + j, 0);
        }
        return;
    }
    const int L = by_y ? d.H : d.W;                // walked axis
    const int Lo = by_y ? d.W : d.H;               // cross axis

    // candidates o of step m: o*A in [lo, lo + 2^14), lo = r*2^14 - 2^13 - m*B;
    // every solution lies in [min(q1,q2), max(q1,q2) + 1], q = floor(. / A)
    auto visit = [&](int m, auto&& emit) {
        const int lo = r * 16384 - 8192 - m * B;
        const int q1 = floor_div_i(lo, A), q2 = floor_div_i(lo + 16384, A);
        const int o0 = min(q1, q2) - 1, o1 = max(q1, q2) + 1;
        for (int o = max(o0, 0); o <= min(o1, Lo - 1); ++o) {
            const int x = by_y ? o : m, y = by_y ? m : o;
            if (((x * C + y * S + 8192) >> 14) != r) continue;
            if (gld(d.edges + (size_t)y * d.W + x) != 255) continue;
            emit(x, y);
        }
    };

    // pass 1: points per thread over a contiguous range of steps
    const int per = (L + kLinesThreads - 1) / kLinesThreads;
    const int m0 = min(tid * per, L), m1 = min(m0 + per, L);
    int n_mine = 0;
    for (int m = m0; m < m1; ++m) visit(m, [&](int, int) { ++n_mine; });
    int total = 0;
    int pos = block_excl_scan(n_mine, s_wave, &total);
    for (int m = m0; m < m1; ++m)
        visit(m, [&](int x, int y) { s_pts[pos++] = (uint32_t)x | ((uint32_t)y << 16); });
    __syncthreads();
    if (tid == 0 && d.npts) gst(d.npts + j, total);

    // pass 2: segment starts (first point, or a gap above fill_gap)
    const long long gap2 = (long long)d.fill_gap * d.fill_gap;
    const long long len2 = (long long)d.min_length * d.min_length;
    const int pp = (total + kLinesThreads - 1) / kLinesThreads;
    const int p0 = min(tid * pp, total), p1 = min(p0 + pp, total);
    int n_starts = 0;
    for (int p = p0; p < p1; ++p) n_starts += (p == 0 || dist2(s_pts[p - 1], s_pts[p]) > gap2);
    int n_seg = 0;
    int sid = block_excl_scan(n_starts, s_wave, &n_seg);
    for (int p = p0; p < p1; ++p)
        if (p == 0 || dist2(s_pts[p - 1], s_pts[p]) > gap2) s_start[sid++] = (uint16_t)p;
    __syncthreads();

    // pass 3: keep segments whose end points are min_length apart, in order
    const int ps = (n_seg + kLinesThreads - 1) / kLinesThreads;
    const int s0 = min(tid * ps, n_seg), s1 = min(s0 + ps, n_seg);
    auto seg_end = [&](int s) { return (s + 1 < n_seg ? (int)s_start[s + 1] : total) - 1; };
    int n_keep = 0;
    for (int s = s0; s < s1; ++s) n_keep += dist2(s_pts[s_start[s]], s_pts[seg_end(s)]) >= len2;
    int kept_total = 0;
    int slot = block_excl_scan(n_keep, s_wave, &kept_total);
    for (int s = s0; s < s1; ++s) {
        const uint32_t a = s_pts[s_start[s]], b = s_pts[seg_end(s)];
        if (dist2(a, b) < len2) continue;
        if (slot < d.max_seg) {
            int32_t* o = out + (size_t)slot * 4;
            gst(o + 0, (int32_t)(a & 0xFFFFu));
            gst(o + 1, (int32_t)(a >> 16));
            gst(o + 2, (int32_t)(b & 0xFFFFu));
            gst(o + 3, (int32_t)(b >> 16));
        }
        ++slot;
    }
    if (tid == 0) gst(d.seg_count + j, kept_total);
}

__global__ void __launch_bounds__(kLinesThreads) k_lines(LinesDesc d, int cap) {
    extern __shared__ __align__(16) uint32_t s_dyn[];
    __shared__ int s_wave[kLinesThreads / kWave];
    lines_item(d, blockIdx.x, s_dyn, (uint16_t*)(s_dyn + cap), s_wave);
}

// Batched: blockIdx.y = frame (a frame switched off keeps its outputs),
// blockIdx.x = peak.
__global__ void __launch_bounds__(kLinesThreads) k_lines_batch(const LinesDesc* __restrict__ descs, int cap) {
    extern __shared__ __align__(16) uint32_t s_dyn[];
    __shared__ int s_wave[kLinesThreads / kWave];
    const LinesDesc d = descs[blockIdx.y];
    if ((int)blockIdx.x >= d.k || !frame_on(d.active)) return;
    lines_item(d, blockIdx.x, s_dyn, (uint16_t*)(s_dyn + cap), s_wave);
}

}  // namespace lane

using namespace lane;

extern "C" LANE_INTERNAL hipError_t lane_launch_lines(const uint8_t* edges, int W, int H, const int16_t* C,
                                                      const int16_t* S, int n_theta, int r_offset,
                                                      const int32_t* theta_idx, const int32_t* r_idx,
                                                      const int32_t* count, int k, int fill_gap,
                                                      int min_length, int max_seg, int32_t* segs,
                                                      int32_t* seg_count, int32_t* npts, hipStream_t s) {
    LinesDesc d;
    d.edges = edges;
    d.W = W;
    d.H = H;
    d.cos_q14 = C;
    d.sin_q14 = S;
    d.n_theta = n_theta;
    d.r_offset = r_offset;
    d.theta_idx = theta_idx;
    d.r_idx = r_idx;
    d.count = count;
    d.k = k;
    d.fill_gap = fill_gap;
    d.min_length = min_length;
    d.max_seg = max_seg;
    d.segs = segs;
    d.seg_count = seg_count;
    d.npts = npts;
    d.active = nullptr;
    const int cap = 2 * (W > H ? W : H);
    hipLaunchKernelGGL(k_lines, dim3(k), dim3(kLinesThreads), lines_lds_bytes(W, H), s, d, cap);
    return hipGetLastError();
}

extern "C" LANE_INTERNAL hipError_t lane_launch_lines_batch(const LinesDesc* descs, int n, int max_k,
                                                            int max_side, hipStream_t s) {
    const int cap = 2 * max_side;
    hipLaunchKernelGGL(k_lines_batch, dim3(max_k, n), dim3(kLinesThreads), (size_t)6 * cap, s, descs, cap);
    return hipGetLastError();
}
