// Pruned edge lists for a split vote with a tile mask (batched plans).
//
// What is computed: the masked vote (Sec. 2.3 Eq. (3) with every 8x8 tile
// voting only the theta rows whose band bits meet its mask byte: 0 = none,
// 0xFF = every row), the same accumulator as the masked vote kernel.
//
// Design.  The masked vote scans the tile masks of every segment in every
// theta slice; when few tiles are kept that scan, not the voting, sets its
// time.  Here one pass per frame copies the entries of the tiles that vote
// every row (mask 0xFF) to the front of their segment in a second list of
// the same layout, which the vote then streams like an unmasked list, and
// the entries of band-restricted tiles (any other non-zero mask) to the back
// of the segment's slot, which the vote reads after them with the band test
// entry by entry (few entries: the proposal network restricts few tiles).
#include "lane_entry.h"

namespace lane {

constexpr int kPruneWaves = 4;  // a workgroup per segment, its waves on interleaved chunks

__global__ void __launch_bounds__(kWave * kPruneWaves) k_prune_lists(const PruneDesc* __restrict__ descs) {
    const PruneDesc d = descs[blockIdx.y];
    if (!frame_on(d.active)) return;
    __shared__ int s_delta[kPruneWaves][kTilesPerChunk];
    const ListLayout L = list_layout(d.W, d.H);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
    for (int seg = blockIdx.x; seg < L.nseg; seg += gridDim.x) {
        const int ty = seg / L.nchunk, chunk = seg - ty * L.nchunk;
        const int tx0 = chunk * kTilesPerChunk;
        const int ntx = min(L.tw - tx0, kTilesPerChunk);
        const uint32_t* info = d.list + L.off_info + (size_t)ty * L.tw + tx0;
        const uint8_t* mrow = d.tile_mask + (size_t)ty * L.tw + tx0;
        // tiles lane and 64 + lane: entry count and start in the segment
        // (info = count << 16 | start), mask byte
        int cnt[2], start[2], fc[2], rc[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int t = h * kWave + lane;
            const bool ok = t < ntx;
            const uint32_t inf = ok ? gld(info + t) : 0u;
            const int m = ok ? (int)gld(mrow + t) : 0;
            cnt[h] = (int)(inf >> 16);
            start[h] = (int)(inf & 0xFFFFu);
            fc[h] = m == 0xFF ? cnt[h] : 0;
            rc[h] = (m != 0 && m != 0xFF) ? cnt[h] : 0;
        }
        // exclusive prefix sums in tile order (tiles 0..63, then 64..127)
        int fpre[2], rpre[2], ftot = 0, rtot = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            int fi = fc[h], ri = rc[h];
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const int a = __shfl_up(fi, o), b = __shfl_up(ri, o);
                if (lane >= o) {
                    fi += a;
                    ri += b;
                }
            }
            fpre[h] = ftot + fi - fc[h];
            rpre[h] = rtot + ri - rc[h];
            ftot += __shfl(fi, kWave - 1);
            rtot += __shfl(ri, kWave - 1);
        }
        // per tile: destination minus source position (full tiles to the
        // front, restricted ones to the back of the slot), INT_MIN: dropped
#pragma unroll
        for (int h = 0; h < 2; ++h)
            s_delta[wave][h * kWave + lane] = fc[h] ? fpre[h] - start[h]
                                              : rc[h] ? (kSegCap - rtot + rpre[h]) - start[h]
                                                      : INT_MIN;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // the entries, eight loads per lane in flight, chunks of 512 taken
        // by the waves in turn (every wave has worked out the same table);
        // an entry's tile is its x / 8 (entries of a segment lie in its own
        // tiles)
        const int n = min((int)gld(d.list + seg), kSegCap);
        const uint32_t* src = d.list + L.off_ent + (size_t)seg * kSegCap;
        uint32_t* dst = d.pruned + L.off_ent + (size_t)seg * kSegCap;
        for (int p0 = wave * 8 * kWave; p0 < n; p0 += kPruneWaves * 8 * kWave) {
            uint32_t e[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) e[u] = gld(src + min(p0 + u * kWave + lane, n - 1));
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int p = p0 + u * kWave + lane;
                if (p >= n) continue;
                const int t = min(max((int)((e[u] & 0xFFFFu) >> 3) - tx0, 0), kTilesPerChunk - 1);
                const int dl = s_delta[wave][t];
                // (a list not written by the Sobel pass could place an entry
                // outside its tile's range: such a position is not written)
                if (dl != INT_MIN && (unsigned)(p + dl) < (unsigned)kSegCap) gst(dst + p + dl, e[u]);
            }
        }
        if (wave == 0 && lane == 0) {
            gst(d.pruned + seg, (uint32_t)ftot);
            gst(d.pruned + L.off_info + seg, (uint32_t)rtot);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

}  // namespace lane

using namespace lane;

// grid: segments (max over the frames, at most 4096) x frames
extern "C" LANE_INTERNAL hipError_t lane_launch_prune_batch(const PruneDesc* descs, int n, int max_nseg,
                                                           hipStream_t s) {
    const int gx = max(1, min(max_nseg, 4096));
    hipLaunchKernelGGL(k_prune_lists, dim3(gx, n), dim3(kWave * kPruneWaves), 0, s, descs);
    return hipGetLastError();
}
