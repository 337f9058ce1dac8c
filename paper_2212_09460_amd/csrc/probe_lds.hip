// LDS atomic-increment rate of this GPU: the practical ceiling of the Hough
// vote, whose inner loop is one ds_add_u32 per (edge pixel, angle).
//
// k_lds_add: every lane adds 1 to its own LDS word at 16 constant offsets per
// step; the 64 lanes of a wave address 64 consecutive words, so no two lanes
// of an instruction share a bank (the conflict-free rate).
// k_lds_add_random: the same count of increments to hashed addresses spread
// over the workgroup's words (the bank pattern of votes from scattered
// pixels), for comparison.
// k_lds_add_vote: the vote's own instruction mix and bank pattern: 16 angle
// rows x 4 pixel slots per wave, each increment preceded by the vote's four
// VALU instructions (dot product, shift, shift-or for the address, and-or
// for the increment) into 16-row interleaved pairs of 14-bit counters; the
// rate a vote can reach when nothing else (loads, set-up, write-out) costs
// anything.
//
// Built into its own library (liblaneprobe.so): it is a measurement, not part
// of the lane-detection path.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 1024;
constexpr int kUnroll = 16;
constexpr int kWords = kThreads * kUnroll;  // 64 KB of counters per workgroup

__global__ void __launch_bounds__(kThreads) k_lds_add(uint32_t* __restrict__ out, int steps) {
    __shared__ uint32_t s[kWords];
    const int t = threadIdx.x;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) s[t + u * kThreads] = 0;
    __syncthreads();
    for (int i = 0; i < steps; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) atomicAdd(&s[t + u * kThreads], 1u);
    }
    __syncthreads();
    uint32_t sum = 0;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) sum += s[t + u * kThreads];
    out[(size_t)blockIdx.x * kThreads + t] = sum;
}

__global__ void __launch_bounds__(kThreads) k_lds_add_random(uint32_t* __restrict__ out, int steps) {
    __shared__ uint32_t s[kWords];
    const int t = threadIdx.x;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) s[t + u * kThreads] = 0;
    __syncthreads();
    uint32_t h = (uint32_t)t * 0x9E3779B9u + blockIdx.x;
    for (int i = 0; i < steps; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            h = h * 1664525u + 1013904223u;  // LCG: a different word each time
            atomicAdd(&s[h >> 18], 1u);      // top 14 bits: [0, 16384)
        }
    }
    __syncthreads();
    uint32_t sum = 0;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) sum += s[t + u * kThreads];
    out[(size_t)blockIdx.x * kThreads + t] = sum;
}

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// inc_mask is zero at run time (every increment is 1, so the counters can be
// checked) but unknown to the compiler, which keeps the and-or.
__global__ void __launch_bounds__(kThreads) k_lds_add_vote(uint32_t* __restrict__ out, int steps, uint32_t inc_mask) {
    __shared__ uint32_t s[kWords];
    const int t = threadIdx.x, lane = t & 63, j = lane & 15, slot = lane >> 4;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) s[t + u * kThreads] = 0;
    __syncthreads();
    // row j: angle (blockIdx.x * 7 % 164 + j) / 2 degrees, in [0, 90): C, S >= 0
    const float th = (float)((blockIdx.x * 7u) % 164u + (uint32_t)j) * (3.14159265f / 360.f);
    const int C = (int)(16384.f * cosf(th) + 0.5f), S = (int)(16384.f * sinf(th) + 0.5f);
    const int CS = (int)(((uint32_t)(uint16_t)S << 16) | (uint32_t)(uint16_t)C);
    // one pixel per slot and unroll step (x, y < 512), shared by the slot's 16 rows
    uint32_t xy[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const uint32_t h = mix32(((blockIdx.x * 16u + (uint32_t)(t >> 6)) * 4u + (uint32_t)slot) * 16u + (uint32_t)u);
        xy[u] = ((h >> 16) & 511u) << 16 | (h & 511u);
    }
    const uint32_t jb = 4u * (uint32_t)j;
    for (int i = 0; i < steps; ++i) {
        const int K = (int)(((uint32_t)i * 2654435761u) >> 8);  // < 2^24: pairs stay below 1024
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            int v;
            asm volatile("v_dot2_i32_i16 %0, %1, %2, %3" : "=v"(v) : "v"((int)xy[u]), "v"(CS), "v"(K));
            const uint32_t adr = (((uint32_t)v >> 15) << 6) | jb;  // pair * 16 rows * 4 B + row
            const uint32_t inc = ((uint32_t)v & inc_mask) | 1u;
            atomicAdd(reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(s) + adr), inc);
        }
    }
    __syncthreads();
    uint32_t sum = 0;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) sum += s[t + u * kThreads];
    out[(size_t)blockIdx.x * kThreads + t] = sum;
}

}  // namespace

extern "C" {

// Runs `groups` workgroups of 1024 threads, each doing `steps` x 16 LDS
// increments per thread (random = 0: conflict-free; 1: hashed addresses;
// 2: the vote's pattern and instruction mix),
// timed with HIP events on a stream of its own after one untimed launch.
// *adds_per_s receives increments per second; *checksum the number of
// increments the counters hold (for the caller to compare with
// groups * 1024 * 16 * steps).  Returns 0, or -1 on a bad argument or a HIP
// error.
int lane_probe_lds_add(int32_t groups, int32_t steps, int32_t random, double* adds_per_s,
                       uint64_t* checksum) {
    if (groups < 1 || groups > 65536 || steps < 1 || steps > (1 << 20) || random < 0 || random > 2 ||
        !adds_per_s || !checksum)
        return -1;
    uint32_t* out = nullptr;
    const size_t n = (size_t)groups * kThreads;
    if (hipMalloc(&out, n * sizeof(uint32_t)) != hipSuccess) return -1;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = -1;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
        hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        auto launch = [&]() {
            if (random == 2)
                hipLaunchKernelGGL(k_lds_add_vote, dim3(groups), dim3(kThreads), 0, st, out, steps, 0u);
            else if (random)
                hipLaunchKernelGGL(k_lds_add_random, dim3(groups), dim3(kThreads), 0, st, out, steps);
            else
                hipLaunchKernelGGL(k_lds_add, dim3(groups), dim3(kThreads), 0, st, out, steps);
        };
        launch();
        hipEventRecord(e0, st);
        launch();
        hipEventRecord(e1, st);
        float ms = 0.f;
        if (hipGetLastError() == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
            hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.f) {
            uint32_t* h = new uint32_t[n];
            if (hipMemcpy(h, out, n * sizeof(uint32_t), hipMemcpyDeviceToHost) == hipSuccess) {
                uint64_t sum = 0;
                for (size_t i = 0; i < n; ++i) sum += h[i];
                *checksum = sum;
                *adds_per_s = (double)n * kUnroll * (double)steps / (ms * 1e-3);
                rc = 0;
            }
            delete[] h;
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (st) hipStreamDestroy(st);
    hipFree(out);
    return rc;
}

}  // extern "C"
