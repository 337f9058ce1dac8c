// Peak search without a caller workspace: the block keys of lane_hough_peaks
// live in a fixed device array of this library (one copy per GPU), so the
// call allocates nothing and takes no workspace argument.
//
// The array's host-side name is only a stand-in for the symbol: kernels get
// the device address that hipGetSymbolAddress returns for the current device,
// looked up once per device on the first call there and kept.
#include <mutex>
#include <string.h>

#include "lane_entry.h"

using namespace lane;


namespace {

// One key per block; the peak search never uses more than kPeaksMaxBlocksLds
// blocks (the block size grows until the count fits), i.e. 64 KiB.
constexpr size_t kScratchBytes = (size_t)kPeaksMaxBlocksLds * sizeof(unsigned long long);
static __device__ __align__(256) unsigned long long scratch[kPeaksMaxBlocksLds];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices];  // device address of `scratch` on each device, once looked up

// The device address of this device's copy of `scratch`, or null on error.
void* scratch_on(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

}  // namespace

extern "C" {

size_t lane_hough_peaks_noalloc_max_bytes(void) { return kScratchBytes; }

int lane_hough_peaks_noalloc(const int32_t* acc, int32_t n_theta, int32_t n_r, int32_t r_offset,
                             int32_t k, int32_t h_theta, int32_t h_r, int32_t min_votes,
                             int32_t* theta_idx, int32_t* r_idx, int32_t* votes, int32_t* count,
                             void* stream) {
    PeaksDesc d;
    size_t need = 0;
    const int st = lane_peaks_prepare(acc, n_theta, n_r, r_offset, k, h_theta, h_r, min_votes,
                                      theta_idx, r_idx, votes, count, &d, &need);
    if (st != LANE_OK) return st;
    if (need > kScratchBytes) return LANE_E_WS;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return LANE_E_DEVICE;
    void* p = scratch_on(dev);
    if (!p) return LANE_E_DEVICE;
    // Every block key is written by the key pass before the selection reads
    // it, so nothing left by an earlier call needs clearing.
    d.keys = (unsigned long long*)p;
    return lane_launch_peaks(&d, (hipStream_t)stream) == hipSuccess ? LANE_OK : LANE_E_DEVICE;
}

}  // extern "C"
