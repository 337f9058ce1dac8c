// Learned tile / theta-band proposal for gfx950: a 4-layer 3x3 CNN in FP16
// with FP32 accumulation on MFMA (forward: v_mfma_f32_16x16x16_f16 for
// conv1, v_mfma_f32_16x16x32_f16 for the 16-channel layers), its backward
// pass, BCE loss, Adam, plain-pipeline tile labels and the mask rule.
//
// Network (zero padding 1):  conv1 1->16 s2 ReLU, conv2 16->16 s2 ReLU,
// conv3 16->16 s2 ReLU, head 16->9 s1; input gray/255; output logits at 1/8
// resolution, channel 0 = keep logit of an 8x8 tile, 1..8 = theta bands.
//
// Layouts.  Activations are NHWC FP16 with 16 channels (32 B per pixel), so
// the 4 consecutive channels an MFMA lane supplies are one 8-byte load.
// Every convolution tile is one wave: 16 output pixels of a row x 16 output
// channels; forward, two kernel taps of 16 input channels per 16x16x32 MFMA
// (five per tile; conv1: K = the 9 taps of the single input channel, one
// 16x16x16 MFMA); backward, K = 16 per 16x16x16 MFMA, nine per tile.  With M = output channel and
// N = pixel the accumulator lane holds 4 consecutive channels of one pixel,
// which is again an 8-byte NHWC store.  Backward data swaps the roles of the
// channel axes (transposed weights); backward weights reduces over pixels
// (K = 16 pixels per MFMA) into per-wave partials that a fixed-order pass
// sums, so training is deterministic.
//
// Master parameters are FP32 in the flat order: for each layer the weights
// [c_out][c_in][3][3] then the biases [c_out] (6105 values).
#include <math.h>

#include <algorithm>
#include <string.h>

#include "lane_entry.h"

namespace lane {

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kCnnParams = 6105;
// offsets of each layer's weights and biases in the master vector
constexpr int kW1 = 0, kB1 = 144, kW2 = 160, kB2 = 2464, kW3 = 2480, kB3 = 4784, kW4 = 4800,
              kB4 = 6096;
// packed buffer: f32 biases [4][16], then f16 blocks
constexpr int kPkBias = 0;                 // floats
constexpr int kPkW1 = 0;                   // halves, after the biases: [16 co][16 tap]
constexpr int kPkBlock = 9 * 16 * 16;      // [tap][16][16]
constexpr int kPkW2 = 256, kPkW2T = kPkW2 + kPkBlock, kPkW3 = kPkW2T + kPkBlock,
              kPkW3T = kPkW3 + kPkBlock, kPkW4 = kPkW3T + kPkBlock, kPkW4T = kPkW4 + kPkBlock;
constexpr int kPkHalves = kPkW4T + kPkBlock;
constexpr size_t kPackedBytes = 4 * 16 * sizeof(float) + (size_t)kPkHalves * sizeof(_Float16);

__device__ __forceinline__ const _Float16* pk_h(const void* pk) {
    return reinterpret_cast<const _Float16*>(reinterpret_cast<const char*>(pk) + 4 * 16 * sizeof(float));
}
__device__ __forceinline__ const float* pk_bias(const void* pk, int layer) {
    return reinterpret_cast<const float*>(pk) + layer * 16;
}

__device__ __forceinline__ h4 ld_h4(const _Float16* p) { return *(const LANE_GLOBAL h4*)p; }
__device__ __forceinline__ void st_h4(_Float16* p, h4 v) { *(LANE_GLOBAL h4*)p = v; }

__device__ __forceinline__ f4 mfma16(h4 a, h4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

// gfx950's 16x16x32 FP16 MFMA: K = 32 per instruction (two taps of 16
// channels), each lane supplying 8 consecutive K values of A and of B
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ f4 mfma32(h8 a, h8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ pack --
// master f32 -> kernel layouts (f16): W[tap][co][ci], W^T[tap][ci][co],
// conv1 as [co][tap], biases f32 [layer][16]; unused slots are zero.
__global__ void k_cnn_pack(const float* __restrict__ m, void* __restrict__ pk) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float* bias = reinterpret_cast<float*>(pk);
    _Float16* h = reinterpret_cast<_Float16*>(reinterpret_cast<char*>(pk) + 4 * 16 * sizeof(float));
    if (i < 64) {
        const int l = i >> 4, co = i & 15;
        const int boff[4] = {kB1, kB2, kB3, kB4};
        const int cout = l == 3 ? 9 : 16;
        bias[i] = co < cout ? m[boff[l] + co] : 0.f;
    }
    if (i < 256) {  // conv1 [co][tap]
        const int co = i >> 4, tap = i & 15;
        h[kPkW1 + i] = (_Float16)(tap < 9 ? m[kW1 + co * 9 + tap] : 0.f);
    }
    if (i < 3 * 2 * kPkBlock) {
        const int which = i / kPkBlock, r = i % kPkBlock;  // which: layer-pair index
        const int l = 1 + (which >> 1), transposed = which & 1;
        const int tap = r >> 8, a = (r >> 4) & 15, b = r & 15;
        const int co = transposed ? b : a, ci = transposed ? a : b;
        const int woff[4] = {kW1, kW2, kW3, kW4};
        const int cout = l == 3 ? 9 : 16;
        const float v = co < cout ? m[woff[l] + (co * 16 + ci) * 9 + tap] : 0.f;
        h[kPkW2 + i] = (_Float16)v;
    }
}

// --------------------------------------------------------------- forward --
struct CnnFwd {
    const uint8_t* img;       // conv1 input, [B][H][pitch] with frame stride
    int W, H, pitch;
    long long img_stride;
    const void* pk;
    _Float16* a1;             // [B][H1][W1][16]
    _Float16* a2;
    _Float16* a3;
    float* logits;            // [B][9][H4][W4]
    int H1, W1, H2, W2, H3, W3;  // layer output sizes; head = (H3, W3)
    long long s1, s2, s3;     // per-frame strides in halves
    int batch;
    const uint8_t* active;    // frame b runs iff active[b] != 0 (null = all)
};

// conv1: K = the 9 taps of the one input channel
__global__ void __launch_bounds__(256) k_cnn_fwd1(CnnFwd p) {
    const int lane = threadIdx.x & 63;
    const int ntx = (p.W1 + 15) >> 4;
    const int item = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (item >= p.batch * p.H1 * ntx) return;
    const int b = item / (p.H1 * ntx), rem = item - b * p.H1 * ntx;
    if (p.active && gld(p.active + b) == 0) return;
    const int oy = rem / ntx, ox0 = (rem - (rem / ntx) * ntx) * 16;
    const int col = lane & 15, grp = lane >> 4;
    const _Float16* w = pk_h(p.pk) + kPkW1;
    const h4 A = ld_h4(w + col * 16 + 4 * grp);  // W1[co = col][tap = 4 grp + j]
    const int ox = ox0 + col;
    const uint8_t* img = p.img + (size_t)b * p.img_stride;
    h4 B;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int tap = 4 * grp + j;
        float v = 0.f;
        if (tap < 9 && ox < p.W1) {
            const int iy = 2 * oy + tap / 3 - 1, ix = 2 * ox + tap % 3 - 1;
            if (iy >= 0 && iy < p.H && ix >= 0 && ix < p.W)
                v = (float)gld(img + (size_t)iy * p.pitch + ix) * (1.0f / 255.0f);
        }
        B[j] = (_Float16)v;
    }
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma16(A, B, acc);
    if (ox < p.W1) {
        const float* bias = pk_bias(p.pk, 0);
        h4 o;
#pragma unroll
        for (int j = 0; j < 4; ++j) o[j] = (_Float16)fmaxf(acc[j] + bias[4 * grp + j], 0.f);
        st_h4(p.a1 + (size_t)b * p.s1 + ((size_t)oy * p.W1 + ox) * 16 + 4 * grp, o);
    }
}

// conv2 / conv3 / head: 16 input channels, 9 taps as five 16x16x32 MFMAs:
// K index 8 grp .. 8 grp + 7 of pair q is tap 2q + (grp >> 1), input
// channels 8 (grp & 1) .. + 7 (tap 9 does not exist: zero weights and input)
__global__ void __launch_bounds__(256) k_cnn_fwd16(CnnFwd p, int layer) {
    const int lane = threadIdx.x & 63;
    const _Float16* in = layer == 1 ? p.a1 : layer == 2 ? p.a2 : p.a3;
    const int Hi = layer == 1 ? p.H1 : layer == 2 ? p.H2 : p.H3;
    const int Wi = layer == 1 ? p.W1 : layer == 2 ? p.W2 : p.W3;
    const long long si = layer == 1 ? p.s1 : layer == 2 ? p.s2 : p.s3;
    const int Ho = layer == 1 ? p.H2 : p.H3, Wo = layer == 1 ? p.W2 : p.W3;
    const int stride = layer == 3 ? 1 : 2;
    const int ntx = (Wo + 15) >> 4;
    const int item = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (item >= p.batch * Ho * ntx) return;
    const int b = item / (Ho * ntx), rem = item - b * Ho * ntx;
    if (p.active && gld(p.active + b) == 0) return;
    const int oy = rem / ntx, ox0 = (rem - (rem / ntx) * ntx) * 16;
    const int col = lane & 15, grp = lane >> 4;
    const _Float16* w = pk_h(p.pk) + (layer == 1 ? kPkW2 : layer == 2 ? kPkW3 : kPkW4);
    const int ox = ox0 + col;
    const _Float16* x = in + (size_t)b * si;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int tap = 2 * q + (grp >> 1);
        h8 A = {}, B = {};
        if (tap < 9) {
            A = *(const LANE_GLOBAL h8*)(w + (tap * 16 + col) * 16 + 8 * (grp & 1));
            const int iy = oy * stride + tap / 3 - 1, ix = ox * stride + tap % 3 - 1;
            if (ox < Wo && iy >= 0 && iy < Hi && ix >= 0 && ix < Wi)
                B = *(const LANE_GLOBAL h8*)(x + ((size_t)iy * Wi + ix) * 16 + 8 * (grp & 1));
        }
        acc = mfma32(A, B, acc);
    }
    if (ox >= Wo) return;
    const float* bias = pk_bias(p.pk, layer);
    if (layer < 3) {
        _Float16* out = (layer == 1 ? p.a2 : p.a3) + (size_t)b * (layer == 1 ? p.s2 : p.s3);
        h4 o;
#pragma unroll
        for (int j = 0; j < 4; ++j) o[j] = (_Float16)fmaxf(acc[j] + bias[4 * grp + j], 0.f);
        st_h4(out + ((size_t)oy * Wo + ox) * 16 + 4 * grp, o);
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int co = 4 * grp + j;
            if (co < 9)
                gst(p.logits + (((size_t)b * 9 + co) * Ho + oy) * Wo + ox, acc[j] + bias[co]);
        }
    }
}

// ------------------------------------------------------- fused inference --
// Forward only, all four layers in one workgroup per 8x8 block of head
// outputs: the input window (87x87 pixels) and the conv1 / conv2 / conv3
// activations the block needs (43x43, 21x21, 10x10 pixels, halo included)
// stay in LDS, so nothing but the frame and the logits touches HBM.  Every
// layer issues the same MFMA sequence on the same FP16 values as the
// layer-by-layer kernels above, so the logits are bit-identical to theirs.
// Positions outside a layer's output are stored as zero: they are the next
// layer's zero padding.
//
// Work per block: conv1 as 43 rows x 3 sixteen-pixel groups (one
// 16x16x16 MFMA each); conv2, conv3 and the head as flat runs of 16 output
// pixels (28, 7 and 4 tiles: no idle lanes past a row's end), five
// 16x16x32 MFMAs each.  Every lane's LDS offsets for those tiles depend on
// the block geometry only and are computed once per kernel.
//
// LDS (79.5 KB, two workgroups per CU): the input window converted once to
// FP16 (rows padded to 98 halves, so the stride-2 taps of the lanes past a
// row's end stay inside the window) shares its space with the conv2 window;
// windows read at stride 2 (conv1 and conv2 outputs) keep even columns
// before odd ones, so a 16-lane stride-2 read touches 16 consecutive
// pixels; the conv3 window lives in the conv1 window's space (dead by
// then); the head weights and all biases are staged once per workgroup.
// The next block's input bytes are loaded into registers while the current
// block computes.
constexpr int kFT = 8;                // head outputs per block side
constexpr int kR3 = kFT + 2;          // conv3 window side
constexpr int kR2 = 2 * kR3 + 1;      // conv2 window side
constexpr int kR1 = 2 * kR2 + 1;      // conv1 window side
constexpr int kR0 = 2 * kR1 + 1;      // input window side
constexpr int kP0 = 98;               // input window row pitch (halves): > 2 * 47 + 2
constexpr int kInferThreads = 512;
constexpr int kT2 = (kR2 * kR2 + 15) / 16;  // conv2 tiles (28)
constexpr int kT3 = (kR3 * kR3 + 15) / 16;  // conv3 tiles (7)
constexpr int kT4 = (kFT * kFT) / 16;       // head tiles (4)
constexpr int kU02 = (kR0 * kP0 > kR2 * kR2 * 16 ? kR0 * kP0 : kR2 * kR2 * 16);  // halves

struct CnnInfer {
    const uint8_t* img;
    int W, H, pitch;
    long long img_stride;
    const void* pk;
    float* logits;             // [B][9][H3][W3]
    int H1, W1, H2, W2, H3, W3;
    int bx, by;                // blocks per frame along x / y
    int batch;
    const uint8_t* active;     // frame b runs iff active[b] != 0 (null = all)
    uint8_t* mask;             // [B][H3][W3] tile masks by the rule of k_mask_from_logits, or null
    float t_hi;                // that rule's threshold
    int wide;                  // frames, pitch and stride 16-byte aligned: 16-byte input loads
};

// column of pixel x in a window of side n stored even columns first
__device__ __forceinline__ int deint(int x, int n) { return (x & 1) ? ((n + 1) >> 1) + (x >> 1) : (x >> 1); }

// A operands of a 16-channel layer for the five 16x16x32 MFMAs: K index
// 8 grp .. 8 grp + 7 of pair q is tap 2q + (grp >> 1), input channels
// 8 (grp & 1) .. + 7 (tap 9 does not exist: zero weights).
struct Taps2 {
    h8 a[5];
};
__device__ __forceinline__ Taps2 load_taps2(const _Float16* __restrict__ w, int col, int grp) {
    Taps2 t;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int tap = 2 * q + (grp >> 1);
        h8 v = {};
        if (tap < 9) v = *(const LANE_GLOBAL h8*)(w + (tap * 16 + col) * 16 + 8 * (grp & 1));
        t.a[q] = v;
    }
    return t;
}

// One 16-pixel x 16-channel tile of a 16-channel layer: lane (col, grp)
// reads, for each tap pair, 8 input channels of its pixel at the tap its
// group supplies; tapoff(t) is the LDS offset (halves) of tap t from the
// pixel's top-left input; tap 9 reuses tap 8's offset (zero weights).
template <class TapOff>
__device__ __forceinline__ f4 conv16x32(const _Float16* __restrict__ in, int base, int grp,
                                        const Taps2& w, TapOff tapoff) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    const int ch = 8 * (grp & 1), hi = grp >> 1;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int tap = min(2 * q + hi, 8);
        const h8 B = *reinterpret_cast<const h8*>(in + base + tapoff(tap) + ch);
        acc = mfma32(w.a[q], B, acc);
    }
    return acc;
}

// bias + ReLU, or zero outside the layer's output, as four FP16 channels
__device__ __forceinline__ h4 relu4(f4 acc, f4 bias, bool inside) {
    h4 o;
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = (_Float16)fmaxf(acc[j] + bias[j], 0.f);
    const h4 z = {};
    return inside ? o : z;
}

__global__ void __launch_bounds__(kInferThreads) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_cnn_infer(CnnInfer p) {
    __shared__ __align__(16) _Float16 r1[kR1 * kR1 * 16];  // conv1 out; later the conv3 window
    __shared__ __align__(16) _Float16 u02[kU02];            // input window, then conv2 out
    __shared__ __align__(16) _Float16 s_w4[9 * 16 * 16];    // head weights [tap][co][ci]
    __shared__ __align__(16) float s_bias[4 * 16];
    _Float16* r0 = u02;
    _Float16* r2 = u02;
    _Float16* r3 = r1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = kInferThreads / 64;
    const int col = lane & 15, grp = lane >> 4;
    const int nblk = p.bx * p.by;
    const _Float16* wk = pk_h(p.pk);
    // the work: (frame, block) pairs of switched-on frames, grid stride
    auto next = [&](int b, int blk, int& nb, int& nblk_out) {
        int f = b, k = blk + (int)gridDim.x;
        while (f < p.batch) {
            if (k < nblk && (!p.active || gld(p.active + f) != 0)) break;
            ++f;
            k = blockIdx.x;
        }
        nb = f;
        nblk_out = k;
    };
    // A block's input window (window position q <-> frame column x0 + q,
    // x0 = 64 TX - 15), into eight registers per thread, in one of two forms.
    // Wide (16-byte aligned frames): thread t < 261 loads row t / 3, frame
    // columns x0 - 1 + 32 (t % 3) .. + 31 as two 16-byte loads; a chunk
    // left of the frame or on a row outside it reads as zero through the
    // buffer's range check (chunks start at multiples of 16, so none
    // straddles column 0), and bytes at columns >= W are masked.  Narrow:
    // thread t < 435 loads row t / 5, columns 18 (t % 5) .. + 17, one byte
    // per load, bytes outside the frame or the window masked; four bytes per
    // register.
    constexpr int kRun = 18, kRuns = 5;
    static_assert(kRun * kRuns >= kR0 && kR0 * kRuns <= kInferThreads, "window runs");
    constexpr int kParts = 3;  // 32-byte parts per row in the wide form
    static_assert(32 * kParts >= kR0 + 1 && kR0 * kParts <= kInferThreads, "wide window");
    const bool wide = p.wide != 0;
    const int frow = wide ? tid / kParts : tid / kRuns;
    const int fcol = wide ? 32 * (tid - frow * kParts) : kRun * (tid - frow * kRuns);
    auto fetch = [&](int b, int blk, uint32_t (&v)[8]) {
        const int TY = blk / p.bx, TX = blk - TY * p.bx;
        // input window origin 2 Y1 - 1 = 8 Y4 - 15 (Y1 = 2 Y2 - 1, Y2 = 2 Y3 - 1, Y3 = Y4 - 1)
        const int y = 8 * TY * kFT - 15 + frow, x0 = 8 * TX * kFT - 15;
        // the frame as a raw buffer: offsets past its end read as zero
        const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(p.img + (size_t)b * p.img_stride), (short)0,
            (int)((uint32_t)p.pitch * (uint32_t)p.H), kBufConfig);
        if (wide) {
            const bool row_in = tid < kR0 * kParts && y >= 0 && y < p.H;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int c = x0 - 1 + fcol + 16 * h;  // a multiple of 16
                const bool in = row_in && c >= 0 && c < p.W;
                const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(
                    rsrc, in ? (uint32_t)(y * p.pitch + c) : kBufOutside, 0, 0);
                const int nv = p.W - c;  // bytes of the chunk inside the frame
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const int keep = nv - 4 * d;  // bytes of this word to keep
                    const uint32_t m = keep >= 4 ? 0xFFFFFFFFu : keep <= 0 ? 0u : (1u << (8 * keep)) - 1u;
                    v[4 * h + d] = q[d] & m;
                }
            }
            return;
        }
        const int xr = x0 + fcol;
        const bool row_in = tid < kR0 * kRuns && y >= 0 && y < p.H;
        const uint32_t off = row_in ? (uint32_t)(y * p.pitch + xr) : kBufOutside;
        uint32_t keep = 0;  // bit j: column xr + j is inside the frame and the window
#pragma unroll
        for (int j = 0; j < kRun; ++j)
            keep |= (uint32_t)(xr + j >= 0 && xr + j < p.W && fcol + j < kR0) << j;
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = 0;
#pragma unroll
        for (int j = 0; j < kRun; ++j) {
            // a column left of the frame gives a negative offset: pass the
            // out-of-range one instead (the byte is masked anyway)
            const uint32_t o = off + (uint32_t)j;
            const uint32_t bj = __builtin_amdgcn_raw_buffer_load_b8(rsrc, xr + j >= 0 ? o : kBufOutside, 0, 0);
            v[j >> 2] |= (((keep >> j) & 1u) ? bj : 0u) << (8 * (j & 3));
        }
    };
    // per-workgroup constants: head weights and biases in LDS
    for (int i = tid; i < 9 * 16 * 16 / 8; i += kInferThreads)
        *reinterpret_cast<h8*>(s_w4 + 8 * i) = *(const LANE_GLOBAL h8*)(wk + kPkW4 + 8 * i);
    if (tid < 64) s_bias[tid] = gld(pk_bias(p.pk, 0) + tid);
    // conv1 taps of this lane: K index 4 grp + j is tap 4 grp + j (taps 9..15
    // have zero weights).  The four halves come from three 32-bit LDS words
    // at the lane's pixel p (even, so every word is aligned): w0 at p + a1,
    // w1 right after it (one ds_read2), w2 at p + c1; two byte permutes
    // put them in K order.  Group 0: taps (0,0) (0,1) | (0,2) (1,0) = w0 |
    // w1.lo w2.lo; group 1: (1,1) (1,2) | (2,0) (2,1) = w0.hi w1.lo | w2;
    // groups 2, 3: tap (2,2) = w1.lo first, the rest (zero weights) finite
    // neighbours in the same row.
    const int a1 = grp == 0 ? 0 : grp == 1 ? kP0 : 2 * kP0;
    const int c1 = grp == 0 ? kP0 : 2 * kP0;
    const uint32_t sel0 = grp == 0 ? 0x03020100u : grp == 1 ? 0x05040302u : 0x01000504u;
    const uint32_t sel1 = grp == 0 ? 0x05040100u : grp == 1 ? 0x07060504u : 0x03020100u;
    const h4 A1 = ld_h4(wk + kPkW1 + col * 16 + 4 * grp);
    const Taps2 T2 = load_taps2(wk + kPkW2, col, grp);
    // conv1 lanes: column of each 16-pixel group and its de-interleaved slot
    int cx1[3];
#pragma unroll
    for (int xg = 0; xg < 3; ++xg) cx1[xg] = deint(min(16 * xg + col, kR1 - 1), kR1);
    // conv3 tile of this wave (waves 0..6) and head tile (waves 0..3)
    const int n3 = min(16 * wave + col, kR3 * kR3 - 1);
    const int y3l = n3 / kR3, x3l = n3 - y3l * kR3;
    const int in3 = (2 * y3l * kR2 + x3l) * 16;
    const int out3 = (y3l * kR3 + x3l) * 16 + 4 * grp;
    const int n4 = 16 * (wave & 3) + col;
    const int y4l = n4 >> 3, x4l = n4 & 7;
    const int in4 = (y4l * kR3 + x4l) * 16;
    __syncthreads();
    const f4 bias1 = *reinterpret_cast<const f4*>(s_bias + 4 * grp);
    const f4 bias2 = *reinterpret_cast<const f4*>(s_bias + 16 + 4 * grp);
    int b, blk;
    next(0, (int)blockIdx.x - (int)gridDim.x, b, blk);
    uint32_t v[8];
    if (b < p.batch) fetch(b, blk, v);
    while (b < p.batch) {
        const int TY = blk / p.bx, TX = blk - TY * p.bx;
        const int Y4 = TY * kFT, X4 = TX * kFT;
        const int Y3 = Y4 - 1, X3 = X4 - 1;
        const int Y2 = 2 * Y3 - 1, X2 = 2 * X3 - 1;
        const int Y1 = 2 * Y2 - 1, X1 = 2 * X2 - 1;
        // the input window, converted once to FP16 (gray / 255)
        auto h16 = [&](int i) {  // byte i of the thread's registers as FP16 bits
            const uint32_t by = (v[i >> 2] >> (8 * (i & 3))) & 0xFFu;
            return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)((float)by * (1.0f / 255.0f)));
        };
        if (wide) {
            // byte i is window position fcol - 1 + i: positions of odd i
            // start a pair (a 32-bit write); bytes 0 and 31 go alone
            if (tid < kR0 * kParts) {
                const int at = frow * kP0 + fcol - 1;  // LDS half of byte 0
                uint16_t* r0h = reinterpret_cast<uint16_t*>(r0);
                if (fcol > 0) r0h[at] = (uint16_t)h16(0);
#pragma unroll
                for (int i = 1; i < 31; i += 2)
                    *reinterpret_cast<uint32_t*>(r0h + at + i) = h16(i) | (h16(i + 1) << 16);
                if (fcol + 30 < kP0) r0h[at + 31] = (uint16_t)h16(31);
            }
        } else if (tid < kR0 * kRuns) {
            // two columns per 32-bit LDS write
#pragma unroll
            for (int j = 0; j < kRun; j += 2) {
                if (fcol + j < kR0)
                    *reinterpret_cast<uint32_t*>(r0 + frow * kP0 + fcol + j) = h16(j) | (h16(j + 1) << 16);
            }
        }
        int nb, nblk2;
        next(b, blk, nb, nblk2);
        __syncthreads();
        // the next block's input bytes travel while this one computes
        if (nb < p.batch) fetch(nb, nblk2, v);
        {  // conv1: K = the 9 taps of the single input channel; three tiles per row
            bool xin[3];
#pragma unroll
            for (int xg = 0; xg < 3; ++xg) {
                const int x1 = X1 + 16 * xg + col;
                xin[xg] = x1 >= 0 && x1 < p.W1;
            }
            for (int ly = wave; ly < kR1; ly += nw) {
                const int y1 = Y1 + ly;
                const bool yin = y1 >= 0 && y1 < p.H1;
                f4 acc[3];
#pragma unroll
                for (int xg = 0; xg < 3; ++xg) {
                    const _Float16* q = r0 + 2 * ly * kP0 + 2 * (16 * xg + col);
                    const uint32_t* qw = reinterpret_cast<const uint32_t*>(q);
                    const uint32_t w0 = qw[a1 >> 1], w1 = qw[(a1 >> 1) + 1], w2 = qw[c1 >> 1];
                    const uint32_t d0 = __builtin_amdgcn_perm(w1, w0, sel0);
                    const uint32_t d1 = __builtin_amdgcn_perm(w2, w1, sel1);
                    const h4 B = __builtin_bit_cast(h4, (unsigned long long)d0 | ((unsigned long long)d1 << 32));
                    const f4 z = {0.f, 0.f, 0.f, 0.f};
                    acc[xg] = mfma16(A1, B, z);
                }
#pragma unroll
                for (int xg = 0; xg < 3; ++xg)
                    if (16 * xg + col < kR1)
                        *reinterpret_cast<h4*>(r1 + (ly * kR1 + cx1[xg]) * 16 + 4 * grp) =
                            relu4(acc[xg], bias1, yin && xin[xg]);
            }
        }
        __syncthreads();
        {  // conv2: flat tiles of the 21x21 output, stride 2 from the de-interleaved r1
            auto tap2 = [](int t) {
                const int ky = t / 3, kx = t - 3 * (t / 3);
                return (ky * kR1 + (kx == 1 ? (kR1 + 1) / 2 : kx >> 1)) * 16;
            };
            // tile t = wave + 8 i: output pixel (y, x) of the 21x21 window, its
            // first input in r1 (row 2y, column x of the even half) and its
            // de-interleaved slot in r2
#pragma unroll 2
            for (int i = 0; i < 4; ++i) {
                if (wave + nw * i < kT2) {
                    const int n = 16 * (wave + nw * i) + col;
                    const int nc = min(n, kR2 * kR2 - 1);
                    const int y = nc / kR2, x = nc - y * kR2;
                    const f4 acc = conv16x32(r1, (2 * y * kR1 + x) * 16, grp, T2, tap2);
                    const int y2 = Y2 + y, x2 = X2 + x;
                    if (n < kR2 * kR2)
                        *reinterpret_cast<h4*>(r2 + (y * kR2 + deint(x, kR2)) * 16 + 4 * grp) =
                            relu4(acc, bias2, y2 >= 0 && y2 < p.H2 && x2 >= 0 && x2 < p.W2);
                }
            }
        }
        __syncthreads();
        if (wave < kT3) {  // conv3: stride 2 from the de-interleaved r2 into r3 (plain layout)
            auto tap3 = [](int t) {
                const int ky = t / 3, kx = t - 3 * (t / 3);
                return (ky * kR2 + (kx == 1 ? (kR2 + 1) / 2 : kx >> 1)) * 16;
            };
            // (conv3's weights come from the L2 here: kept in registers for the
            // whole kernel they would push it past 128 registers per lane)
            const Taps2 T3 = load_taps2(wk + kPkW3, col, grp);
            const f4 acc = conv16x32(r2, in3, grp, T3, tap3);
            const f4 bias3 = *reinterpret_cast<const f4*>(s_bias + 32 + 4 * grp);
            const int y3 = Y3 + y3l, x3 = X3 + x3l;
            if (16 * wave + col < kR3 * kR3)
                *reinterpret_cast<h4*>(r3 + out3) =
                    relu4(acc, bias3, y3 >= 0 && y3 < p.H3 && x3 >= 0 && x3 < p.W3);
        }
        __syncthreads();
        if (wave < kT4) {  // head: logits, no ReLU, stride 1 from r3
            Taps2 T4;
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const int tap = 2 * q + (grp >> 1);
                h8 w = {};
                if (tap < 9) w = *reinterpret_cast<const h8*>(s_w4 + (tap * 16 + col) * 16 + 8 * (grp & 1));
                T4.a[q] = w;
            }
            auto tap4 = [](int t) { return ((t / 3) * kR3 + t - 3 * (t / 3)) * 16; };
            const f4 acc = conv16x32(r3, in4, grp, T4, tap4);
            f4 z;
#pragma unroll
            for (int j = 0; j < 4; ++j) z[j] = acc[j] + s_bias[48 + min(4 * grp + j, 15)];
            const int y4 = Y4 + y4l, x4 = X4 + x4l;
            const bool tile_in = y4 < p.H3 && x4 < p.W3;
            if (tile_in) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int co = 4 * grp + j;
                    if (co < 9) gst(p.logits + (((size_t)b * 9 + co) * p.H3 + y4) * p.W3 + x4, z[j]);
                }
            }
            if (p.mask) {
                // the tile's nine logits meet in its group-0 lane (channels 4..7
                // from group 1, 8 from group 2), which applies the mask rule
                float zb[8];
                zb[0] = z[1];
                zb[1] = z[2];
                zb[2] = z[3];
#pragma unroll
                for (int j = 0; j < 4; ++j) zb[3 + j] = __shfl(z[j], col + 16);
                zb[7] = __shfl(z[0], col + 32);
                if (grp == 0 && tile_in) {
                    uint8_t m;
                    if (z[0] >= p.t_hi) {
                        int bits = 0, arg = 0;
                        float best = zb[0];
#pragma unroll
                        for (int c = 0; c < 8; ++c) {
                            if (zb[c] >= 0.f) bits |= 1 << c;
                            if (zb[c] > best) {
                                best = zb[c];
                                arg = c;
                            }
                        }
                        m = (uint8_t)(bits ? bits : (1 << arg));
                    } else if (z[0] <= -p.t_hi) {
                        m = 0;
                    } else {
                        m = 0xFF;
                    }
                    gst(p.mask + ((size_t)b * p.H3 + y4) * p.W3 + x4, m);
                }
            }
        }
        __syncthreads();  // the windows are rewritten by the next block
        b = nb;
        blk = nblk2;
    }
}

// ------------------------------------------------------------------ loss --
// One workgroup per frame.  dL/dlogits, times `scale`, goes to dy4 as NHWC
// f16 with channels 9..15 zero; loss (unscaled, float) per frame.
__global__ void __launch_bounds__(1024) k_cnn_loss(const float* __restrict__ logits,
                                                   const uint8_t* __restrict__ keep,
                                                   const uint8_t* __restrict__ bands, int th,
                                                   int tw, float scale, _Float16* dy4,
                                                   float* loss) {
    __shared__ float s_red[32];
    __shared__ int s_npos;
    const int b = blockIdx.x, tid = threadIdx.x, n = th * tw;
    const float* z = logits + (size_t)b * 9 * n;
    const uint8_t* yk = keep + (size_t)b * n;
    const uint8_t* yb = bands + (size_t)b * n;
    if (tid == 0) s_npos = 0;
    __syncthreads();
    int np = 0;
    for (int t = tid; t < n; t += blockDim.x) np += yk[t] ? 1 : 0;
    atomicAdd(&s_npos, np);  // integer: order-free
    __syncthreads();
    const int npos = s_npos;
    float lsum = 0.f;
    for (int t = tid; t < n; t += blockDim.x) {
        const float y = yk[t] ? 1.f : 0.f;
        const float zk = z[t];
        lsum += (fmaxf(zk, 0.f) - zk * y + log1pf(expf(-fabsf(zk)))) / (float)n;
        h4 g0 = {(_Float16)0, (_Float16)0, (_Float16)0, (_Float16)0}, g1 = g0, g2 = g0, g3 = g0;
        const float sk = 1.f / (1.f + expf(-zk));
        g0[0] = (_Float16)((sk - y) / (float)n * scale);
        float gb[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float zb = z[(size_t)(1 + c) * n + t];
            const float ybit = ((yb[t] >> c) & 1) ? 1.f : 0.f;
            gb[c] = 0.f;
            if (npos > 0 && y > 0.f) {
                lsum += (fmaxf(zb, 0.f) - zb * ybit + log1pf(expf(-fabsf(zb)))) / (float)(npos * 8);
                gb[c] = (1.f / (1.f + expf(-zb)) - ybit) / (float)(npos * 8) * scale;
            }
        }
        g0[1] = (_Float16)gb[0];
        g0[2] = (_Float16)gb[1];
        g0[3] = (_Float16)gb[2];
        g1[0] = (_Float16)gb[3];
        g1[1] = (_Float16)gb[4];
        g1[2] = (_Float16)gb[5];
        g1[3] = (_Float16)gb[6];
        g2[0] = (_Float16)gb[7];
        _Float16* d = dy4 + ((size_t)b * n + t) * 16;
        st_h4(d, g0);
        st_h4(d + 4, g1);
        st_h4(d + 8, g2);
        st_h4(d + 12, g3);
    }
    // fixed-order reduction of the loss
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o);
    if ((tid & 63) == 0) s_red[tid >> 6] = lsum;
    __syncthreads();
    if (tid == 0) {
        float s = 0.f;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += s_red[w];
        loss[b] = s;
    }
}

// -------------------------------------------------------- backward data --
// dPre_{l-1}[iy][ix][ci] = (a_{l-1} > 0) * sum_{tap, co} W[co][ci][tap] dY[oy][ox][co]
// for the input pixels (iy, ix) of layer l (l = head, conv3, conv2).
struct CnnBwd {
    const void* pk;
    const _Float16 *a1, *a2, *a3;
    _Float16 *d1, *d2, *d3;   // gradients of the pre-activations of conv1..3
    const _Float16* dy4;      // gradient of the head output
    const uint8_t* img;
    int W, H, pitch;
    long long img_stride;
    int H1, W1, H2, W2, H3, W3;
    long long s1, s2, s3;
    int batch;
    float* partial;           // per-wave dW partials
    int rows_per_wave;
};

__global__ void __launch_bounds__(256) k_cnn_bwd_data(CnnBwd p, int layer) {
    // layer: 3 = head (dy4 -> d3), 2 = conv3 (d3 -> d2), 1 = conv2 (d2 -> d1)
    const int lane = threadIdx.x & 63;
    const _Float16* dy = layer == 3 ? p.dy4 : layer == 2 ? p.d3 : p.d2;
    const int Ho = layer == 3 ? p.H3 : layer == 2 ? p.H3 : p.H2;
    const int Wo = layer == 3 ? p.W3 : layer == 2 ? p.W3 : p.W2;
    const long long so = layer == 3 ? p.s3 : layer == 2 ? p.s3 : p.s2;
    const _Float16* act = layer == 3 ? p.a3 : layer == 2 ? p.a2 : p.a1;
    _Float16* dx = layer == 3 ? p.d3 : layer == 2 ? p.d2 : p.d1;
    const int Hi = layer == 3 ? p.H3 : layer == 2 ? p.H2 : p.H1;
    const int Wi = layer == 3 ? p.W3 : layer == 2 ? p.W2 : p.W1;
    const long long si = layer == 3 ? p.s3 : layer == 2 ? p.s2 : p.s1;
    const int stride = layer == 3 ? 1 : 2;
    const _Float16* wT = pk_h(p.pk) + (layer == 3 ? kPkW4T : layer == 2 ? kPkW3T : kPkW2T);
    const int ntx = (Wi + 15) >> 4;
    const int item = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (item >= p.batch * Hi * ntx) return;
    const int b = item / (Hi * ntx), rem = item - b * Hi * ntx;
    const int iy = rem / ntx, ix0 = (rem - (rem / ntx) * ntx) * 16;
    const int col = lane & 15, grp = lane >> 4;
    const int ix = ix0 + col;
    const _Float16* dyb = dy + (size_t)b * so;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const h4 A = ld_h4(wT + (tap * 16 + col) * 16 + 4 * grp);  // W^T[tap][ci = col][co = 4 grp + j]
        const int ny = iy + 1 - tap / 3, nx = ix + 1 - tap % 3;
        h4 B = {(_Float16)0, (_Float16)0, (_Float16)0, (_Float16)0};
        if (ix < Wi && ny >= 0 && nx >= 0 && (ny % stride) == 0 && (nx % stride) == 0) {
            const int oy = ny / stride, ox = nx / stride;
            if (oy < Ho && ox < Wo) B = ld_h4(dyb + ((size_t)oy * Wo + ox) * 16 + 4 * grp);
        }
        acc = mfma16(A, B, acc);
    }
    if (ix >= Wi) return;
    const size_t o = (size_t)b * si + ((size_t)iy * Wi + ix) * 16 + 4 * grp;
    const h4 a = ld_h4(act + o);
    h4 r;
#pragma unroll
    for (int j = 0; j < 4; ++j) r[j] = a[j] > (_Float16)0 ? (_Float16)acc[j] : (_Float16)0;
    st_h4(dx + o, r);
}

// ------------------------------------------------------ backward weights --
// dW[tap][co][ci] = sum_pixels dY[p][co] * X[p + tap][ci], K = 16 pixels per
// MFMA; each wave covers rows_per_wave output rows of one frame and writes
// its partial sums (2304 weights + 16 biases) to partial[wave].
constexpr int kPartial = 9 * 16 * 16 + 16;

__global__ void __launch_bounds__(256) k_cnn_bwd_w16(CnnBwd p, int layer) {
    // layer: 3 = head (dy4, x = a3), 2 = conv3 (d3, x = a2), 1 = conv2 (d2, x = a1)
    const int lane = threadIdx.x & 63;
    const _Float16* dy = layer == 3 ? p.dy4 : layer == 2 ? p.d3 : p.d2;
    const int Ho = layer == 1 ? p.H2 : p.H3, Wo = layer == 1 ? p.W2 : p.W3;
    const long long so = layer == 1 ? p.s2 : p.s3;
    const _Float16* x = layer == 3 ? p.a3 : layer == 2 ? p.a2 : p.a1;
    const int Hi = layer == 3 ? p.H3 : layer == 2 ? p.H2 : p.H1;
    const int Wi = layer == 3 ? p.W3 : layer == 2 ? p.W2 : p.W1;
    const long long si = layer == 3 ? p.s3 : layer == 2 ? p.s2 : p.s1;
    const int stride = layer == 3 ? 1 : 2;
    const int R = p.rows_per_wave;
    const int nchunk = (Ho + R - 1) / R;
    const int item = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (item >= p.batch * nchunk) return;
    const int b = item / nchunk, r0 = (item - b * nchunk) * R, r1 = min(Ho, r0 + R);
    const int col = lane & 15, grp = lane >> 4;
    const _Float16* dyb = dy + (size_t)b * so;
    const _Float16* xb = x + (size_t)b * si;
    f4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    f4 accb = {0.f, 0.f, 0.f, 0.f};
    const h4 ones = {(_Float16)1, (_Float16)1, (_Float16)1, (_Float16)1};
    for (int oy = r0; oy < r1; ++oy) {
        for (int ox0 = 0; ox0 < Wo; ox0 += 16) {
            h4 A;  // A[co = col][pixel = 4 grp + j] = dY[oy][ox0 + 4 grp + j][co]
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int ox = ox0 + 4 * grp + j;
                A[j] = ox < Wo ? gld(dyb + ((size_t)oy * Wo + ox) * 16 + col) : (_Float16)0;
            }
            accb = mfma16(A, ones, accb);
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                h4 B;  // B[pixel = 4 grp + j][ci = col] = X[iy][ix][ci]
                const int iy = oy * stride + tap / 3 - 1;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int ox = ox0 + 4 * grp + j;
                    const int ix = ox * stride + tap % 3 - 1;
                    B[j] = (ox < Wo && iy >= 0 && iy < Hi && ix >= 0 && ix < Wi)
                               ? gld(xb + ((size_t)iy * Wi + ix) * 16 + col)
                               : (_Float16)0;
                }
                acc[tap] = mfma16(A, B, acc[tap]);
            }
        }
    }
    // D[co = 4 grp + j][ci = col]
    float* part = p.partial + (size_t)item * kPartial;
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int j = 0; j < 4; ++j) gst(part + (tap * 16 + 4 * grp + j) * 16 + col, acc[tap][j]);
    if (col == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) gst(part + 9 * 256 + 4 * grp + j, accb[j]);
    }
}

// conv1: dW1[co][tap] = sum_pixels dPre1[p][co] * x(p, tap)
__global__ void __launch_bounds__(256) k_cnn_bwd_w1(CnnBwd p) {
    const int lane = threadIdx.x & 63;
    const int R = p.rows_per_wave;
    const int nchunk = (p.H1 + R - 1) / R;
    const int item = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (item >= p.batch * nchunk) return;
    const int b = item / nchunk, r0 = (item - b * nchunk) * R, r1 = min(p.H1, r0 + R);
    const int col = lane & 15, grp = lane >> 4;
    const _Float16* dyb = p.d1 + (size_t)b * p.s1;
    const uint8_t* img = p.img + (size_t)b * p.img_stride;
    f4 acc = {0.f, 0.f, 0.f, 0.f}, accb = {0.f, 0.f, 0.f, 0.f};
    const h4 ones = {(_Float16)1, (_Float16)1, (_Float16)1, (_Float16)1};
    for (int oy = r0; oy < r1; ++oy) {
        for (int ox0 = 0; ox0 < p.W1; ox0 += 16) {
            h4 A, B;  // A[co = col][pixel], B[pixel][tap = col]
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int ox = ox0 + 4 * grp + j;
                A[j] = ox < p.W1 ? gld(dyb + ((size_t)oy * p.W1 + ox) * 16 + col) : (_Float16)0;
                float v = 0.f;
                if (ox < p.W1 && col < 9) {
                    const int iy = 2 * oy + col / 3 - 1, ix = 2 * ox + col % 3 - 1;
                    if (iy >= 0 && iy < p.H && ix >= 0 && ix < p.W)
                        v = (float)gld(img + (size_t)iy * p.pitch + ix) * (1.0f / 255.0f);
                }
                B[j] = (_Float16)v;
            }
            acc = mfma16(A, B, acc);
            accb = mfma16(A, ones, accb);
        }
    }
    float* part = p.partial + (size_t)item * kPartial;
#pragma unroll
    for (int j = 0; j < 4; ++j) gst(part + (4 * grp + j) * 16 + col, acc[j]);
    if (col == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) gst(part + 9 * 256 + 4 * grp + j, accb[j]);
    }
}

// Sum the partials in fixed order into the master-layout gradient of one
// layer (overwrites that layer's slice of grads).
__global__ void k_cnn_reduce(const float* __restrict__ partial, int nparts, int layer,
                             float* __restrict__ grads) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int cin = layer == 0 ? 1 : 16, cout = layer == 3 ? 9 : 16;
    const int woff[4] = {kW1, kW2, kW3, kW4}, boff[4] = {kB1, kB2, kB3, kB4};
    const int nw = cout * cin * 9;
    if (i >= nw + cout) return;
    int src, dst;
    if (i < nw) {
        const int co = i / (cin * 9), ci = (i / 9) % cin, tap = i % 9;
        src = layer == 0 ? co * 16 + tap : (tap * 16 + co) * 16 + ci;
        dst = woff[layer] + i;
    } else {
        src = 9 * 256 + (i - nw);
        dst = boff[layer] + (i - nw);
    }
    float s = 0.f;
    for (int w = 0; w < nparts; ++w) s += partial[(size_t)w * kPartial + src];
    grads[dst] = s;
}

// ------------------------------------------------------------------ adam --
__global__ void k_adam(float* __restrict__ prm, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2, float gscale) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i] * gscale;
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    prm[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------- labels --
// One thread per 8x8 tile: keep iff one of the tile's edge pixels has, for
// the angle of one of the top-k plain peaks, r within 1 of that peak's r;
// the band label is the union of those peaks' band bits.
__global__ void k_tile_labels(const uint32_t* __restrict__ list, int W, int H,
                              const int16_t* __restrict__ cq, const int16_t* __restrict__ sq,
                              int n_theta, int r_offset, const int32_t* __restrict__ peaks, int k,
                              uint8_t* keep, uint8_t* bands) {
    const ListLayout L = list_layout(W, H);
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= L.th * L.tw) return;
    const int ty = t / L.tw, tx = t - ty * L.tw;
    const uint32_t inf = gld(list + L.off_info + t);
    int cnt = min((int)(inf >> 16), 64);
    const int start = (int)(inf & 0xFFFFu);
    if (start > kSegCap - cnt) cnt = 0;  // malformed list: stay inside the segment
    const int seg = ty * L.nchunk + tx / kTilesPerChunk;
    const uint32_t* ents = list + L.off_ent + (size_t)seg * kSegCap + start;
    const int count = min(gld(peaks + 3 * k), k);
    int kp = 0, bits = 0;
    for (int q = 0; q < count; ++q) {
        const int th = gld(peaks + q), rp = gld(peaks + k + q) - r_offset;
        if (th < 0 || th >= n_theta) continue;
        const int C = gld(cq + th), S = gld(sq + th);
        bool hit = false;
        for (int e = 0; e < cnt && !hit; ++e) {
            const uint32_t xy = gld(ents + e);
            const int r = ((int)(xy & 0xFFFFu) * C + (int)(xy >> 16) * S + 8192) >> 14;
            hit = abs(r - rp) <= 1;
        }
        if (hit) {
            kp = 1;
            int bb = 0;
            for (int b = 0; b < 8; ++b) {
                const int st = (b * n_theta) / 8;
                int dd = (th - st) % n_theta;
                if (dd < 0) dd += n_theta;
                if (dd < n_theta / 4) bb |= 1 << b;
            }
            bits |= bb;
        }
    }
    keep[t] = (uint8_t)kp;
    bands[t] = (uint8_t)bits;
}

// ------------------------------------------------------------------ mask --
__global__ void k_mask_from_logits(const float* __restrict__ logits, int th, int tw, int batch,
                                   float t_hi, uint8_t* mask, const uint8_t* active) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = th * tw;
    if (i >= n * batch) return;
    const int b = i / n, t = i - b * n;
    if (active && active[b] == 0) return;
    const float* z = logits + (size_t)b * 9 * n;
    const float zk = z[t];
    uint8_t m;
    if (zk >= t_hi) {
        int bits = 0, arg = 0;
        float best = z[n + t];
        for (int c = 0; c < 8; ++c) {
            const float zb = z[(size_t)(1 + c) * n + t];
            if (zb >= 0.f) bits |= 1 << c;
            if (zb > best) {
                best = zb;
                arg = c;
            }
        }
        m = (uint8_t)(bits ? bits : (1 << arg));
    } else if (zk <= -t_hi) {
        m = 0;
    } else {
        m = 0xFF;
    }
    mask[i] = m;
}

}  // namespace lane

// ------------------------------------------------------------------- ABI --
using namespace lane;

namespace {
struct Geo {
    int H1, W1, H2, W2, H3, W3;
    long long s1, s2, s3;
};
inline int osz(int n, int s) { return (n + 2 - 3) / s + 1; }
Geo geo(int W, int H) {
    Geo g;
    g.H1 = osz(H, 2);
    g.W1 = osz(W, 2);
    g.H2 = osz(g.H1, 2);
    g.W2 = osz(g.W1, 2);
    g.H3 = osz(g.H2, 2);
    g.W3 = osz(g.W2, 2);
    g.s1 = (long long)g.H1 * g.W1 * 16;
    g.s2 = (long long)g.H2 * g.W2 * 16;
    g.s3 = (long long)g.H3 * g.W3 * 16;
    return g;
}
// activation buffer: a1 a2 a3 dy4 d3 d2 d1 (halves), each [batch][...]
struct ActPtrs {
    _Float16 *a1, *a2, *a3, *dy4, *d3, *d2, *d1;
    size_t halves;
};
ActPtrs act_ptrs(void* base, const Geo& g, int batch) {
    ActPtrs a;
    _Float16* h = (_Float16*)base;
    size_t o = 0;
    auto take = [&](long long per) {
        _Float16* p = h + o;
        o += (size_t)per * batch;
        o = (o + 127) & ~(size_t)127;
        return p;
    };
    a.a1 = take(g.s1);
    a.a2 = take(g.s2);
    a.a3 = take(g.s3);
    a.dy4 = take(g.s3);
    a.d3 = take(g.s3);
    a.d2 = take(g.s2);
    a.d1 = take(g.s1);
    a.halves = o;
    return a;
}
constexpr int kRowsPerWave = 4;
int n_parts(const Geo& g, int layer, int batch) {
    const int Ho = layer == 0 ? g.H1 : layer == 1 ? g.H2 : g.H3;
    return batch * ((Ho + kRowsPerWave - 1) / kRowsPerWave);
}
inline bool a16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
}  // namespace

extern "C" {

int lane_cnn_param_count(void) { return kCnnParams; }

int lane_cnn_sizes(int32_t W, int32_t H, int32_t batch, size_t* packed_bytes, size_t* act_bytes,
                   size_t* partial_bytes) {
    if (W < 1 || H < 1 || batch < 1) return LANE_E_ARG;
    if (W > LANE_MAX_DIM || H > LANE_MAX_DIM || batch > 4096) return LANE_E_SIZE;
    const Geo g = geo(W, H);
    if (packed_bytes) *packed_bytes = kPackedBytes;
    if (act_bytes) *act_bytes = act_ptrs(nullptr, g, batch).halves * sizeof(_Float16);
    if (partial_bytes) {
        int np = 0;
        for (int l = 0; l < 4; ++l) np = n_parts(g, l, batch) > np ? n_parts(g, l, batch) : np;
        *partial_bytes = (size_t)np * kPartial * sizeof(float);
    }
    return LANE_OK;
}

int lane_cnn_pack(const float* params, void* packed, void* stream) {
    if (!params || !packed || !a16(packed)) return LANE_E_ARG;
    const int n = 3 * 2 * kPkBlock;
    hipLaunchKernelGGL(k_cnn_pack, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, params,
                       packed);
    return hipGetLastError() == hipSuccess ? LANE_OK : LANE_E_DEVICE;
}

int lane_cnn_forward(const uint8_t* img, int32_t W, int32_t H, int32_t pitch, int64_t img_stride,
                     int32_t batch, const void* packed, void* act, float* logits, void* stream) {
    return lane_cnn_forward_active(img, W, H, pitch, img_stride, batch, packed, act, logits, nullptr,
                                   stream);
}

// Forward with per-frame flags (device uint8 [batch] or null): frames whose
// flag is 0 are skipped and keep their previous logits.
LANE_INTERNAL int lane_cnn_forward_active(const uint8_t* img, int32_t W, int32_t H, int32_t pitch,
                                          int64_t img_stride, int32_t batch, const void* packed,
                                          void* act, float* logits, const uint8_t* active,
                                          void* stream) {
    if (!img || !packed || !act || !logits || W < 1 || H < 1 || pitch < W || batch < 1 ||
        img_stride < (int64_t)H * pitch || !a16(packed) || !a16(act))
        return LANE_E_ARG;
    if (W > LANE_MAX_DIM || H > LANE_MAX_DIM || batch > 4096) return LANE_E_SIZE;
    const Geo g = geo(W, H);
    const ActPtrs a = act_ptrs(act, g, batch);
    CnnFwd p;
    memset(&p, 0, sizeof(p));
    p.img = img;
    p.W = W;
    p.H = H;
    p.pitch = pitch;
    p.img_stride = img_stride;
    p.pk = packed;
    p.a1 = a.a1;
    p.a2 = a.a2;
    p.a3 = a.a3;
    p.logits = logits;
    p.H1 = g.H1; p.W1 = g.W1; p.H2 = g.H2; p.W2 = g.W2; p.H3 = g.H3; p.W3 = g.W3;
    p.s1 = g.s1; p.s2 = g.s2; p.s3 = g.s3;
    p.batch = batch;
    p.active = active;
    hipStream_t s = (hipStream_t)stream;
    auto waves = [&](int Ho, int Wo) { return batch * Ho * ((Wo + 15) / 16); };
    hipLaunchKernelGGL(k_cnn_fwd1, dim3((waves(g.H1, g.W1) + 3) / 4), dim3(256), 0, s, p);
    hipLaunchKernelGGL(k_cnn_fwd16, dim3((waves(g.H2, g.W2) + 3) / 4), dim3(256), 0, s, p, 1);
    hipLaunchKernelGGL(k_cnn_fwd16, dim3((waves(g.H3, g.W3) + 3) / 4), dim3(256), 0, s, p, 2);
    hipLaunchKernelGGL(k_cnn_fwd16, dim3((waves(g.H3, g.W3) + 3) / 4), dim3(256), 0, s, p, 3);
    return hipGetLastError() == hipSuccess ? LANE_OK : LANE_E_DEVICE;
}

// Inference with per-frame switches (device uint8 [batch] or null): one
// persistent launch of the fused kernel; switched-off frames are skipped
// whole and keep their previous logits.  With mask != null the kernel also
// writes the tile masks of lane_mask_from_logits (confidence conf) from the
// same logits, so no mask pass follows.
LANE_INTERNAL int lane_cnn_infer_mask_active(const uint8_t* img, int32_t W, int32_t H, int32_t pitch,
                                             int64_t img_stride, int32_t batch, const void* packed,
                                             float* logits, float conf, uint8_t* mask,
                                             const uint8_t* active, void* stream) {
    if (!img || !packed || !logits || W < 1 || H < 1 || pitch < W || batch < 1 ||
        img_stride < (int64_t)H * pitch || !a16(packed))
        return LANE_E_ARG;
    if (mask && !(conf > 0.5f && conf < 1.f)) return LANE_E_ARG;
    if (W > LANE_MAX_DIM || H > LANE_MAX_DIM || batch > 4096) return LANE_E_SIZE;
    if ((int64_t)pitch * H > 0x7FFFFFFFll) return LANE_E_SIZE;  // a frame is one raw buffer
    const Geo g = geo(W, H);
    CnnInfer p;
    memset(&p, 0, sizeof(p));
    p.img = img;
    p.W = W;
    p.H = H;
    p.pitch = pitch;
    p.img_stride = img_stride;
    p.pk = packed;
    p.logits = logits;
    p.H1 = g.H1; p.W1 = g.W1; p.H2 = g.H2; p.W2 = g.W2; p.H3 = g.H3; p.W3 = g.W3;
    p.bx = (g.W3 + kFT - 1) / kFT;
    p.by = (g.H3 + kFT - 1) / kFT;
    p.batch = batch;
    p.active = active;
    p.mask = mask;
    p.wide = ((uintptr_t)img % 16 == 0 && pitch % 16 == 0 && img_stride % 16 == 0) ? 1 : 0;
    // the decision threshold in float32, the same value lane_mask_from_logits uses
    p.t_hi = mask ? (float)log((double)conf / (1.0 - (double)conf)) : 0.f;
    int dev = 0, cus = 256;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // blocks of one frame spread over the chip (two workgroups per CU);
    // frames run one after another
    const int grid = std::max(1, std::min(p.bx * p.by, 2 * cus));
    hipLaunchKernelGGL(k_cnn_infer, dim3(grid), dim3(kInferThreads), 0, (hipStream_t)stream, p);
    return hipGetLastError() == hipSuccess ? LANE_OK : LANE_E_DEVICE;
}

LANE_INTERNAL int lane_cnn_infer_active(const uint8_t* img, int32_t W, int32_t H, int32_t pitch,
                                        int64_t img_stride, int32_t batch, const void* packed,
                                        float* logits, const uint8_t* active, void* stream) {
    return lane_cnn_infer_mask_active(img, W, H, pitch, img_stride, batch, packed, logits, 0.f,
                                      nullptr, active, stream);
}

int lane_cnn_infer(const uint8_t* img, int32_t W, int32_t H, int32_t pitch, int64_t img_stride,
                   int32_t batch, const void* packed, float* logits, void* stream) {
    return lane_cnn_infer_active(img, W, H, pitch, img_stride, batch, packed, logits, nullptr,
                                 stream);
}

int lane_cnn_loss(const float* logits, const uint8_t* keep, const uint8_t* bands, int32_t W,
                  int32_t H, int32_t batch, float scale, void* act, float* loss, void* stream) {
    if (!logits || !keep || !bands || !act || !loss || W < 1 || H < 1 || batch < 1 || !a16(act))
        return LANE_E_ARG;
    if (W > LANE_MAX_DIM || H > LANE_MAX_DIM || batch > 4096) return LANE_E_SIZE;
    const Geo g = geo(W, H);
    const ActPtrs a = act_ptrs(act, g, batch);
    hipLaunchKernelGGL(k_cnn_loss, dim3(batch), dim3(1024), 0, (hipStream_t)stream, logits, keep,
                       bands, g.H3, g.W3, scale, a.dy4, loss);
    return hipGetLastError() == hipSuccess ? LANE_OK : LANE_E_DEVICE;
}

int lane_cnn_backward(const uint8_t* img, int32_t W, int32_t H, int32_t pitch, int64_t img_stride,
                      int32_t batch, const void* packed, void* act, void* partial, size_t partial_bytes,
                      float* grads, void* stream) {
    if (!img || !packed || !act || !partial || !grads || W < 1 || H < 1 || pitch < W ||
        batch < 1 || img_stride < (int64_t)H * pitch || !a16(packed) || !a16(act) || !a16(partial))
        return LANE_E_ARG;
    if (W > LANE_MAX_DIM || H > LANE_MAX_DIM || batch > 4096) return LANE_E_SIZE;
    size_t need = 0;
    lane_cnn_sizes(W, H, batch, nullptr, nullptr, &need);
    if (partial_bytes < need) return LANE_E_WS;
    const Geo g = geo(W, H);
    const ActPtrs a = act_ptrs(act, g, batch);
    CnnBwd p;
    memset(&p, 0, sizeof(p));
    p.pk = packed;
    p.a1 = a.a1; p.a2 = a.a2; p.a3 = a.a3;
    p.d1 = a.d1; p.d2 = a.d2; p.d3 = a.d3;
    p.dy4 = a.dy4;
    p.img = img;
    p.W = W; p.H = H; p.pitch = pitch; p.img_stride = img_stride;
    p.H1 = g.H1; p.W1 = g.W1; p.H2 = g.H2; p.W2 = g.W2; p.H3 = g.H3; p.W3 = g.W3;
    p.s1 = g.s1; p.s2 = g.s2; p.s3 = g.s3;
    p.batch = batch;
    p.partial = (float*)partial;
    p.rows_per_wave = kRowsPerWave;
    hipStream_t s = (hipStream_t)stream;
    auto waves_px = [&](int Hx, int Wx) { return batch * Hx * ((Wx + 15) / 16); };
    // head: weights from (dy4, a3); then data gradient into d3
    for (int layer = 3; layer >= 1; --layer) {
        const int np = n_parts(g, layer, batch);
        hipLaunchKernelGGL(k_cnn_bwd_w16, dim3((np + 3) / 4), dim3(256), 0, s, p, layer);
        hipLaunchKernelGGL(k_cnn_reduce, dim3((kPartial + 255) / 256), dim3(256), 0, s,
                           (const float*)partial, np, layer, grads);
        const int Hi = layer == 3 ? g.H3 : layer == 2 ? g.H2 : g.H1;
        const int Wi = layer == 3 ? g.W3 : layer == 2 ? g.W2 : g.W1;
        hipLaunchKernelGGL(k_cnn_bwd_data, dim3((waves_px(Hi, Wi) + 3) / 4), dim3(256), 0, s, p,
                           layer);
    }
    const int np1 = n_parts(g, 0, batch);
    hipLaunchKernelGGL(k_cnn_bwd_w1, dim3((np1 + 3) / 4), dim3(256), 0, s, p);
    hipLaunchKernelGGL(k_cnn_reduce, dim3((kPartial + 255) / 256), dim3(256), 0, s,
                       (const float*)partial, np1, 0, grads);
    return hipGetLastError() == hipSuccess ? LANE_OK : LANE_E_DEVICE;
}

int lane_adam_step(float* params, const float* grads, float* m, float* v, int32_t n, float lr,
                   float beta1, float beta2, float eps, int32_t step, float grad_scale,
                   void* stream) {
    if (!params || !grads || !m || !v || n < 1 || step < 1 || !(lr >= 0.f)) return LANE_E_ARG;
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, params,
                       grads, m, v, n, lr, beta1, beta2, eps, c1, c2, grad_scale);
    return hipGetLastError() == hipSuccess ? LANE_OK : LANE_E_DEVICE;
}

int lane_tile_labels(const uint32_t* list, int32_t W, int32_t H, const int16_t* cos_q14,
                     const int16_t* sin_q14, int32_t n_theta, int32_t r_offset,
                     const int32_t* peaks, int32_t k, uint8_t* keep, uint8_t* bands, void* stream) {
    if (!list || !cos_q14 || !sin_q14 || !peaks || !keep || !bands || W < 1 || H < 1 ||
        n_theta < 1 || k < 1 || k > 1024 || !a16(list))
        return LANE_E_ARG;
    if (W > LANE_MAX_DIM || H > LANE_MAX_DIM) return LANE_E_SIZE;
    const ListLayout L = list_layout(W, H);
    const int n = L.th * L.tw;
    hipLaunchKernelGGL(k_tile_labels, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, list,
                       W, H, cos_q14, sin_q14, n_theta, r_offset, peaks, k, keep, bands);
    return hipGetLastError() == hipSuccess ? LANE_OK : LANE_E_DEVICE;
}

int lane_mask_from_logits(const float* logits, int32_t W, int32_t H, int32_t batch, float conf,
                          uint8_t* mask, void* stream) {
    return lane_mask_from_logits_active(logits, W, H, batch, conf, mask, nullptr, stream);
}

LANE_INTERNAL int lane_mask_from_logits_active(const float* logits, int32_t W, int32_t H,
                                               int32_t batch, float conf, uint8_t* mask,
                                               const uint8_t* active, void* stream) {
    if (!logits || !mask || W < 1 || H < 1 || batch < 1 || !(conf > 0.5f && conf < 1.f))
        return LANE_E_ARG;
    if (W > LANE_MAX_DIM || H > LANE_MAX_DIM || batch > 4096) return LANE_E_SIZE;
    const Geo g = geo(W, H);
    // the decision threshold in float32, the same value the CPU rule uses
    const float t_hi = (float)log((double)conf / (1.0 - (double)conf));
    const int n = g.H3 * g.W3 * batch;
    hipLaunchKernelGGL(k_mask_from_logits, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       logits, g.H3, g.W3, batch, t_hi, mask, active);
    return hipGetLastError() == hipSuccess ? LANE_OK : LANE_E_DEVICE;
}

}  // extern "C"
