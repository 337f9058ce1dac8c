// Canny edge detector for gfx950: the detector the paper proposes in place of
// Sobel + binarization (Sec. 7).  What is computed (all integer, so exact):
//
//   blur   B = (sum_{i,j in [-2,2]} w_i w_j I(clamp x+i, clamp y+j) + 128) >> 8,
//          w = (1, 4, 6, 4, 1), frame edge replicated;
//   grad   gx, gy = the Sobel operator on B (edge replicated); m = |gx| + |gy|;
//   sector the gradient direction to the nearest 45 degrees, tan 22.5 = 13573/2^15;
//   thin   keep iff m > m(neighbour behind) and m >= m(neighbour ahead) along
//          the sector, m = 0 outside the frame;
//   class  kept and m > t_high: strong; kept and t_low < m <= t_high: weak;
//          border mode 1 leaves the one-pixel ring out;
//   link   edges = strong pixels and weak pixels 8-connected to a strong one
//          through strong or weak pixels.
//
// k_canny_thin does blur, gradient, thinning and classes for a 64 x 16 tile in
// LDS (the image tile with a 4-pixel apron, separable blur, gradient with a
// 1-pixel apron), then labels the tile's candidate pixels (strong or weak)
// by union-find in LDS and stores each pixel's label as the global index of
// its tile-local root.  The linking across tiles is lock-free union-find over
// those labels (a root always hangs under a smaller index, so every chain
// strictly decreases and ends): only the pixels of each tile's top row and
// left column unite with their neighbours across the boundary; then every
// candidate takes its root, the components holding a strong pixel are
// flagged, and the edge map is written.  A fixed number of kernels, no host
// loop, so it can sit in a graph.
#include "lane_entry.h"

namespace lane {

constexpr int kCannyTW = 64, kCannyTH = 16;  // output tile
constexpr int kCannyThreads = 256;
constexpr int kCTanQ15 = 13573;  // tan(22.5 deg) * 2^15

struct CannyDesc {
    const uint8_t* img;
    int W, H, pitch;
    int t_low, t_high, border_mode;
    uint8_t* cls;        // [H][W]: 0 none, 1 weak, 2 strong
    int32_t* label;      // [H][W]: union-find parent, -1 for non-candidates
    uint8_t* flag;       // [H][W]: 1 at the root of a component with a strong pixel
    uint8_t* edges;      // [H][W] 0/255
    uint8_t* mag;        // [H][W] or null: min(m, 255)
    uint32_t* edge_count;  // device scalar or null (zeroed beforehand)
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Union-find in LDS over a tile's pixels (parents have smaller indices).
__device__ __forceinline__ int lds_find(const int* lab, int i) {
    int r = i;
    for (int hops = 0; hops <= i; ++hops) {
        const int p = __hip_atomic_load(lab + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (p == r) return r;
        r = p;
    }
    return r;
}

__device__ __forceinline__ void lds_unite(int* lab, int a, int b) {
    for (int tries = 0; tries <= a + b + 1; ++tries) {
        a = lds_find(lab, a);
        b = lds_find(lab, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        int expected = a;
        if (__hip_atomic_compare_exchange_strong(lab + a, &expected, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP))
            return;
        a = expected;
    }
}

__global__ void __launch_bounds__(kCannyThreads) k_canny_thin(CannyDesc d) {
    // tile coordinates are image coordinates; aprons: image 4, blur 2, grad 1
    constexpr int IW = kCannyTW + 8, IH = kCannyTH + 8;   // image, clamped
    constexpr int BW = kCannyTW + 4, BH = kCannyTH + 4;   // blur at clamped positions
    constexpr int GW = kCannyTW + 2, GH = kCannyTH + 2;   // gradient
    __shared__ uint8_t s_img[IH][IW];
    __shared__ int s_h[IH][BW];          // horizontal blur pass
    __shared__ uint8_t s_b[BH][BW];
    __shared__ int16_t s_m[GH][GW];
    __shared__ int16_t s_gx[GH][GW], s_gy[GH][GW];
    __shared__ uint8_t s_cls[kCannyTH][kCannyTW];
    __shared__ int s_lab[kCannyTH * kCannyTW];
    const int X0 = blockIdx.x * kCannyTW, Y0 = blockIdx.y * kCannyTH;
    const int tid = threadIdx.x;
    const int W = d.W, H = d.H;

    for (int i = tid; i < IW * IH; i += kCannyThreads) {
        const int v = i / IW, u = i - v * IW;
        const int x = clampi(X0 - 4 + u, 0, W - 1), y = clampi(Y0 - 4 + v, 0, H - 1);
        s_img[v][u] = gld(d.img + (size_t)y * d.pitch + x);
    }
    __syncthreads();
    // B at the clamped position of each blur-tile cell: the taps of B(cx, cy)
    // are I(clamp(cx + i), ...), and s_img holds I(clamp(z)) for every z of
    // the tile, so tap z = cx + i reads s_img at z - (X0 - 4)
    for (int i = tid; i < IH * BW; i += kCannyThreads) {
        const int v = i / BW, u = i - v * BW;
        const int cx = clampi(X0 - 2 + u, 0, W - 1) - (X0 - 4);
        s_h[v][u] = s_img[v][cx - 2] + 4 * s_img[v][cx - 1] + 6 * s_img[v][cx] + 4 * s_img[v][cx + 1] +
                    s_img[v][cx + 2];
    }
    __syncthreads();
    for (int i = tid; i < BH * BW; i += kCannyThreads) {
        const int v = i / BW, u = i - v * BW;
        const int cy = clampi(Y0 - 2 + v, 0, H - 1) - (Y0 - 4);
        const int acc = s_h[cy - 2][u] + 4 * s_h[cy - 1][u] + 6 * s_h[cy][u] + 4 * s_h[cy + 1][u] +
                        s_h[cy + 2][u];
        s_b[v][u] = (uint8_t)((acc + 128) >> 8);
    }
    __syncthreads();
    // gradient on B with the edge replicated: the neighbour (cx +- 1, cy +- 1)
    // of a frame pixel is read at its clamped position, which s_b holds
    for (int i = tid; i < GH * GW; i += kCannyThreads) {
        const int v = i / GW, u = i - v * GW;
        const int x = X0 - 1 + u, y = Y0 - 1 + v;
        int m = 0, gx = 0, gy = 0;
        if (x >= 0 && y >= 0 && x < W && y < H) {
            const int xl = clampi(x - 1, 0, W - 1) - (X0 - 2), xc = x - (X0 - 2), xr = clampi(x + 1, 0, W - 1) - (X0 - 2);
            const int yu = clampi(y - 1, 0, H - 1) - (Y0 - 2), yc = y - (Y0 - 2), yd = clampi(y + 1, 0, H - 1) - (Y0 - 2);
            gx = s_b[yu][xr] + 2 * s_b[yc][xr] + s_b[yd][xr] - s_b[yu][xl] - 2 * s_b[yc][xl] - s_b[yd][xl];
            gy = s_b[yd][xl] + 2 * s_b[yd][xc] + s_b[yd][xr] - s_b[yu][xl] - 2 * s_b[yu][xc] - s_b[yu][xr];
            m = (gx < 0 ? -gx : gx) + (gy < 0 ? -gy : gy);
        }
        s_m[v][u] = (int16_t)m;
        s_gx[v][u] = (int16_t)gx;
        s_gy[v][u] = (int16_t)gy;
    }
    __syncthreads();
    for (int i = tid; i < kCannyTW * kCannyTH; i += kCannyThreads) {
        const int v = i / kCannyTW, u = i - v * kCannyTW;
        const int x = X0 + u, y = Y0 + v;
        int c = 0;
        if (x < W && y < H) {
            const int gu = u + 1, gv = v + 1;
            const int gx = s_gx[gv][gu], gy = s_gy[gv][gu], m = s_m[gv][gu];
            const int ax = gx < 0 ? -gx : gx, ay = gy < 0 ? -gy : gy;
            int m1, m2;
            if (32768 * ay <= kCTanQ15 * ax) {
                m1 = s_m[gv][gu - 1];
                m2 = s_m[gv][gu + 1];
            } else if (32768 * ax <= kCTanQ15 * ay) {
                m1 = s_m[gv - 1][gu];
                m2 = s_m[gv + 1][gu];
            } else if ((gx > 0) == (gy > 0)) {
                m1 = s_m[gv - 1][gu - 1];
                m2 = s_m[gv + 1][gu + 1];
            } else {
                m1 = s_m[gv - 1][gu + 1];
                m2 = s_m[gv + 1][gu - 1];
            }
            if (m > m1 && m >= m2) c = m > d.t_high ? 2 : (m > d.t_low ? 1 : 0);
            if (d.border_mode == 1 && (x == 0 || y == 0 || x == W - 1 || y == H - 1)) c = 0;
            if (d.mag) gst(d.mag + (size_t)y * W + x, (uint8_t)(m > 255 ? 255 : m));
        }
        s_cls[v][u] = (uint8_t)c;
        s_lab[i] = c ? i : -1;
    }
    __syncthreads();
    // the tile's components: union with the already-visited neighbours
    for (int i = tid; i < kCannyTW * kCannyTH; i += kCannyThreads) {
        const int v = i / kCannyTW, u = i - v * kCannyTW;
        if (!s_cls[v][u]) continue;
        if (u > 0 && s_cls[v][u - 1]) lds_unite(s_lab, i, i - 1);
        if (v > 0) {
            if (u > 0 && s_cls[v - 1][u - 1]) lds_unite(s_lab, i, i - kCannyTW - 1);
            if (s_cls[v - 1][u]) lds_unite(s_lab, i, i - kCannyTW);
            if (u + 1 < kCannyTW && s_cls[v - 1][u + 1]) lds_unite(s_lab, i, i - kCannyTW + 1);
        }
    }
    __syncthreads();
    for (int i = tid; i < kCannyTW * kCannyTH; i += kCannyThreads) {
        const int v = i / kCannyTW, u = i - v * kCannyTW;
        const int x = X0 + u, y = Y0 + v;
        if (x >= W || y >= H) continue;
        const int c = s_cls[v][u];
        const size_t o = (size_t)y * W + x;
        int32_t lab = -1;
        if (c) {
            const int r = lds_find(s_lab, i);  // the tile's smallest index of the component
            lab = (int32_t)((size_t)(Y0 + r / kCannyTW) * W + X0 + r % kCannyTW);
        }
        gst(d.cls + o, (uint8_t)c);
        gst(d.label + o, lab);
        gst(d.flag + o, (uint8_t)0);
    }
}

__device__ __forceinline__ int ld_label(const int32_t* label, int i) {
    return __hip_atomic_load(label + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of i: parents always have smaller indices, so at most i hops.
__device__ __forceinline__ int find_root(const int32_t* label, int i) {
    int r = i;
    for (int hops = 0; hops <= i; ++hops) {
        const int p = ld_label(label, r);
        if (p == r) return r;
        r = p;
    }
    return r;
}

__device__ __forceinline__ void unite(int32_t* label, int a, int b) {
    for (int tries = 0; tries <= a + b + 1; ++tries) {
        a = find_root(label, a);
        b = find_root(label, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        // hang root a under the smaller root b, unless a got a parent meanwhile
        int expected = a;
        if (__hip_atomic_compare_exchange_strong(label + a, &expected, b, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
        a = expected;
    }
}

// One workgroup per tile: its top row unites with the row above (N, NW, NE),
// its left column with the column to the left (W, NW, SW); inside a tile the
// labels already point at the tile-local roots.
__global__ void k_canny_merge(CannyDesc d) {
    const int X0 = blockIdx.x * kCannyTW, Y0 = blockIdx.y * kCannyTH;
    const int t = threadIdx.x;
    int x, y;
    bool top;
    if (t < kCannyTW) {
        x = X0 + t;
        y = Y0;
        top = true;
    } else if (t < kCannyTW + kCannyTH) {
        x = X0;
        y = Y0 + (t - kCannyTW);
        top = false;
    } else {
        return;
    }
    if (x >= d.W || y >= d.H) return;
    const int o = y * d.W + x;
    if (gld(d.cls + o) == 0) return;
    if (top && y > 0) {
        const int u = o - d.W;
        if (x > 0 && gld(d.cls + u - 1)) unite(d.label, o, u - 1);
        if (gld(d.cls + u)) unite(d.label, o, u);
        if (x + 1 < d.W && gld(d.cls + u + 1)) unite(d.label, o, u + 1);
    }
    if (!top && x > 0) {
        if (gld(d.cls + o - 1)) unite(d.label, o, o - 1);
        if (y > 0 && gld(d.cls + o - d.W - 1)) unite(d.label, o, o - d.W - 1);
        if (y + 1 < d.H && gld(d.cls + o + d.W - 1)) unite(d.label, o, o + d.W - 1);
    }
}

__global__ void k_canny_flatten(CannyDesc d) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= d.W) return;
    const int o = y * d.W + x;
    const int c = gld(d.cls + o);
    if (c == 0) return;
    const int r = find_root(d.label, o);
    if (c == 2) gst(d.flag + r, (uint8_t)1);
    gst(d.label + o, r);  // later kernels read the root directly
}

__global__ void k_canny_link(CannyDesc d) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    const bool in = x < d.W;
    uint32_t e = 0;
    if (in) {
        const int o = y * d.W + x;
        e = gld(d.cls + o) != 0 && gld(d.flag + gld(d.label + o)) != 0;
        gst(d.edges + o, (uint8_t)(e ? 255 : 0));
    }
    if (d.edge_count) {
        // one atomic per wave
        const uint64_t ball = __ballot(e);
        if ((threadIdx.x & (kWave - 1)) == 0 && ball) atomicAdd(d.edge_count, (uint32_t)__popcll(ball));
    }
}

}  // namespace lane

using namespace lane;

extern "C" LANE_INTERNAL size_t lane_canny_ws_bytes(int W, int H) {
    const size_t n = (size_t)W * H;
    const size_t a = (n * sizeof(int32_t) + 255) & ~(size_t)255;
    const size_t b = (n + 255) & ~(size_t)255;
    return a + 2 * b;
}

extern "C" LANE_INTERNAL hipError_t lane_launch_canny(const uint8_t* img, int W, int H, int pitch, int t_low,
                                                      int t_high, int border_mode, uint8_t* edges,
                                                      uint8_t* mag, uint32_t* edge_count, void* ws,
                                                      hipStream_t s) {
    const size_t n = (size_t)W * H;
    char* base = (char*)ws;
    CannyDesc d;
    d.img = img;
    d.W = W;
    d.H = H;
    d.pitch = pitch;
    d.t_low = t_low;
    d.t_high = t_high;
    d.border_mode = border_mode;
    d.label = (int32_t*)base;
    d.cls = (uint8_t*)(base + ((n * sizeof(int32_t) + 255) & ~(size_t)255));
    d.flag = d.cls + ((n + 255) & ~(size_t)255);
    d.edges = edges;
    d.mag = mag;
    d.edge_count = edge_count;
    const dim3 tiles((W + kCannyTW - 1) / kCannyTW, (H + kCannyTH - 1) / kCannyTH);
    hipLaunchKernelGGL(k_canny_thin, tiles, dim3(kCannyThreads), 0, s, d);
    const dim3 rows((W + 255) / 256, H);
    hipLaunchKernelGGL(k_canny_merge, tiles, dim3(kCannyTW + kCannyTH), 0, s, d);
    hipLaunchKernelGGL(k_canny_flatten, rows, dim3(256), 0, s, d);
    hipLaunchKernelGGL(k_canny_link, rows, dim3(256), 0, s, d);
    return hipGetLastError();
}
