// C ABI of liblane.so: argument validation, then asynchronous launches on
// the caller's stream.  No allocation, no synchronisation, no state.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "lane_entry.h"

using namespace lane;


namespace {

inline bool dims_ok(int W, int H) { return W >= 1 && H >= 1; }
inline bool dims_small(int W, int H) { return W <= LANE_MAX_DIM && H <= LANE_MAX_DIM; }
inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
inline int dev_status(hipError_t e) { return e == hipSuccess ? LANE_OK : LANE_E_DEVICE; }

int isqrt_ceil(int64_t q) {
    int64_t d = (int64_t)sqrt((double)q);
    while (d * d < q) ++d;
    while (d > 0 && (d - 1) * (d - 1) >= q) --d;
    return (int)d;
}

}  // namespace

extern "C" {

int lane_abi_version(void) { return LANE_ABI_VERSION; }

const char* lane_strerror(int status) {
    switch (status) {
        case LANE_OK: return "ok";
        case LANE_E_ARG: return "invalid argument";
        case LANE_E_SIZE: return "size out of range";
        case LANE_E_RANGE: return "accumulator range invalid";
        case LANE_E_WS: return "workspace too small";
        case LANE_E_DEVICE: return "HIP device error";
        case LANE_E_UNSUPPORTED: return "unsupported option";
        case LANE_E_BUSY: return "request dropped or server busy";
        case LANE_E_TIMEOUT: return "request deadline passed";
        default: return "unknown status";
    }
}

int lane_make_trig_q14(int32_t n_theta, int16_t* cos_q14, int16_t* sin_q14) {
    if (n_theta <= 0 || !cos_q14 || !sin_q14) return LANE_E_ARG;
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < n_theta; ++k) {
        const double a = (double)k * pi / (double)n_theta;
        const double c = cos(a) * 16384.0, s = sin(a) * 16384.0;
        cos_q14[k] = (int16_t)(c >= 0 ? floor(c + 0.5) : -floor(-c + 0.5));
        sin_q14[k] = (int16_t)(s >= 0 ? floor(s + 0.5) : -floor(-s + 0.5));
    }
    return LANE_OK;
}

int lane_r_offset(int32_t W, int32_t H, int32_t* D_out) {
    if (!dims_ok(W, H) || !D_out) return LANE_E_ARG;
    if (!dims_small(W, H)) return LANE_E_SIZE;
    *D_out = isqrt_ceil((int64_t)(W - 1) * (W - 1) + (int64_t)(H - 1) * (H - 1));
    return LANE_OK;
}

int lane_edge_list_size(int32_t W, int32_t H, size_t* bytes) {
    if (!dims_ok(W, H) || !bytes) return LANE_E_ARG;
    if (!dims_small(W, H)) return LANE_E_SIZE;
    *bytes = list_layout(W, H).words * sizeof(uint32_t);
    return LANE_OK;
}

int lane_sobel_binarize(const uint8_t* img, int32_t W, int32_t H, int32_t pitch, int32_t threshold,
                        int32_t border_mode, uint8_t* edges, uint8_t* mag_opt, uint32_t* list_opt,
                        uint32_t* edge_count_opt, void* stream) {
    if (!img || !edges || !dims_ok(W, H) || pitch < W || threshold < 0 || threshold > 255)
        return LANE_E_ARG;
    if (!dims_small(W, H)) return LANE_E_SIZE;
    if (border_mode != LANE_BORDER_ZERO && border_mode != LANE_BORDER_ZERO_MASKRING)
        return LANE_E_UNSUPPORTED;
    if (list_opt && !aligned16(list_opt)) return LANE_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    SobelDesc d;
    memset(&d, 0, sizeof(d));
    d.img = img;
    d.W = W;
    d.H = H;
    d.pitch = pitch;
    d.threshold = threshold;
    d.border_mode = border_mode;
    d.edges = edges;
    d.mag = mag_opt;
    d.list = list_opt;
    d.edge_count = edge_count_opt;
    d.strip_rows = kStripRows;
    if (edge_count_opt) {
        hipError_t e = lane_launch_fill_u32(edge_count_opt, 1, 0u, s);
        if (e != hipSuccess) return LANE_E_DEVICE;
    }
    return dev_status(lane_launch_sobel(&d, 0, s));
}

int lane_edges_to_list(const uint8_t* edges, int32_t W, int32_t H, int32_t pitch, uint32_t* list,
                       uint32_t* edge_count_opt, void* stream) {
    if (!edges || !list || !dims_ok(W, H) || pitch < W) return LANE_E_ARG;
    if (!dims_small(W, H)) return LANE_E_SIZE;
    if (!aligned16(list)) return LANE_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    SobelDesc d;
    memset(&d, 0, sizeof(d));
    d.img = edges;
    d.W = W;
    d.H = H;
    d.pitch = pitch;
    d.list = list;
    d.edge_count = edge_count_opt;
    d.strip_rows = kStripRows;
    if (edge_count_opt) {
        hipError_t e = lane_launch_fill_u32(edge_count_opt, 1, 0u, s);
        if (e != hipSuccess) return LANE_E_DEVICE;
    }
    return dev_status(lane_launch_sobel(&d, 1, s));
}

// LDS cells one theta row needs: the r range of one angle across the frame
// (at most D + 1 cells, plus rounding), never more than n_r.
LANE_INTERNAL int lane_vote_row_cap(int32_t W, int32_t H, int32_t n_r) {
    int32_t D = 0;
    lane_r_offset(W, H, &D);
    return D + 3 < n_r ? D + 3 : n_r;
}

// LDS words a vote workgroup needs for slices of T rows: the rows back to
// back (T x the row cap) or, for a slice whose rows all bound their cell
// pairs below 2^14 votes (vote_pair_bound on the lane_make_trig_q14 table),
// T x ceil(span / 2) with span the r range of the slice's rows -- from the
// exact corner values, widened by 4 for the table's rounding.  The kernel
// measures the real span and the bound of the table it is given and picks
// the layout that fits (another table may fall back to global memory).
LANE_INTERNAL long lane_vote_slice_words(int32_t W, int32_t H, int32_t n_theta, int32_t n_r, int T) {
    const long plain = (long)T * lane_vote_row_cap(W, H, n_r);
    if (T > n_theta) return plain;
    const double pi = 3.14159265358979323846;
    long worst = 0;
    for (int s = 0; s * T < n_theta; ++s) {
        const int k0 = s * T < n_theta - T ? s * T : n_theta - T;
        double lo = 1e300, hi = -1e300;
        bool pair_ok = true;
        for (int k = k0; k < k0 + T; ++k) {
            const double a = (double)k * pi / (double)n_theta;
            const double cq = cos(a) * 16384.0, sq = sin(a) * 16384.0;
            const int Cq = (int)(cq >= 0 ? floor(cq + 0.5) : -floor(-cq + 0.5));
            const int Sq = (int)(sq >= 0 ? floor(sq + 0.5) : -floor(-sq + 0.5));
            if (vote_pair_bound(W, H, Cq, Sq) > kPairCountMax) pair_ok = false;
            const double c = cos(pi * k / n_theta), sn = sin(pi * k / n_theta);
            const double xs[4] = {0.0, (double)(W - 1), 0.0, (double)(W - 1)};
            const double ys[4] = {0.0, 0.0, (double)(H - 1), (double)(H - 1)};
            for (int q = 0; q < 4; ++q) {
                const double r = xs[q] * c + ys[q] * sn;
                lo = r < lo ? r : lo;
                hi = r > hi ? r : hi;
            }
        }
        const long span = (long)(floor(hi + 0.5) - floor(lo + 0.5)) + 1 + 4;
        const long words = pair_ok && (span + 1) / 2 * T < plain ? (span + 1) / 2 * T : plain;
        worst = words > worst ? words : worst;
    }
    return worst < plain ? worst : plain;
}

// Rows per vote workgroup: the largest power of two <= 64 and <= n_theta
// whose slices fit in LDS.
LANE_INTERNAL int lane_vote_rows_per_group(int32_t W, int32_t H, int32_t n_theta, int32_t n_r) {
    int T = kMaxT;
    while (T > 1 && (T > n_theta || lane_vote_slice_words(W, H, n_theta, n_r, T) > kVoteLdsWords)) T >>= 1;
    return T;
}

// Default rows per batched vote workgroup: the largest T whose slices fit the
// half-size LDS variant (two workgroups per CU hide each other's LDS latency),
// unless the full-size maximum is more than twice that.
LANE_INTERNAL int lane_vote_rows_default(int32_t W, int32_t H, int32_t n_theta, int32_t n_r) {
    const int tmax = lane_vote_rows_per_group(W, H, n_theta, n_r);
    int th = tmax;
    while (th > 1 && lane_vote_slice_words(W, H, n_theta, n_r, th) > kVoteLdsWordsHalf) th >>= 1;
    return 2 * th >= tmax ? th : tmax;
}

int lane_hough_vote(const uint32_t* list, int32_t W, int32_t H, const int16_t* cos_q14,
                    const int16_t* sin_q14, int32_t n_theta, int32_t r_offset, int32_t n_r,
                    const uint8_t* tile_mask_opt, int32_t* acc, uint32_t* dropped_opt,
                    void* stream) {
    if (!list || !cos_q14 || !sin_q14 || !acc || !dims_ok(W, H) || n_theta <= 0 || n_r <= 0)
        return LANE_E_ARG;
    if (!aligned16(list)) return LANE_E_ARG;
    if (!dims_small(W, H) || (int64_t)n_theta * n_r > 0x7FFFFFFFll) return LANE_E_SIZE;
    if (tile_mask_opt && (n_theta % 4) != 0) return LANE_E_UNSUPPORTED;
    if (r_offset < -32768 * 4 || r_offset > 32768 * 4) return LANE_E_RANGE;
    hipStream_t s = (hipStream_t)stream;
    VoteDesc d;
    memset(&d, 0, sizeof(d));
    d.list = list;
    d.W = W;
    d.H = H;
    d.cos_q14 = cos_q14;
    d.sin_q14 = sin_q14;
    d.n_theta = n_theta;
    d.r_offset = r_offset;
    d.n_r = n_r;
    d.tile_mask = tile_mask_opt;
    d.acc = acc;
    d.dropped = dropped_opt;
    // one frame: few rows per workgroup, so the slices fill the CUs
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    d.T = lane_vote_rows_per_group(W, H, n_theta, n_r);
    while (d.T > 1 && (n_theta + d.T - 1) / d.T < cus) d.T >>= 1;
    d.log2T = ilog2_floor((unsigned)d.T);
    d.n_slices = (n_theta + d.T - 1) / d.T;
    if (dropped_opt) {
        hipError_t e = lane_launch_fill_u32(dropped_opt, 1, 0u, s);
        if (e != hipSuccess) return LANE_E_DEVICE;
    }
    return dev_status(lane_launch_vote(&d, s));
}

int lane_hough_vote_paired(const uint32_t* list, int32_t W, int32_t H, const int16_t* cos_q14,
                           const int16_t* sin_q14, int32_t n_theta, int32_t r_offset, int32_t n_r,
                           int32_t pairing, int32_t* acc, uint32_t* dropped_opt, void* stream) {
    if (!list || !cos_q14 || !sin_q14 || !acc || !dims_ok(W, H) || n_theta <= 0 || n_r <= 0 ||
        (pairing != 0 && pairing != 1))
        return LANE_E_ARG;
    if (!aligned16(list)) return LANE_E_ARG;
    if (!dims_small(W, H) || (int64_t)n_theta * n_r > 0x7FFFFFFFll) return LANE_E_SIZE;
    if (r_offset < 0 || r_offset > 32768) return LANE_E_RANGE;
    hipStream_t s = (hipStream_t)stream;
    VoteDesc d;
    memset(&d, 0, sizeof(d));
    d.list = list;
    d.W = W;
    d.H = H;
    d.cos_q14 = cos_q14;
    d.sin_q14 = sin_q14;
    d.n_theta = n_theta;
    d.r_offset = r_offset;
    d.n_r = n_r;
    d.acc = acc;
    d.dropped = dropped_opt;
    if (dropped_opt) {
        hipError_t e = lane_launch_fill_u32(dropped_opt, 1, 0u, s);
        if (e != hipSuccess) return LANE_E_DEVICE;
    }
    return dev_status(lane_launch_vote_pair(&d, pairing, s));
}

// Key blocks are row chunks of 1 << lg cells; the smallest lg >= 6 (one
// wave per block) whose block count fits the selection pass's LDS table.
LANE_INTERNAL int lane_peaks_block_log2(int32_t n_theta, int32_t n_r) {
    int lg = 6;
    while ((int64_t)n_theta * (((int64_t)n_r + (1ll << lg) - 1) >> lg) > kPeaksMaxBlocksLds) ++lg;
    return lg;
}

LANE_INTERNAL int lane_peaks_blocks_per_row(int32_t n_r, int lg) {
    return (int)(((int64_t)n_r + (1ll << lg) - 1) >> lg);
}

int lane_hough_peaks_workspace_size(int32_t n_theta, int32_t n_r, size_t* bytes) {
    if (n_theta <= 0 || n_r <= 0 || !bytes) return LANE_E_ARG;
    if ((int64_t)n_theta * n_r > 0x7FFFFFFFll || n_theta > kPeaksMaxBlocksLds) return LANE_E_SIZE;
    const int lg = lane_peaks_block_log2(n_theta, n_r);
    *bytes = (size_t)n_theta * (size_t)lane_peaks_blocks_per_row(n_r, lg) * sizeof(unsigned long long);
    return LANE_OK;
}

// Validates the arguments of a peak search and fills *d (all but the
// workspace pointer); *need receives the workspace bytes.
LANE_INTERNAL int lane_peaks_prepare(const int32_t* acc, int32_t n_theta, int32_t n_r, int32_t r_offset,
                                     int32_t k, int32_t h_theta, int32_t h_r, int32_t min_votes,
                                     int32_t* theta_idx, int32_t* r_idx, int32_t* votes, int32_t* count,
                                     PeaksDesc* d, size_t* need) {
    if (!acc || !theta_idx || !r_idx || !votes || !count || n_theta <= 0 || n_r <= 0 || k < 1 ||
        k > 1024 || h_theta < 0 || h_r < 0)
        return LANE_E_ARG;
    if ((int64_t)n_theta * n_r > 0x7FFFFFFFll || h_theta > 1000000 || h_r > 1000000 ||
        n_theta > kPeaksMaxBlocksLds)
        return LANE_E_SIZE;
    if (n_r != 2 * r_offset + 1) return LANE_E_RANGE;
    lane_hough_peaks_workspace_size(n_theta, n_r, need);
    memset(d, 0, sizeof(*d));
    d->acc = acc;
    d->n_theta = n_theta;
    d->n_r = n_r;
    d->r_offset = r_offset;
    d->k = k;
    d->h_theta = h_theta;
    d->h_r = h_r;
    d->min_votes = min_votes;
    d->theta_idx = theta_idx;
    d->r_idx = r_idx;
    d->votes = votes;
    d->count = count;
    d->block_log2 = lane_peaks_block_log2(n_theta, n_r);
    d->nbr = lane_peaks_blocks_per_row(n_r, d->block_log2);
    d->n_blocks = n_theta * d->nbr;
    return LANE_OK;
}

int lane_hough_peaks(const int32_t* acc, int32_t n_theta, int32_t n_r, int32_t r_offset, int32_t k,
                     int32_t h_theta, int32_t h_r, int32_t min_votes, int32_t* theta_idx,
                     int32_t* r_idx, int32_t* votes, int32_t* count, void* ws, size_t ws_bytes,
                     void* stream) {
    if (!ws || !aligned16(ws)) return LANE_E_ARG;
    PeaksDesc d;
    size_t need = 0;
    const int st = lane_peaks_prepare(acc, n_theta, n_r, r_offset, k, h_theta, h_r, min_votes,
                                      theta_idx, r_idx, votes, count, &d, &need);
    if (st != LANE_OK) return st;
    if (ws_bytes < need) return LANE_E_WS;
    d.keys = (unsigned long long*)ws;
    return dev_status(lane_launch_peaks(&d, (hipStream_t)stream));
}

int lane_canny_workspace_size(int32_t W, int32_t H, size_t* bytes) {
    if (!bytes || !dims_ok(W, H)) return LANE_E_ARG;
    if (!dims_small(W, H)) return LANE_E_SIZE;
    *bytes = lane_canny_ws_bytes(W, H);
    return LANE_OK;
}

int lane_canny(const uint8_t* img, int32_t W, int32_t H, int32_t pitch, int32_t t_low, int32_t t_high,
               int32_t border_mode, uint8_t* edges, uint8_t* mag_opt, uint32_t* list_opt,
               uint32_t* edge_count_opt, void* ws, size_t ws_bytes, void* stream) {
    if (!img || !edges || !ws || !dims_ok(W, H) || pitch < W || t_low < 0 || t_high < t_low ||
        t_high > 65535)
        return LANE_E_ARG;
    if (!dims_small(W, H)) return LANE_E_SIZE;
    if (border_mode != LANE_BORDER_ZERO && border_mode != LANE_BORDER_ZERO_MASKRING)
        return LANE_E_UNSUPPORTED;
    if ((list_opt && !aligned16(list_opt)) || !aligned16(ws)) return LANE_E_ARG;
    if (ws_bytes < lane_canny_ws_bytes(W, H)) return LANE_E_WS;
    hipStream_t s = (hipStream_t)stream;
    if (edge_count_opt && lane_launch_fill_u32(edge_count_opt, 1, 0u, s) != hipSuccess) return LANE_E_DEVICE;
    hipError_t e = lane_launch_canny(img, W, H, pitch, t_low, t_high, border_mode, edges, mag_opt,
                                     list_opt ? nullptr : edge_count_opt, ws, s);
    if (e != hipSuccess || !list_opt) return dev_status(e);
    // the edge list, as lane_edges_to_list builds it (counting the edges)
    SobelDesc d;
    memset(&d, 0, sizeof(d));
    d.img = edges;
    d.W = W;
    d.H = H;
    d.pitch = W;
    d.list = list_opt;
    d.edge_count = edge_count_opt;
    d.strip_rows = kStripRows;
    return dev_status(lane_launch_sobel(&d, 1, s));
}

int lane_hough_lines(const uint8_t* edges, int32_t W, int32_t H, const int16_t* cos_q14,
                     const int16_t* sin_q14, int32_t n_theta, int32_t r_offset,
                     const int32_t* theta_idx, const int32_t* r_idx, const int32_t* count_opt,
                     int32_t k, int32_t fill_gap, int32_t min_length, int32_t max_segments,
                     int32_t* segments, int32_t* seg_count, int32_t* npts_opt, void* stream) {
    if (!edges || !cos_q14 || !sin_q14 || !theta_idx || !r_idx || !segments || !seg_count ||
        !dims_ok(W, H) || n_theta <= 0 || k < 1 || k > 4096 || fill_gap < 0 || fill_gap > 65535 ||
        min_length < 0 || min_length > 65535 || max_segments < 1 || max_segments > 1024)
        return LANE_E_ARG;
    if (!dims_small(W, H)) return LANE_E_SIZE;
    if (r_offset < 0 || r_offset > 131072) return LANE_E_RANGE;
    return dev_status(lane_launch_lines(edges, W, H, cos_q14, sin_q14, n_theta, r_offset, theta_idx,
                                        r_idx, count_opt, k, fill_gap, min_length, max_segments,
                                        segments, seg_count, npts_opt, (hipStream_t)stream));
}

}  // extern "C"

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Geometry, workspace layout and launch shape of the coarse-to-fine Hough;
// LANE_OK or the error of the first limit broken.
int prog_plan(int32_t W, int32_t H, int32_t n_theta, int32_t r_offset, const lane_progressive* p,
              lane_progressive_layout* lay, ProgDesc* d) {
    if (!p || !lay || !dims_ok(W, H) || n_theta <= 0) return LANE_E_ARG;
    if (!dims_small(W, H)) return LANE_E_SIZE;
    if (r_offset < 0 || r_offset > 16384) return LANE_E_RANGE;
    const int f = p->theta_step, w = p->r_width, kc = p->k_coarse, k = p->k;
    if (f < 1 || n_theta % f != 0 || w < 1 || w > 63 || (w % 2) == 0 || kc < 1 || kc > 64 || k < 1 ||
        k > kc || p->h_theta_coarse < 0 || p->h_r_coarse < 0 || p->h_theta_coarse > 1000000 ||
        p->h_r_coarse > 1000000 || p->margin_theta < 0 || p->margin_theta > 512 || p->margin_r < 0 ||
        p->margin_r > 8192 || p->h_theta < 0 || p->h_theta >= n_theta || p->h_r < 0 ||
        p->h_r > 1000000)
        return LANE_E_ARG;
    const int q = (w - 1) / 2;
    const int n_c = n_theta / f, Dc = (r_offset + q) / w, n_rc = 2 * Dc + 1;
    const int R = f + 2 * p->margin_theta, Wc = w + 2 * p->margin_r;
    if (n_c > kPeaksMaxBlocksLds || n_theta > kPeaksMaxBlocksLds) return LANE_E_SIZE;
    if ((size_t)(n_rc + 1) * sizeof(int32_t) > (size_t)kProgCoarseLdsMax) return LANE_E_SIZE;
    if (lane_prog_refine_lds(1, R, Wc) > (size_t)kProgRefineLdsMax) return LANE_E_SIZE;
    size_t keys = 0;
    if (lane_hough_peaks_workspace_size(n_c, n_rc, &keys) != LANE_OK) return LANE_E_SIZE;

    lay->n_coarse_theta = n_c;
    lay->n_coarse_r = n_rc;
    lay->coarse_r_offset = Dc;
    lay->win_rows = R;
    lay->win_cols = Wc;
    lay->coarse_acc = 0;
    lay->windows = align256((size_t)n_c * n_rc * sizeof(int32_t));
    lay->coarse_peaks = align256(lay->windows + (size_t)kc * R * Wc * sizeof(int32_t));
    lay->candidates = align256(lay->coarse_peaks + (size_t)(3 * kc + 1) * sizeof(int32_t));
    const size_t off_keys = align256(lay->candidates + (size_t)3 * kc * sizeof(int32_t));
    lay->bytes = off_keys + keys;
    if (!d) return LANE_OK;

    memset(d, 0, sizeof(*d));
    d->W = W;
    d->H = H;
    d->n_theta = n_theta;
    d->D = r_offset;
    d->f = f;
    d->w = w;
    d->q = q;
    d->kc = kc;
    d->mt = p->margin_theta;
    d->mr = p->margin_r;
    d->k = k;
    d->ht = p->h_theta;
    d->hr = p->h_r;
    d->min_votes = p->min_votes;
    d->n_c = n_c;
    d->n_rc = n_rc;
    d->Dc = Dc;
    d->R = R;
    d->Wc = Wc;
    d->inv_w = (float)(1.0 / (double)w);
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    const ListLayout L = list_layout(W, H);
    // coarse: chunks of 16-segment groups, about kProgTargetGroups workgroups
    // in total; the most rows per workgroup (4, 2, 1) whose LDS stays within
    // 64 KB and whose grid still gives 2 workgroups per CU
    const int n_groups = (L.nseg + 15) / 16;
    auto chunks_for = [&](int T) {
        const int slices = (n_c + T - 1) / T;
        int c = (kProgTargetGroups + slices - 1) / slices;
        return c < 1 ? 1 : (c > n_groups ? n_groups : c);
    };
    d->T = 4;
    while (d->T > 1 && ((size_t)(n_rc + 1) * d->T * sizeof(int32_t) > 65536 ||
                        ((n_c + d->T - 1) / d->T) * chunks_for(d->T) < 2 * cus))
        d->T >>= 1;
    d->n_slices = (n_c + d->T - 1) / d->T;
    const int chunks = chunks_for(d->T);
    d->groups_per_chunk = (n_groups + chunks - 1) / chunks;
    d->n_chunks = (n_groups + d->groups_per_chunk - 1) / d->groups_per_chunk;
    // refine: as many windows per workgroup as fit 64 KB; the edges cut into
    // units (parts of segments) so that about kProgRefineGroups workgroups run
    d->wpg = kc;
    while (d->wpg > 1 && lane_prog_refine_lds(d->wpg, R, Wc) > (size_t)kProgRefineLdsMax) --d->wpg;
    d->n_wgroups = (kc + d->wpg - 1) / d->wpg;
    const int want = (kProgRefineGroups + d->n_wgroups - 1) / d->n_wgroups;
    int P = (want + L.nseg - 1) / L.nseg;
    d->r_parts = P < 1 ? 1 : (P > 16 ? 16 : P);
    const long units = (long)L.nseg * d->r_parts;
    d->r_chunks = (int)(units < want ? units : want);
    return LANE_OK;
}

}  // namespace

extern "C" {

int lane_hough_progressive_layout(int32_t W, int32_t H, int32_t n_theta, int32_t r_offset,
                                  const lane_progressive* p, lane_progressive_layout* out) {
    if (!out) return LANE_E_ARG;
    lane_progressive_layout lay;
    const int st = prog_plan(W, H, n_theta, r_offset, p, &lay, nullptr);
    if (st == LANE_OK) *out = lay;
    return st;
}

int lane_hough_progressive(const uint32_t* list, int32_t W, int32_t H, const int16_t* cos_q14,
                           const int16_t* sin_q14, int32_t n_theta, int32_t r_offset,
                           const lane_progressive* p, int32_t* theta_idx, int32_t* r_idx,
                           int32_t* votes, int32_t* count, void* ws, size_t ws_bytes, void* stream) {
    if (!list || !cos_q14 || !sin_q14 || !theta_idx || !r_idx || !votes || !count || !ws)
        return LANE_E_ARG;
    if (!aligned16(list) || !aligned16(ws)) return LANE_E_ARG;
    lane_progressive_layout lay;
    ProgDesc d;
    const int st = prog_plan(W, H, n_theta, r_offset, p, &lay, &d);
    if (st != LANE_OK) return st;
    if (ws_bytes < lay.bytes) return LANE_E_WS;
    char* base = (char*)ws;
    d.list = list;
    d.cos_q14 = cos_q14;
    d.sin_q14 = sin_q14;
    d.coarse_acc = (int32_t*)(base + lay.coarse_acc);
    d.windows = (int32_t*)(base + lay.windows);
    d.cpk = (int32_t*)(base + lay.coarse_peaks);
    d.cand = (int32_t*)(base + lay.candidates);
    d.theta_idx = theta_idx;
    d.r_idx = r_idx;
    d.votes = votes;
    d.count = count;
    PeaksDesc pk;
    memset(&pk, 0, sizeof(pk));
    pk.acc = d.coarse_acc;
    pk.n_theta = d.n_c;
    pk.n_r = d.n_rc;
    pk.r_offset = d.Dc;
    pk.k = d.kc;
    pk.h_theta = p->h_theta_coarse;
    pk.h_r = p->h_r_coarse;
    pk.min_votes = p->min_votes_coarse;
    pk.theta_idx = d.cpk;
    pk.r_idx = d.cpk + d.kc;
    pk.votes = d.cpk + 2 * d.kc;
    pk.count = d.cpk + 3 * d.kc;
    pk.keys = (unsigned long long*)(base + align256(lay.candidates + (size_t)3 * d.kc * sizeof(int32_t)));
    pk.block_log2 = lane_peaks_block_log2(d.n_c, d.n_rc);
    pk.nbr = lane_peaks_blocks_per_row(d.n_rc, pk.block_log2);
    pk.n_blocks = d.n_c * pk.nbr;
    return dev_status(lane_launch_progressive(&d, &pk, (hipStream_t)stream));
}

}  // extern "C"
