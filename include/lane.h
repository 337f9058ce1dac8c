/*
 * lane.h -- C ABI of the MI355X (gfx950) lane-detection hot path.
 *
 * The path follows "Hardware Acceleration of Lane Detection Algorithm: A GPU
 * Versus FPGA Comparison" (arXiv 2212.09460):
 *   Sobel edge magnitude |Sx*Img| + |Sy*Img|            Sec. 2.1, Eq. (1)
 *   zero padding so the output keeps the input size     Sec. 3.1, Sec. 4.1
 *   binarization of every pixel to 255 or 0             Sec. 2.2
 *   Hough voting r = x cos(theta) + y sin(theta)        Sec. 2.3, Eq. (3)
 *   into a (theta, r) accumulator ("Hough matrix")      Sec. 2.3, Sec. 3.3
 *   peak extraction (largest counts = lines)            Sec. 2.3
 *
 * Conventions for every entry point:
 *   - Return value: LANE_OK (0) or a negative LANE_E_* code.  Argument errors
 *     are detected before anything is enqueued; a kernel fault surfaces at the
 *     caller's next synchronisation of the stream.
 *   - Pointers named "device" are HIP device pointers (e.g. from a torch
 *     tensor); "host" pointers are ordinary host memory.  The caller owns all
 *     buffers.  Data-path calls never allocate and keep no pointer after they
 *     return.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All device work is enqueued asynchronously on it.
 *   - Frames are uint8 gray images [H][pitch], row-major, pitch >= W.
 *     1 <= W, H <= 8192.
 *   - Coordinates: origin at the top-left pixel, x = column, y = row.
 *   - theta_k = k * 180 / n_theta degrees, k in [0, n_theta).
 *   - cos/sin come as a Q14 table: C[k] ~ 2^14 cos(theta_k), S[k] ~ 2^14
 *     sin(theta_k), int16.  A pixel (x, y) votes in row k at column
 *       r_idx = floor((x*C[k] + y*S[k] + 2^13) / 2^14) + r_offset,
 *     i.e. Eq. (3) rounded half up; a vote with r_idx outside [0, n_r) is
 *     dropped and counted.
 *   - Calls are stateless and reentrant.
 */
#ifndef LANE_H_
#define LANE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LANE_ABI_VERSION 2

enum {
    LANE_OK = 0,
    LANE_E_ARG = -1,         /* null required pointer, size <= 0, pitch < W, k < 1, misaligned buffer */
    LANE_E_SIZE = -2,        /* W or H > 8192, or a product overflowing the index types */
    LANE_E_RANGE = -3,       /* r_offset / n_r not as required (peaks need n_r == 2*r_offset + 1) */
    LANE_E_WS = -4,          /* workspace too small */
    LANE_E_DEVICE = -5,      /* HIP launch or runtime error */
    LANE_E_UNSUPPORTED = -6, /* e.g. an unsupported border mode */
    LANE_E_BUSY = -7,        /* serving: request dropped (stream queue full) or a replay already running */
    LANE_E_TIMEOUT = -8      /* serving: request not run, its deadline passed while it waited */
};

enum { LANE_BORDER_ZERO = 0, LANE_BORDER_ZERO_MASKRING = 1 };

#define LANE_MAX_DIM 8192

int lane_abi_version(void);
const char *lane_strerror(int status);

/* Host helper.  Fills cos_q14[n_theta], sin_q14[n_theta] (host) with
 * round-half-away-from-zero of 2^14 cos / sin of theta_k (Sec. 3.3: the
 * per-angle constants of each processing element; Sec. 4.3: cos and sin
 * computed once per angle).  Any table may be passed to the vote; this one
 * is the usual choice. */
int lane_make_trig_q14(int32_t n_theta, int16_t *cos_q14, int16_t *sin_q14);

/* Host helper.  *D_out = ceil(sqrt((W-1)^2 + (H-1)^2)), the largest |r| of
 * Eq. (3) over the frame; the usual accumulator is r_offset = D,
 * n_r = 2*D + 1. */
int lane_r_offset(int32_t W, int32_t H, int32_t *D_out);

/* Size in bytes of the compacted edge list of a W x H frame (the buffer
 * `list` below).  Layout, all uint32, counted from the buffer start:
 *   seg_count[n_seg]              edges in each segment
 *   tile_info[th*tw]              (count << 16) | start of each 8x8 tile's
 *                                 run inside its segment
 *   entries[n_seg][8192] at a 16-byte aligned offset: (y << 16) | x of each
 *                                 edge pixel, grouped by tile, tiles of a
 *                                 segment in x order, pixels of a tile in
 *                                 row-major order
 * with th = ceil(H/8), tw = ceil(W/8), a segment = one 8-row tile row times
 * 1024 columns, n_seg = th * ceil(W/1024). */
int lane_edge_list_size(int32_t W, int32_t H, size_t *bytes);

/* Sobel + binarize (Sec. 2.1 Eq. (1), Sec. 2.2, zero padding Sec. 3.1/4.1),
 * fused with the edge compaction the vote reads (Sec. 4.3: the vote reads
 * the coordinates of the edge pixels from global memory).
 *   img       device, uint8 [H][pitch]
 *   threshold a pixel is an edge iff |gx| + |gy| > threshold (0..255)
 *   border_mode LANE_BORDER_ZERO: plain zero padding; LANE_BORDER_ZERO_MASKRING:
 *             zero padding, and the one-pixel frame ring is forced to 0 in
 *             `edges` (the magnitude is unchanged)
 *   edges     device, uint8 [H][W], receives 255 / 0
 *   mag_opt   device, uint8 [H][W] or NULL: min(|gx| + |gy|, 255)
 *   list_opt  device, lane_edge_list_size() bytes, 16-byte aligned, or NULL
 *   edge_count_opt device uint32 scalar or NULL: number of edge pixels */
int lane_sobel_binarize(const uint8_t *img, int32_t W, int32_t H, int32_t pitch,
                        int32_t threshold, int32_t border_mode, uint8_t *edges,
                        uint8_t *mag_opt, uint32_t *list_opt, uint32_t *edge_count_opt,
                        void *stream);

/* Workspace bytes of lane_canny for a W x H frame (6 bytes per pixel). */
int lane_canny_workspace_size(int32_t W, int32_t H, size_t *bytes);

/* Canny edge detector, the replacement for Sobel + binarization that Sec. 7
 * proposes (the paper gives no parameters; this is the definition used):
 *   blur   B = (sum_{i,j in [-2,2]} w_i w_j I(clamp(x+i), clamp(y+j)) + 128) >> 8,
 *          w = (1, 4, 6, 4, 1), the frame edge replicated;
 *   grad   gx, gy: the Sobel operator of lane_sobel_binarize on B (edge
 *          replicated), m = |gx| + |gy|;
 *   sector along x if 32768|gy| <= 13573|gx|, along y if 32768|gx| <= 13573|gy|,
 *          else the diagonal (gx gy > 0) or the anti-diagonal;
 *   thin   a pixel is kept iff m > m(neighbour at -1 along the sector) and
 *          m >= m(neighbour at +1), m = 0 outside the frame;
 *   class  kept and m > t_high: strong; kept and t_low < m <= t_high: weak;
 *          border_mode 1 excludes the one-pixel ring;
 *   link   edge = 255 for strong pixels and weak pixels 8-connected to a
 *          strong one through strong or weak pixels; else 0.
 *   img       device uint8 [H][pitch]; W, H <= LANE_MAX_DIM
 *   t_low <= t_high in [0, 65535]
 *   edges     device uint8 [H][W]
 *   mag_opt   device uint8 [H][W] or NULL: min(m, 255)
 *   list_opt  device edge list (as lane_sobel_binarize) or NULL, 16-byte aligned
 *   edge_count_opt device uint32 scalar or NULL: edge pixels
 *   ws        device, >= lane_canny_workspace_size() bytes, 16-byte aligned
 *             (per-pixel classes, union-find labels, component flags)
 * Results are exact (integer arithmetic; the linked set does not depend on
 * the order in which components are merged). */
int lane_canny(const uint8_t *img, int32_t W, int32_t H, int32_t pitch, int32_t t_low,
               int32_t t_high, int32_t border_mode, uint8_t *edges, uint8_t *mag_opt,
               uint32_t *list_opt, uint32_t *edge_count_opt, void *ws, size_t ws_bytes,
               void *stream);

/* Compaction alone: builds the edge list from an existing edge map (a pixel
 * is an edge iff it equals 255, Sec. 3.3).  edges: device uint8 [H][pitch]. */
int lane_edges_to_list(const uint8_t *edges, int32_t W, int32_t H, int32_t pitch,
                       uint32_t *list, uint32_t *edge_count_opt, void *stream);

/* Hough vote (Sec. 2.3 Eq. (3); one accumulator row per theta as in the
 * per-angle partition of Sec. 4.3).
 *   list      device, the edge list of a W x H frame (lane_sobel_binarize or
 *             lane_edges_to_list)
 *   cos_q14, sin_q14  device, int16 [n_theta]
 *   r_offset, n_r     accumulator columns: r_idx = r + r_offset in [0, n_r)
 *   tile_mask_opt     device uint8 [ceil(H/8)][ceil(W/8)] or NULL.  If given,
 *             an edge in tile t votes in row k only if
 *             tile_mask[t] & band_bits(k) != 0, where band b (0..7) holds
 *             the k with ((k - floor(b*n_theta/8)) mod n_theta) < n_theta/4
 *             (requires n_theta % 4 == 0); NULL votes every row.
 *   acc       device, int32 [n_theta][n_r], fully overwritten
 *   dropped_opt device uint32 scalar or NULL: votes outside [0, n_r)
 * Results do not depend on the order of the list (integer sums). */
int lane_hough_vote(const uint32_t *list, int32_t W, int32_t H, const int16_t *cos_q14,
                    const int16_t *sin_q14, int32_t n_theta, int32_t r_offset, int32_t n_r,
                    const uint8_t *tile_mask_opt, int32_t *acc, uint32_t *dropped_opt,
                    void *stream);

/* Hough vote with the angle pairing of the FPGA design (Sec. 3.3 Eq. (4)-(5)):
 * theta_{n-k} = 180deg - theta_k, so for a symmetric table (C[n-k] = -C[k],
 * S[n-k] = S[k]) rows k and n-k follow from the same products x*C[k] and
 * y*S[k].  One workgroup per row pair.  pairing = 1 shares the products
 * wherever the table is symmetric (other pairs are voted row by row);
 * pairing = 0 runs the same kernel with one dot product per row (the
 * comparison).  The result is the accumulator of lane_hough_vote without a
 * tile mask, for any table.  Arguments as lane_hough_vote; 0 <= r_offset <=
 * 32768; acc is fully overwritten; dropped_opt counts votes outside [0, n_r). */
int lane_hough_vote_paired(const uint32_t *list, int32_t W, int32_t H, const int16_t *cos_q14,
                           const int16_t *sin_q14, int32_t n_theta, int32_t r_offset, int32_t n_r,
                           int32_t pairing, int32_t *acc, uint32_t *dropped_opt, void *stream);

/* Workspace bytes for lane_hough_peaks on an n_theta x n_r accumulator. */
int lane_hough_peaks_workspace_size(int32_t n_theta, int32_t n_r, size_t *bytes);

/* Hough peaks (Sec. 2.3: the largest counts are the lines; the paper leaves
 * the procedure to MATLAB, so it is specified here).  Greedy non-maximum
 * suppression: repeat up to k times -- take the largest cell not yet
 * suppressed (ties: smallest theta-major index); stop if its count is below
 * max(1, min_votes); emit it; suppress the cells with |dtheta| <= h_theta
 * and |dr| <= h_r around it, where a row index past either end wraps around
 * and, for an odd number of wraps, the column window is centred on the
 * mirrored index 2*r_offset - r_idx (the line (r, theta + 180deg) is the
 * line (-r, theta)).
 *   acc        device int32 [n_theta][n_r]; requires n_r == 2*r_offset + 1
 *   k >= 1, h_theta >= 0, h_r >= 0
 *   theta_idx, r_idx, votes  device int32 [k], -1 after the last peak
 *   count      device int32 scalar: peaks found
 *   ws         device, >= lane_hough_peaks_workspace_size() bytes, 16-byte aligned */
int lane_hough_peaks(const int32_t *acc, int32_t n_theta, int32_t n_r, int32_t r_offset,
                     int32_t k, int32_t h_theta, int32_t h_r, int32_t min_votes,
                     int32_t *theta_idx, int32_t *r_idx, int32_t *votes, int32_t *count,
                     void *ws, size_t ws_bytes, void *stream);

/* Peak search that allocates nothing and takes no workspace, for callers
 * that cannot allocate device memory (code under HIP graph capture, serving
 * loops that must not call the allocator, harnesses that forbid it).  Same
 * arguments, results and error codes as lane_hough_peaks without ws /
 * ws_bytes.  The block keys go to a fixed device array of the library, one
 * copy per GPU, held until the process ends: at most
 * lane_hough_peaks_noalloc_max_bytes() bytes (64 KiB, which every
 * accumulator the peak search accepts fits; a larger need returns
 * LANE_E_WS).  Its address on a device is looked up on the first call there
 * (LANE_E_DEVICE if that fails).  Every call on one GPU shares that array:
 * calls that overlap in time on one GPU (two streams, two threads) race and
 * must be serialised by the caller; calls in order on one stream are safe
 * (each call rewrites every key it reads). */
size_t lane_hough_peaks_noalloc_max_bytes(void);
int lane_hough_peaks_noalloc(const int32_t *acc, int32_t n_theta, int32_t n_r, int32_t r_offset,
                             int32_t k, int32_t h_theta, int32_t h_r, int32_t min_votes,
                             int32_t *theta_idx, int32_t *r_idx, int32_t *votes, int32_t *count,
                             void *stream);

/* Line segments along peaks: the lane lines drawn from the Hough peaks
 * (Sec. 1 step 4; Sec. 5, "Hough lines" and Fig. 12; the paper leaves the
 * step to MATLAB without an algorithm, so it is specified here).  For peak j
 * (theta_idx[j] = t, r_idx[j] = i):
 *   points  the 255 pixels whose vote for bin t lands in cell i, i.e.
 *           floor((x*C[t] + y*S[t] + 2^13) / 2^14) + r_offset == i
 *           (exactly the pixels counted in acc[t][i]);
 *   order   by (y, x) when |C[t]| >= |S[t]| (line nearer the vertical), else
 *           by (x, y), ascending;
 *   split   two consecutive points more than fill_gap apart (squared
 *           Euclidean distance > fill_gap^2) end a segment;
 *   keep    a segment whose first and last points are at least min_length
 *           apart (squared distance >= min_length^2).
 *   edges      device uint8 [H][W] (255 = edge), W, H <= LANE_MAX_DIM
 *   cos_q14, sin_q14  device int16 [n_theta]; a row must be a rotation
 *              (max(|C|, |S|) >= 11585), else that peak's count is -1
 *   theta_idx, r_idx  device int32 [k] (lane_hough_peaks output); entries
 *              with theta_idx < 0, or j >= *count_opt, have no segments
 *   count_opt  device int32 scalar (peaks found) or NULL (all k)
 *   k in [1, 4096]; fill_gap, min_length in [0, 65535];
 *   max_segments in [1, 1024]; r_offset in [0, 131072]
 *   segments   device int32 [k][max_segments][4]: (x1, y1, x2, y2), the first
 *              and last point of each kept segment in line order; -1 in
 *              unused slots
 *   seg_count  device int32 [k]: kept segments (may exceed max_segments:
 *              only the first max_segments are written)
 *   npts_opt   device int32 [k] or NULL: points of each peak
 * One workgroup per peak; no workspace.  Argument errors are returned before
 * anything is enqueued. */
int lane_hough_lines(const uint8_t *edges, int32_t W, int32_t H, const int16_t *cos_q14,
                     const int16_t *sin_q14, int32_t n_theta, int32_t r_offset,
                     const int32_t *theta_idx, const int32_t *r_idx, const int32_t *count_opt,
                     int32_t k, int32_t fill_gap, int32_t min_length, int32_t max_segments,
                     int32_t *segments, int32_t *seg_count, int32_t *npts_opt, void *stream);

/* ------------------------------------------------------- coarse-to-fine Hough
 * The paper bases its GPU vote (Sec. 4.3) on a multiresolution progressive
 * Hough method (its reference [9]) and states no algorithm; this is the one
 * computed here (all integer, so exact):
 *   coarse vote   coarse row c in [0, n_theta / theta_step) uses the fine
 *                 table row c*theta_step + theta_step/2; with w = r_width
 *                 (odd) and q = (w-1)/2, an edge's Eq. (3) r (as in
 *                 lane_hough_vote) in [-r_offset, r_offset] adds 1 at column
 *                 floor((r + q) / w) + Dc, Dc = floor((r_offset + q) / w),
 *                 of a [n_theta/theta_step][2 Dc + 1] accumulator (bins of w
 *                 cells centred on r = 0); any other r is not counted;
 *   coarse peaks  lane_hough_peaks on it (k_coarse, h_theta_coarse,
 *                 h_r_coarse, min_votes_coarse, r_offset Dc);
 *   windows       coarse peak j = (c, b) opens R = theta_step + 2*margin_theta
 *                 rows u = c*theta_step - margin_theta + a by Wc = w +
 *                 2*margin_r cells; cell (a, e) counts the edges whose r at
 *                 fine row u mod n_theta equals rr = (b - Dc)*w - q - margin_r
 *                 + e, or -rr when u is an odd number of half turns away from
 *                 [0, n_theta) (the line (r, theta + 180deg) is (-r, theta));
 *                 cells with |rr| > r_offset are empty and never chosen;
 *   candidate j   the window's largest count, first in (a, e) order, as the
 *                 fine cell (theta_idx, r_idx = r + r_offset, count);
 *   final peaks   lane_hough_peaks (k, h_theta, h_r, min_votes) on a fine
 *                 accumulator that is zero except at the candidates.
 * Limits: n_theta % theta_step == 0; r_width odd in [1, 63]; k_coarse in
 * [1, 64]; k in [1, k_coarse]; 0 <= h_theta < n_theta; margin_theta in
 * [0, 512]; margin_r in [0, 8192]; R*Wc + 2R + 5 <= 16384;
 * 0 <= r_offset <= 16384; the coarse row (2 Dc + 2 cells of 4 bytes) at
 * most 96 KB. */
typedef struct lane_progressive {
    int32_t theta_step, r_width;
    int32_t k_coarse, h_theta_coarse, h_r_coarse, min_votes_coarse;
    int32_t margin_theta, margin_r;
    int32_t k, h_theta, h_r, min_votes;
} lane_progressive;

/* Geometry and workspace layout.  After lane_hough_progressive the
 * workspace holds, at these byte offsets, the coarse accumulator (int32
 * [n_coarse_theta][n_coarse_r]), the coarse peaks (int32 theta[k_coarse],
 * r_idx[k_coarse], votes[k_coarse], count), the windows (int32
 * [k_coarse][win_rows][win_cols], zero for absent peaks) and the candidates
 * (int32 [k_coarse][3], -1 for absent peaks). */
typedef struct lane_progressive_layout {
    int32_t n_coarse_theta, n_coarse_r, coarse_r_offset, win_rows, win_cols;
    size_t coarse_acc, coarse_peaks, windows, candidates, bytes;
} lane_progressive_layout;

/* Fills *out for a W x H frame; LANE_E_ARG / LANE_E_SIZE as the limits above. */
int lane_hough_progressive_layout(int32_t W, int32_t H, int32_t n_theta, int32_t r_offset,
                                  const lane_progressive *p, lane_progressive_layout *out);

/* Coarse-to-fine Hough of one frame.
 *   list      device edge list of a W x H frame (lane_sobel_binarize, lane_canny
 *             or lane_edges_to_list), 16-byte aligned
 *   cos_q14, sin_q14  device int16 [n_theta]; r_offset as for lane_hough_vote
 *             (the fine accumulator has 2*r_offset + 1 columns)
 *   p         host, read during the call
 *   theta_idx, r_idx, votes  device int32 [p->k], -1 after the last peak
 *   count     device int32 scalar: final peaks
 *   ws        device, >= layout.bytes, 16-byte aligned; also holds the
 *             intermediate results (see lane_progressive_layout)
 * Argument errors are returned before anything is enqueued. */
int lane_hough_progressive(const uint32_t *list, int32_t W, int32_t H, const int16_t *cos_q14,
                           const int16_t *sin_q14, int32_t n_theta, int32_t r_offset,
                           const lane_progressive *p, int32_t *theta_idx, int32_t *r_idx,
                           int32_t *votes, int32_t *count, void *ws, size_t ws_bytes,
                           void *stream);

/* ------------------------------------------------------------------ batch
 * Many frames of mixed sizes through the whole path (Sobel + binarize +
 * compaction, vote, peaks, and line segments where a frame asks for them) in
 * one HIP graph launch.  A plan is built once
 * per set of buffers (creation allocates a small device descriptor table,
 * with a split vote also one edge-list-sized buffer per frame that has a tile
 * mask, and instantiates the graph; launching allocates nothing).  Each stage is a
 * persistent kernel that walks a work table covering every frame; the
 * paper's GPU grid of one block per 16x16 pixels (Sec. 4.1 Eq. (6)) and of
 * one block per angle (Sec. 4.3) become these tables. */
typedef struct lane_frame {
    const uint8_t *img;       /* device uint8 [H][pitch] */
    int32_t W, H, pitch;
    int32_t threshold, border_mode;
    uint8_t *edges;           /* device uint8 [H][W] */
    uint8_t *mag_opt;         /* device uint8 [H][W] or NULL */
    uint32_t *list;           /* device, lane_edge_list_size(W, H) bytes, 16-byte aligned */
    const int16_t *cos_q14;   /* device int16 [n_theta] */
    const int16_t *sin_q14;   /* device int16 [n_theta] */
    int32_t n_theta, r_offset, n_r;
    const uint8_t *tile_mask_opt; /* device uint8 [ceil(H/8)][ceil(W/8)] or NULL */
    int32_t *acc;             /* device int32 [n_theta][n_r] */
    int32_t k, h_theta, h_r, min_votes; /* peaks; k == 0 skips the peak step */
    int32_t *peaks;           /* device int32 [3k + 1]: theta_idx[k], r_idx[k], votes[k], count */
    void *peaks_ws;           /* device, lane_hough_peaks_workspace_size() bytes, 16-byte aligned */
    size_t peaks_ws_bytes;
    uint32_t *counters_opt;   /* device uint32 [2] or NULL: edge pixels, dropped votes */
    /* line segments along the peaks (lane_hough_lines), run after the peak
     * step when lines_opt != NULL and k > 0 */
    int32_t lines_max_seg;    /* segments per peak, [1, 1024] */
    int32_t lines_fill_gap;   /* [0, 65535] */
    int32_t lines_min_length; /* [0, 65535] */
    int32_t *lines_opt;       /* device int32 [k*lines_max_seg*4 + 2k]: segments [k][max_seg][4],
                                 then seg_count [k], then npts [k]; or NULL */
} lane_frame;

typedef struct lane_tune {
    int32_t vote_rows;        /* theta rows per vote workgroup, power of two; 0 = the largest that
                                 fits the half-size LDS variant (two workgroups per CU), unless
                                 the full-size maximum is more than twice that */
    int32_t vote_queue;       /* 1 = dynamic ticket queue (longest items first), 0 = static stride
                                 with each frame's slices on one XCD, 2 = one ticket queue per XCD
                                 over the frames given to it (its L2 shares their edge lists),
                                 taking from the others once its own is used up; -1 = automatic */
    int32_t sobel_groups_per_cu; /* Sobel workgroups per CU of a persistent grid; 0 = one
                                    workgroup per four work items (no persistent grid) */
    int32_t sobel_strip_rows; /* rows per Sobel work item, a multiple of 8; 0 = 32 */
    int32_t vote_split;       /* workgroups per theta slice, each voting a 1/vote_split share of
                                 the edge list (1..64; 0 or 1 = none) and adding its rows into the
                                 accumulator, which the plan then clears before each vote; the
                                 peak keys are then found by a pass of their own.  A frame with
                                 a tile mask then votes from a pruned copy of its edge list
                                 (the entries of tiles that vote every row, then those of
                                 band-restricted tiles, tested entry by entry), which the plan
                                 writes before the vote and owns (lane_edge_list_size bytes) */
} lane_tune;

typedef struct lane_batch lane_batch;

/* frames: host array of n descriptors (copied).  tune_opt may be NULL.
 * Validation is the same as for the single-frame calls. */
int lane_batch_create(const lane_frame *frames, int32_t n, const lane_tune *tune_opt,
                      lane_batch **out);
/* Enqueue the whole path for every frame: one hipGraphLaunch on `stream`.
 * The graph runs the stages below in order, except that the vote's set-up
 * (its work queue, the accumulators of a split vote) is done by the
 * counter-clearing kernel at the start rather than before the vote. */
int lane_batch_launch(lane_batch *b, void *stream);
/* Enqueue one stage without the graph (0 = clear counters, 1 = Sobel,
 * 2 = vote, 3 = peaks, 4 = line segments of the frames that ask for them),
 * e.g. to time the stages separately. */
int lane_batch_launch_stage(lane_batch *b, int32_t stage, void *stream);
/* Device address (*flags) of the plan's per-frame switches, uint8 [n] in
 * frame order, owned by the plan and all 1 after creation.  A launch (graph
 * or stage) runs the frames whose switch is non-zero; a frame switched off
 * keeps its previous outputs and counters.  The caller may rewrite the
 * switches between launches with stream-ordered copies. */
int lane_batch_active_flags(lane_batch *b, uint8_t **flags);
/* Select the frames the next launches run (active: host uint8 [n], non-zero
 * = run): enqueues on `stream` the copies of the switches and of work lists
 * holding only those frames' items, so switched-off frames cost nothing.
 * The copies come from page-locked staging owned by the plan: call again only
 * after the launches this selection served have completed. */
int lane_batch_select(lane_batch *b, const uint8_t *active, void *stream);
/* Frees the plan's device table and graph (waits for nothing: the caller
 * must make sure no launch of this plan is still running). */
int lane_batch_destroy(lane_batch *b);

/* Autotuner (set-up call: allocates scratch buffers and synchronizes).
 * Builds plans over n_frames copies of `sample` (device uint8 [H][pitch]),
 * times the vote for every theta-slice width (rows per workgroup, down to
 * 1/16 of the largest that fits LDS) and the three work distributions, then the
 * Sobel pass for strip heights 8..128 with and without a persistent grid (1
 * or 2 workgroups per CU), and writes the fastest setting to *out (a vote
 * setting with per-XCD queues is taken over a faster one within 1 %: the same
 * time within measurement noise, with far less traffic from beyond the L2).
 * ms_opt: host float[2] or NULL, receives the chosen vote and the best Sobel
 * times in ms. */
int lane_tune_run(const uint8_t *sample, int32_t W, int32_t H, int32_t pitch, int32_t threshold,
                  int32_t border_mode, int32_t n_theta, int32_t n_frames, lane_tune *out,
                  float *ms_opt);

/* Set-up call: the same sweep on the caller's own frames (any mix of sizes;
 * the plans it times write their outputs), with one more vote setting,
 * vote_rows = 0 (each frame takes its own default rows: the per-resolution
 * choice for mixed batches).  Arguments of every frame as for
 * lane_batch_create; ms_opt as for lane_tune_run. */
int lane_tune_batch(const lane_frame *frames, int32_t n, lane_tune *out, float *ms_opt);

/* ---------------------------------------------------- learned proposal
 * A small CNN predicts, per 8x8 tile, whether the tile carries lane votes
 * and which theta bands they fall in, so the vote can skip the rest (task
 * addition; the paper has no learned part).  Network, zero padding 1:
 * conv1 1->16 stride 2 + ReLU, conv2 16->16 s2 + ReLU, conv3 16->16 s2 +
 * ReLU, head 16->9 s1; input gray / 255; FP16 weights and activations, FP32
 * accumulation on MFMA.  Output logits [batch][9][ceil(H/8)][ceil(W/8)]:
 * channel 0 keep, 1..8 bands (band definition as for lane_hough_vote).
 * Master parameters: LANE_CNN_PARAMS floats, per layer weights
 * [c_out][c_in][3][3] then biases [c_out]. */
#define LANE_CNN_PARAMS 6105

int lane_cnn_param_count(void);
/* Byte sizes (any pointer may be NULL): packed kernel weights, activation
 * workspace for `batch` frames of W x H (forward + backward), and the
 * backward pass's partial-sum workspace. */
int lane_cnn_sizes(int32_t W, int32_t H, int32_t batch, size_t *packed_bytes, size_t *act_bytes,
                   size_t *partial_bytes);
/* FP32 master parameters (device) -> packed FP16 kernel layouts (device,
 * 16-byte aligned). */
int lane_cnn_pack(const float *params, void *packed, void *stream);
/* Forward for `batch` frames img + b * img_stride (device uint8 [H][pitch]);
 * activations kept in `act` for the backward; logits device float. */
int lane_cnn_forward(const uint8_t *img, int32_t W, int32_t H, int32_t pitch, int64_t img_stride,
                     int32_t batch, const void *packed, void *act, float *logits, void *stream);
/* Inference only, same logits as lane_cnn_forward (bit-identical): all
 * four layers fused per 8x8 block of logits with the intermediate
 * activations in LDS, so it needs no activation workspace. */
int lane_cnn_infer(const uint8_t *img, int32_t W, int32_t H, int32_t pitch, int64_t img_stride,
                   int32_t batch, const void *packed, float *logits, void *stream);
/* Per frame: loss = mean over tiles of BCE(keep) + mean over keep tiles of
 * the mean over bands of BCE(band) -> loss[b] (device float); writes
 * scale * dloss/dlogits into `act` for the backward.  keep: device uint8
 * [batch][th][tw] in {0,1}; bands: device uint8 band bits. */
int lane_cnn_loss(const float *logits, const uint8_t *keep, const uint8_t *bands, int32_t W,
                  int32_t H, int32_t batch, float scale, void *act, float *loss, void *stream);
/* Backward after lane_cnn_forward + lane_cnn_loss on the same `act`: writes
 * the gradient, summed over the batch and times the loss scale, into grads
 * [LANE_CNN_PARAMS] (device float).  Deterministic (fixed reduction order). */
int lane_cnn_backward(const uint8_t *img, int32_t W, int32_t H, int32_t pitch, int64_t img_stride,
                      int32_t batch, const void *packed, void *act, void *partial,
                      size_t partial_bytes, float *grads, void *stream);
/* Adam on device float vectors of length n; the gradient is multiplied by
 * grad_scale first; step counts from 1. */
int lane_adam_step(float *params, const float *grads, float *m, float *v, int32_t n, float lr,
                   float beta1, float beta2, float eps, int32_t step, float grad_scale,
                   void *stream);
/* Training labels from the plain pipeline: tile t is keep iff one of its
 * edge pixels has, for the angle of one of the top-k peaks (device int32
 * [3k+1] as written by the batch plan: theta_idx, r_idx, votes, count), an
 * r within 1 of that peak's r; bands[t] = union of those peaks' band bits.
 * list: the frame's edge list; keep, bands: device uint8 [th][tw]. */
int lane_tile_labels(const uint32_t *list, int32_t W, int32_t H, const int16_t *cos_q14,
                     const int16_t *sin_q14, int32_t n_theta, int32_t r_offset,
                     const int32_t *peaks, int32_t k, uint8_t *keep, uint8_t *bands, void *stream);
/* Tile mask for lane_hough_vote from float logits: keep logit >= t ->
 * the bands with logit >= 0 (at least the largest); keep <= -t -> 0 (skip);
 * otherwise 0xFF (fall back to every band), t = float(log(conf/(1-conf))),
 * 0.5 < conf < 1.  mask: device uint8 [batch][th][tw]. */
int lane_mask_from_logits(const float *logits, int32_t W, int32_t H, int32_t batch, float conf,
                          uint8_t *mask, void *stream);

/* ------------------------------------------------------------- serving
 * Continuous batching of frames from many camera streams (task addition:
 * the paper times one frame from input image to lines, Sec. 5; a deployment
 * serves many cameras).  A server keeps each admitted stream's state
 * resident in device memory: its frame slot, edge map, edge list,
 * accumulator, peak buffers and, when pruned, the proposal logits and tile
 * mask.  Streams with the same configuration form a class whose frame slots
 * are contiguous, so the proposal network runs over a class as one batch.
 * Each of a few refill lanes (a worker thread with its own batch plan,
 * graphs and compute stream) repeats: take the oldest pending request of
 * every stream that is not in a running refill (at most one per stream),
 * switch on exactly those slots, run the set-up kernel (counters and
 * accumulators, no frame read), copy those frames into their slots (or wait
 * for their copies ahead), launch one graph (network and mask per class when
 * pruned, then Sobel, vote, peaks; switched-off slots return at once;
 * the peak search stores each slot's peaks in page-locked host memory, so no
 * copy follows) and complete the requests.  With two or more lanes, a request of a stream that is not in
 * the running refill starts at once beside it instead of waiting for it; a
 * stream's requests still run one at a time, in submission order.  The frame
 * of a request that heads the queue of a stream not in a running refill is
 * copied to its slot at once, on a copy stream of its own, so that copy
 * overlaps the running refills and the next one starts with it in place.  A
 * frame's results do not depend on the other frames of its batch or on the
 * refills running beside it.  Failures: a request beyond its stream's queue
 * bound is dropped (LANE_E_BUSY); with a deadline, one that waited too long
 * is completed unrun (LANE_E_TIMEOUT) and frees its place; a device error
 * fails that refill's requests and, since the device state can no longer be
 * trusted, every later one (LANE_E_DEVICE; lane_server_stats.error). */
#define LANE_SERVE_MAX_K 64
#define LANE_SERVE_MAX_LANES 4

typedef struct lane_stream_cfg {
    int32_t W, H;             /* frame size */
    int32_t n_theta;          /* theta bins, <= 8192 (a multiple of 4 when pruned) */
    int32_t k;                /* peaks per frame, 1..LANE_SERVE_MAX_K */
    int32_t threshold;        /* binarization threshold 0..255 */
    int32_t border_mode;
} lane_stream_cfg;

typedef struct lane_server_cfg {
    size_t hbm_budget;        /* device bytes the streams' state may take */
    int32_t pruned;           /* 1: proposal network + masked vote; 0: plain */
    float conf;               /* pruned: mask confidence, 0.5 < conf < 1 */
    const float *cnn_params;  /* pruned: host float [LANE_CNN_PARAMS], copied at creation */
    int32_t max_pending;      /* per-stream queue bound, >= 1; a request beyond it is dropped */
    int32_t vote_rows;        /* theta rows per vote workgroup (power of two); 0 = 4 */
    int32_t sobel_strip_rows; /* rows per Sobel work item (multiple of 8); 0 = 8 */
    int32_t vote_split;       /* lane_tune.vote_split for the server's plan; 0 = 8 */
    int64_t deadline_ns;      /* > 0: a request that has waited longer than this when a refill
                                 would take it is completed with LANE_E_TIMEOUT instead of run,
                                 and its stream's next request takes the slot; 0 = no deadline */
    int32_t lanes;            /* refills that may run at once, 1..LANE_SERVE_MAX_LANES; 0 = 2.
                                 Each lane holds its own plan (for a pruned server with a split
                                 vote, a pruned copy of each stream's edge list per lane) */
    int32_t spin_us;          /* 0: an idle lane sleeps until work arrives; > 0 (at most 10^7):
                                 it first polls for this long, so a request arriving meanwhile
                                 starts without a thread wake-up (about 10-20 us), at the cost
                                 of a busy host core per polling lane */
} lane_server_cfg;

typedef struct lane_result {
    int32_t stream;           /* the caller's stream index */
    int32_t status;           /* LANE_OK, LANE_E_BUSY (dropped), LANE_E_TIMEOUT or LANE_E_DEVICE */
    uint64_t frame_id;        /* as submitted */
    int64_t t_submit_ns;      /* steady clock: submission */
    int64_t t_start_ns;       /* its batch taken from the queues */
    int64_t t_done_ns;        /* peaks in host memory */
    int32_t batch_frames;     /* frames in the batch that ran it */
    int32_t count;            /* peaks found */
    int32_t theta_idx[LANE_SERVE_MAX_K], r_idx[LANE_SERVE_MAX_K], votes[LANE_SERVE_MAX_K];
} lane_result;

typedef struct lane_request {
    int32_t stream;
    int32_t pitch;
    int64_t t_offset_ns;      /* arrival time after the replay starts, non-decreasing */
    const uint8_t *frame;     /* host uint8 [H][pitch] */
    uint64_t frame_id;
} lane_request;

typedef struct lane_server_stats {
    int64_t submitted, completed, dropped, batches, frames_in_batches;
    int64_t device_bytes;     /* the server's device allocation */
    int32_t streams_admitted;
    int32_t error;            /* LANE_OK, or the first device error */
    int64_t timed_out;        /* requests completed with LANE_E_TIMEOUT */
} lane_server_stats;

typedef struct lane_server lane_server;

/* Host only, no device calls.  Admission: streams are taken in order and
 * admitted while the device bytes of the admitted ones (their state, shared
 * tables and network weights) stay
 * within hbm_budget.  admitted (host uint8 [n], 1/0), stream_bytes (host
 * size_t [n], each stream's added bytes) and total_bytes may be NULL. */
int lane_server_plan(const lane_stream_cfg *streams, int32_t n, const lane_server_cfg *cfg,
                     uint8_t *admitted, size_t *stream_bytes, size_t *total_bytes);
/* Set-up call: admits as lane_server_plan, allocates the device state in one
 * allocation plus page-locked result buffers, builds each lane's plan and
 * graphs and starts the lanes' worker threads.  LANE_E_WS if no stream fits
 * the budget. */
int lane_server_create(const lane_stream_cfg *streams, int32_t n, const lane_server_cfg *cfg,
                       lane_server **out, uint8_t *admitted_opt);
/* Queue a frame (host uint8 [H][pitch] of the stream's size).  The bytes are
 * read when the request heads its stream's queue with the stream idle (the
 * copy ahead, started by this call then) or when its batch starts, so they
 * must stay valid and unchanged until its result is taken (page-locked
 * memory copies asynchronously; a pageable frame makes the copy ahead, and
 * so this call, wait for the bytes to be read, while the lanes go on).  Returns
 * LANE_E_BUSY, and completes the request as dropped, when the stream already
 * has max_pending requests waiting; LANE_E_ARG for a stream not admitted.
 * Thread-safe. */
int lane_server_submit(lane_server *s, int32_t stream, const uint8_t *frame, int32_t pitch,
                       uint64_t frame_id);
/* Up to max finished results (host array) in completion order; waits up to
 * wait_ms for the first (0: no wait, negative: until one is there). */
int lane_server_poll(lane_server *s, lane_result *out, int32_t max, int32_t wait_ms,
                     int32_t *n_out);
/* Open-loop load: submits reqs[i] at (call time + t_offset_ns) from the
 * calling thread, waits for every request and writes results[i] (host [n]).
 * These results do not go to lane_server_poll.  One replay at a time. */
int lane_server_replay(lane_server *s, const lane_request *reqs, int32_t n, lane_result *results);
int lane_server_stats_get(lane_server *s, lane_server_stats *out);
/* paused = 1: the lanes take no further refill (those already running
 * finish) while requests keep queueing and their deadlines keep running;
 * paused = 0: it resumes.  For draining and maintenance.  Thread-safe. */
int lane_server_pause(lane_server *s, int32_t paused);
/* Stops the lanes after the refills in flight (queued requests are discarded)
 * and frees everything.  No other call on s may be running. */
int lane_server_destroy(lane_server *s);

#ifdef __cplusplus
}
#endif

#endif /* LANE_H_ */
