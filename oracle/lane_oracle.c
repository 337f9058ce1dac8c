/*
 * CPU ORACLE for the lane-detection hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct nested loops that state what the path
 * computes.  Only the tests, the smoke check and the benchmark's CPU
 * baseline use this file; the product (the HIP library) never links, loads
 * or calls it, and this file includes nothing from the product.
 *
 * What is computed, and where the paper defines it:
 *   oracle_sobel_binarize  Sec. 2.1 Eq. (1): |G| = |Sx*Img| + |Sy*Img| with
 *                          the zero padding of Sec. 3.1 / Sec. 4.1 (output
 *                          has the input's size); Sec. 2.2: every pixel
 *                          becomes 255 or 0.
 *   oracle_hough_vote      Sec. 2.3 Eq. (3): r = x cos(theta) + y sin(theta);
 *                          every 255 pixel votes for every theta bin
 *                          (Sec. 3.3: 1-degree bins over 180 degrees) into
 *                          the accumulator ("Hough matrix").
 *   oracle_hough_peaks     Sec. 2.3: the line with the largest count is the
 *                          line with the most pixels ("Hough peak"; the paper
 *                          delegates it to MATLAB and gives no algorithm).
 *   oracle_hough_lines     Sec. 1 step 4 and Sec. 5 ("Hough lines", Fig. 12):
 *                          the lane lines drawn from the peaks; again MATLAB
 *                          in the paper, no algorithm given (reading below).
 *   oracle_canny           Sec. 7: the Canny detector the paper proposes in
 *                          place of Sobel + binarization (specified below).
 *   oracle_hough_progressive  the coarse-to-fine Hough transform of the
 *                          multiresolution method the paper cites for its
 *                          GPU vote (Sec. 4.3, reference [9]); the paper
 *                          gives no algorithm, so it is specified below.
 *
 * Readings where the paper is silent (each one is listed with its reason in
 * the design notes):
 *   - Sobel coefficients: [1 2 1]^T x [-1 0 1] and its transpose; with the
 *     absolute values of Eq. (1) sign and orientation do not matter.
 *   - magnitude saturates at 255; edge iff |gx|+|gy| > T (strict).
 *   - border_mode 1 forces the one-pixel frame ring to 0 in the edge map.
 *   - theta_k = k*180/n_theta degrees, k in [0, n_theta) (half open).
 *   - origin at the top-left pixel, x = column, y = row, 0-based.
 *   - cos/sin come as a Q14 integer table (input data);
 *     r = floor((x*C[k] + y*S[k] + 2^13) / 2^14), stored at r + r_offset;
 *     votes whose index falls outside [0, n_r) are counted as dropped.
 *   - peaks: greedy non-maximum suppression, see oracle_hough_peaks.
 *   - lines: the pixels that voted into a peak's cell, ordered along the
 *     line, split at gaps, short pieces dropped; see oracle_hough_lines.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* pixel of the zero-padded image */
static int P(const uint8_t *img, int W, int H, int pitch, int u, int v)
{
    if (u < 0 || v < 0 || u >= W || v >= H) return 0;
    return img[(size_t)v * pitch + u];
}

static int iabs(int a) { return a < 0 ? -a : a; }

/* Sec. 2.1 Eq. (1) + Sec. 2.2.  edges[H][W] gets 0/255, mag[H][W] (nullable)
 * gets min(|gx|+|gy|, 255).  Returns the number of 255 pixels. */
int64_t oracle_sobel_binarize(const uint8_t *img, int W, int H, int pitch, int T,
                              int border_mode, uint8_t *edges, uint8_t *mag)
{
    int64_t n = 0;
    /* rows are independent (the OpenMP build splits them over threads) */
#pragma omp parallel for reduction(+ : n) schedule(static)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int gx = P(img, W, H, pitch, x + 1, y - 1) + 2 * P(img, W, H, pitch, x + 1, y) +
                     P(img, W, H, pitch, x + 1, y + 1) - P(img, W, H, pitch, x - 1, y - 1) -
                     2 * P(img, W, H, pitch, x - 1, y) - P(img, W, H, pitch, x - 1, y + 1);
            int gy = P(img, W, H, pitch, x - 1, y + 1) + 2 * P(img, W, H, pitch, x, y + 1) +
                     P(img, W, H, pitch, x + 1, y + 1) - P(img, W, H, pitch, x - 1, y - 1) -
                     2 * P(img, W, H, pitch, x, y - 1) - P(img, W, H, pitch, x + 1, y - 1);
            int g = iabs(gx) + iabs(gy);
            int e = g > T ? 255 : 0;
            if (border_mode == 1 && (x == 0 || y == 0 || x == W - 1 || y == H - 1)) e = 0;
            edges[(size_t)y * W + x] = (uint8_t)e;
            if (mag) mag[(size_t)y * W + x] = (uint8_t)(g > 255 ? 255 : g);
            n += e == 255;
        }
    }
    return n;
}

/* floor(a / b) for b > 0 */
static int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) --q;
    return q;
}

/* Membership of theta bin k in band b (8 overlapping bands, each a quarter
 * of the half turn, starting every eighth): ((k - floor(b*n/8)) mod n) < n/4. */
int oracle_band_bits(int n_theta, int k)
{
    int bits = 0;
    for (int b = 0; b < 8; ++b) {
        int start = (b * n_theta) / 8;
        int d = ((k - start) % n_theta + n_theta) % n_theta;
        if (d < n_theta / 4) bits |= 1 << b;
    }
    return bits;
}

/* Sec. 2.3 Eq. (3) voting.  edges[H][epitch]: a pixel votes iff it equals
 * 255.  tile_mask (nullable) [ceil(H/8)][ceil(W/8)]: the pixel votes for bin
 * k only if mask & band_bits(k) != 0.  acc[n_theta][n_r] is overwritten.
 * Returns the number of votes cast into acc; *dropped gets the rest (-1 if
 * the edge set could not be held).
 *
 * The edge set E is listed first (row-major), then every theta row k counts
 * the votes of all of E.  Rows are independent, so the build of this file
 * with OpenMP (the multi-core CPU baseline) gives each thread whole rows:
 * no shared counters, and integer sums that do not depend on the split. */
int64_t oracle_hough_vote(const uint8_t *edges, int W, int H, int epitch, const int16_t *C,
                          const int16_t *S, int n_theta, int r_offset, int n_r,
                          const uint8_t *tile_mask, int32_t *acc, int64_t *dropped)
{
    int tw = (W + 7) / 8;
    int64_t cast = 0, drop = 0, ne = 0;
    memset(acc, 0, sizeof(int32_t) * (size_t)n_theta * (size_t)n_r);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) ne += edges[(size_t)y * epitch + x] == 255;
    int32_t *ex = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
    int32_t *ey = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
    if (!ex || !ey) {
        free(ex);
        free(ey);
        if (dropped) *dropped = -1;
        return 0;
    }
    int64_t j = 0;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            if (edges[(size_t)y * epitch + x] == 255) {
                ex[j] = x;
                ey[j] = y;
                ++j;
            }
#pragma omp parallel for reduction(+ : cast, drop) schedule(dynamic, 1)
    for (int k = 0; k < n_theta; ++k) {
        int bits = tile_mask ? oracle_band_bits(n_theta, k) : 0xFF;
        int32_t *row = acc + (size_t)k * n_r;
        for (int64_t e = 0; e < ne; ++e) {
            int x = ex[e], y = ey[e];
            if (tile_mask && (tile_mask[(size_t)(y / 8) * tw + (x / 8)] & bits) == 0) continue;
            int64_t v = (int64_t)x * C[k] + (int64_t)y * S[k];
            int64_t r = floor_div(v + 8192, 16384);
            int64_t i = r + r_offset;
            if (i >= 0 && i < n_r) {
                row[i] += 1;
                ++cast;
            } else {
                ++drop;
            }
        }
    }
    free(ex);
    free(ey);
    if (dropped) *dropped = drop;
    return cast;
}

/* Peak extraction by greedy non-maximum suppression.
 *
 * Working copy A = acc.  Repeat up to k times:
 *   1. (t, i) = position of the largest A, first in theta-major order;
 *   2. stop if A[t][i] < max(1, min_votes);
 *   3. emit (t, i, acc[t][i]);
 *   4. set A to -1 on the window |dt| <= h_theta, |di| <= h_r around it.
 *      A row index t + dt outside [0, n_theta) wraps to (t + dt) mod n_theta;
 *      each wrap by half a turn turns the line (r, theta) into
 *      (-r, theta +- 180deg), so the window's column centre becomes the
 *      mirrored index 2*r_offset - i for an odd number of wraps.
 * Needs n_r == 2*r_offset + 1.  Outputs are padded with -1.  Returns the
 * number of peaks found, or -1 on bad arguments. */
int oracle_hough_peaks(const int32_t *acc, int n_theta, int n_r, int r_offset, int k,
                       int h_theta, int h_r, int min_votes, int32_t *theta_idx,
                       int32_t *r_idx, int32_t *votes)
{
    if (n_theta <= 0 || n_r != 2 * r_offset + 1 || k < 1 || h_theta < 0 || h_r < 0) return -1;
    size_t ncell = (size_t)n_theta * (size_t)n_r;
    int64_t *A = (int64_t *)malloc(sizeof(int64_t) * ncell);
    if (!A) return -1;
    for (size_t c = 0; c < ncell; ++c) A[c] = acc[c];
    int floor_votes = min_votes > 1 ? min_votes : 1;
    int found = 0;
    for (int j = 0; j < k; ++j) {
        theta_idx[j] = r_idx[j] = votes[j] = -1;
    }
    for (int j = 0; j < k; ++j) {
        size_t best = 0;
        for (size_t c = 1; c < ncell; ++c)
            if (A[c] > A[best]) best = c;
        if (A[best] < floor_votes) break;
        int t = (int)(best / (size_t)n_r), i = (int)(best % (size_t)n_r);
        theta_idx[j] = t;
        r_idx[j] = i;
        votes[j] = acc[best];
        ++found;
        for (int dt = -h_theta; dt <= h_theta; ++dt) {
            int64_t traw = (int64_t)t + dt;
            int64_t q = floor_div(traw, n_theta);
            int row = (int)(traw - q * n_theta);
            int centre = (q % 2 != 0) ? 2 * r_offset - i : i;
            for (int di = -h_r; di <= h_r; ++di) {
                int col = centre + di;
                if (col < 0 || col >= n_r) continue;
                A[(size_t)row * n_r + col] = -1;
            }
        }
    }
    free(A);
    return found;
}

/* Line segments along peaks.  For peak j with theta_idx t >= 0 and r_idx i:
 *   points: the 255 pixels (x, y) whose vote for bin t lands in cell i, i.e.
 *           floor((x*C[t] + y*S[t] + 2^13) / 2^14) + r_offset == i;
 *   order:  by (y, x) when |C[t]| >= |S[t]| (line nearer the vertical), else
 *           by (x, y), ascending;
 *   split:  two consecutive points more than fill_gap apart (squared
 *           distance > fill_gap^2) end one segment and start the next;
 *   keep:   a segment whose first and last point are at least min_length
 *           apart (squared distance >= min_length^2);
 *   output: segs[j][s] = (x1, y1, x2, y2), its first and last point, for the
 *           first max_seg kept segments in order; counts[j] = number kept
 *           (may exceed max_seg); npts[j] (nullable) = number of points.
 * A peak with theta_idx < 0 (padding) has no points.  Unused slots are -1.
 * Returns 0, or -1 on bad arguments. */
typedef struct { int32_t a, b, x, y; } LinePoint;

static int line_point_cmp(const void *p, const void *q)
{
    const LinePoint *u = (const LinePoint *)p, *v = (const LinePoint *)q;
    if (u->a != v->a) return u->a < v->a ? -1 : 1;
    if (u->b != v->b) return u->b < v->b ? -1 : 1;
    return 0;
}

static int64_t dist2(const LinePoint *u, const LinePoint *v)
{
    int64_t dx = (int64_t)u->x - v->x, dy = (int64_t)u->y - v->y;
    return dx * dx + dy * dy;
}

int oracle_hough_lines(const uint8_t *edges, int W, int H, int epitch, const int16_t *C,
                       const int16_t *S, int n_theta, int r_offset, const int32_t *theta_idx,
                       const int32_t *r_idx, int k, int fill_gap, int min_length, int max_seg,
                       int32_t *segs, int32_t *counts, int32_t *npts)
{
    if (W <= 0 || H <= 0 || n_theta <= 0 || k < 0 || fill_gap < 0 || min_length < 0 || max_seg < 1)
        return -1;
    LinePoint *pts = (LinePoint *)malloc(sizeof(LinePoint) * (size_t)W * (size_t)H);
    if (!pts) return -1;
    const int64_t gap2 = (int64_t)fill_gap * fill_gap, len2 = (int64_t)min_length * min_length;
    for (int j = 0; j < k; ++j) {
        for (int s = 0; s < 4 * max_seg; ++s) segs[(size_t)j * 4 * max_seg + s] = -1;
        counts[j] = 0;
        if (npts) npts[j] = 0;
        int t = theta_idx[j];
        if (t < 0 || t >= n_theta) continue;
        int by_y = abs(C[t]) >= abs(S[t]);
        size_t n = 0;
        for (int y = 0; y < H; ++y) {
            for (int x = 0; x < W; ++x) {
                if (edges[(size_t)y * epitch + x] != 255) continue;
                int64_t v = (int64_t)x * C[t] + (int64_t)y * S[t];
                if (floor_div(v + 8192, 16384) + r_offset != r_idx[j]) continue;
                pts[n].a = by_y ? y : x;
                pts[n].b = by_y ? x : y;
                pts[n].x = x;
                pts[n].y = y;
                ++n;
            }
        }
        if (npts) npts[j] = (int32_t)n;
        qsort(pts, n, sizeof(LinePoint), line_point_cmp);
        int kept = 0;
        size_t first = 0;
        for (size_t m = 1; m <= n; ++m) {
            if (m < n && dist2(&pts[m - 1], &pts[m]) <= gap2) continue;
            /* segment [first, m) */
            if (n > 0 && dist2(&pts[first], &pts[m - 1]) >= len2) {
                if (kept < max_seg) {
                    int32_t *o = segs + ((size_t)j * max_seg + kept) * 4;
                    o[0] = pts[first].x;
                    o[1] = pts[first].y;
                    o[2] = pts[m - 1].x;
                    o[3] = pts[m - 1].y;
                }
                ++kept;
            }
            first = m;
        }
        counts[j] = kept;
    }
    free(pts);
    return 0;
}

/* Canny edge detector (Sec. 7 proposes it instead of Sobel + binarization;
 * the paper gives no parameters, so this is the definition used here, all in
 * integers):
 *   blur   B = (sum over i, j in [-2, 2] of w[i] w[j] I(clamp x+i, clamp y+j)
 *          + 128) >> 8 with w = (1, 4, 6, 4, 1) (binomial, sum 256; the frame
 *          edge is replicated);
 *   grad   gx, gy: the Sobel operator of oracle_sobel_binarize applied to B,
 *          edge replicated; m = |gx| + |gy|;
 *   sector the gradient direction to the nearest multiple of 45 degrees with
 *          tan(22.5 deg) = 13573 / 2^15:
 *            32768 |gy| <= 13573 |gx|  -> along x   (neighbours (x-1,y), (x+1,y))
 *            32768 |gx| <= 13573 |gy|  -> along y   ((x,y-1), (x,y+1))
 *            else gx gy > 0            -> diagonal  ((x-1,y-1), (x+1,y+1))
 *            else                      -> anti-diag ((x+1,y-1), (x-1,y+1));
 *   thin   keep m iff m > m(first neighbour) and m >= m(second), m = 0
 *          outside the frame;
 *   class  a kept pixel with m > t_high is strong, with t_low < m <= t_high
 *          weak; with border_mode 1 the one-pixel ring is neither;
 *   link   edge = 255 for the strong pixels and the weak pixels joined to a
 *          strong one by a chain of 8-neighbouring strong or weak pixels.
 * edges[H][W] gets 0/255; mag (nullable) gets min(m, 255) of the blurred
 * image.  Returns the number of edge pixels, or -1 on bad arguments. */
static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

int64_t oracle_canny(const uint8_t *img, int W, int H, int pitch, int t_low, int t_high,
                     int border_mode, uint8_t *edges, uint8_t *mag)
{
    if (W <= 0 || H <= 0 || pitch < W || t_low < 0 || t_high < t_low) return -1;
    static const int w5[5] = {1, 4, 6, 4, 1};
    size_t n = (size_t)W * H;
    int *B = (int *)malloc(sizeof(int) * n);
    int *M = (int *)malloc(sizeof(int) * n);
    int *GX = (int *)malloc(sizeof(int) * n);
    int *GY = (int *)malloc(sizeof(int) * n);
    uint8_t *cls = (uint8_t *)malloc(n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * n);
    if (!B || !M || !GX || !GY || !cls || !queue) {
        free(B); free(M); free(GX); free(GY); free(cls); free(queue);
        return -1;
    }
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int acc = 0;
            for (int j = -2; j <= 2; ++j)
                for (int i = -2; i <= 2; ++i)
                    acc += w5[i + 2] * w5[j + 2] *
                           img[(size_t)clampi(y + j, 0, H - 1) * pitch + clampi(x + i, 0, W - 1)];
            B[(size_t)y * W + x] = (acc + 128) >> 8;
        }
#define BB(u, v) B[(size_t)clampi((v), 0, H - 1) * W + clampi((u), 0, W - 1)]
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int gx = BB(x + 1, y - 1) + 2 * BB(x + 1, y) + BB(x + 1, y + 1) - BB(x - 1, y - 1) -
                     2 * BB(x - 1, y) - BB(x - 1, y + 1);
            int gy = BB(x - 1, y + 1) + 2 * BB(x, y + 1) + BB(x + 1, y + 1) - BB(x - 1, y - 1) -
                     2 * BB(x, y - 1) - BB(x + 1, y - 1);
            size_t o = (size_t)y * W + x;
            GX[o] = gx;
            GY[o] = gy;
            M[o] = iabs(gx) + iabs(gy);
            if (mag) mag[o] = (uint8_t)(M[o] > 255 ? 255 : M[o]);
        }
#undef BB
#define MM(u, v) (((u) < 0 || (v) < 0 || (u) >= W || (v) >= H) ? 0 : M[(size_t)(v) * W + (u)])
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t o = (size_t)y * W + x;
            int ax = iabs(GX[o]), ay = iabs(GY[o]), m = M[o];
            int m1, m2;
            if ((int64_t)32768 * ay <= (int64_t)13573 * ax) {
                m1 = MM(x - 1, y); m2 = MM(x + 1, y);
            } else if ((int64_t)32768 * ax <= (int64_t)13573 * ay) {
                m1 = MM(x, y - 1); m2 = MM(x, y + 1);
            } else if ((int64_t)GX[o] * GY[o] > 0) {
                m1 = MM(x - 1, y - 1); m2 = MM(x + 1, y + 1);
            } else {
                m1 = MM(x + 1, y - 1); m2 = MM(x - 1, y + 1);
            }
            int c = 0;
            if (m > m1 && m >= m2) c = m > t_high ? 2 : (m > t_low ? 1 : 0);
            if (border_mode == 1 && (x == 0 || y == 0 || x == W - 1 || y == H - 1)) c = 0;
            cls[o] = (uint8_t)c;
            edges[o] = 0;
        }
#undef MM
    /* breadth-first search from every strong pixel through strong/weak ones */
    size_t head = 0, tail = 0;
    for (size_t o = 0; o < n; ++o)
        if (cls[o] == 2) {
            edges[o] = 255;
            queue[tail++] = (int32_t)o;
        }
    while (head < tail) {
        int o = queue[head++];
        int x = o % W, y = o / W;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int u = x + dx, v = y + dy;
                if (u < 0 || v < 0 || u >= W || v >= H) continue;
                size_t q = (size_t)v * W + u;
                if (cls[q] != 0 && edges[q] == 0) {
                    edges[q] = 255;
                    queue[tail++] = (int32_t)q;
                }
            }
    }
    int64_t count = (int64_t)tail;
    free(B); free(M); free(GX); free(GY); free(cls); free(queue);
    return count;
}

/* Progressive (coarse-to-fine) Hough transform.  The paper bases its GPU
 * vote (Sec. 4.3) on a multiresolution progressive Hough method (its
 * reference [9]) without stating one; this is the definition used here.
 * p[12] = {f, w, kc, hc_t, hc_r, minc, m_t, m_r, k, h_t, h_r, min_votes}.
 *
 *   coarse table   row c in [0, n_c), n_c = n_theta / f, is the fine row
 *                  t_c = c*f + f/2 (f divides n_theta);
 *   coarse r bins  odd width w, q = (w-1)/2: bin b = floor((r + q) / w) holds
 *                  r in [b*w - q, b*w + q], so r -> -r maps b -> -b;
 *                  Dc = floor((D + q) / w), n_rc = 2*Dc + 1, index b + Dc;
 *   coarse vote    every 255 pixel adds 1 to (c, bin of its Eq. (3) r at
 *                  row t_c); an r outside [-D, D] is not counted;
 *   coarse peaks   oracle_hough_peaks on the coarse accumulator (kc, hc_t,
 *                  hc_r, minc, r_offset Dc);
 *   windows        coarse peak j = (c, bi) opens R = f + 2*m_t fine rows
 *                  u = c*f - m_t + a (a in [0, R)) by Wc = w + 2*m_r cells
 *                  e in [0, Wc): cell (a, e) is the line at unfolded angle
 *                  row u and r = (bi - Dc)*w - q - m_r + e; its count is the
 *                  number of 255 pixels whose Eq. (3) r at fine row
 *                  t = u mod n_theta equals r, or -r when u is an odd number
 *                  of half turns away (the line (r, theta + 180) is (-r,
 *                  theta)); cells whose fine index falls outside [0, 2D]
 *                  count 0 and are never the candidate;
 *   candidate j    the window's largest count, first in (a, e) order, as the
 *                  fine cell (t, r_idx, count);
 *   final peaks    oracle_hough_peaks (k, h_t, h_r, min_votes) on a fine
 *                  accumulator that is zero except at the candidates' cells.
 * Outputs: coarse_acc [n_c][n_rc]; cpk_theta/cpk_r/cpk_votes [kc] (the
 * coarse peaks, -1 padded); windows [kc][R][Wc] (0 for absent peaks);
 * cand [kc][3] (-1 for absent peaks); theta_idx/r_idx/votes [k].
 * Returns the number of final peaks, or -1 on bad arguments. */
int oracle_hough_progressive(const uint8_t *edges, int W, int H, int epitch,
                             const int16_t *C, const int16_t *S, int n_theta, int D,
                             const int32_t *p, int32_t *coarse_acc, int32_t *cpk_theta,
                             int32_t *cpk_r, int32_t *cpk_votes, int32_t *windows,
                             int32_t *cand, int32_t *theta_idx, int32_t *r_idx, int32_t *votes)
{
    int f = p[0], w = p[1], kc = p[2], m_t = p[6], m_r = p[7], k = p[8];
    if (f < 1 || n_theta % f != 0 || w < 1 || (w % 2) == 0 || kc < 1 || k < 1 || k > kc ||
        m_t < 0 || m_r < 0 || D < 0)
        return -1;
    int q = (w - 1) / 2;
    int n_c = n_theta / f;
    int Dc = (D + q) / w;
    int n_rc = 2 * Dc + 1;
    int n_r = 2 * D + 1;
    int R = f + 2 * m_t, Wc = w + 2 * m_r;

    /* coarse vote */
    memset(coarse_acc, 0, sizeof(int32_t) * (size_t)n_c * (size_t)n_rc);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            if (edges[(size_t)y * epitch + x] != 255) continue;
            for (int c = 0; c < n_c; ++c) {
                int t = c * f + f / 2;
                int64_t r = floor_div((int64_t)x * C[t] + (int64_t)y * S[t] + 8192, 16384);
                if (r < -D || r > D) continue;
                int64_t b = floor_div(r + q, w);
                coarse_acc[(size_t)c * n_rc + (size_t)(b + Dc)] += 1;
            }
        }

    /* coarse peaks */
    int nc = oracle_hough_peaks(coarse_acc, n_c, n_rc, Dc, kc, p[3], p[4], p[5], cpk_theta, cpk_r,
                                cpk_votes);
    if (nc < 0) return -1;

    /* windows around the coarse peaks */
    memset(windows, 0, sizeof(int32_t) * (size_t)kc * (size_t)R * (size_t)Wc);
    for (int j = 0; j < kc; ++j) cand[3 * j] = cand[3 * j + 1] = cand[3 * j + 2] = -1;
    for (int j = 0; j < nc; ++j) {
        int c = cpk_theta[j];
        int64_t rlo = (int64_t)(cpk_r[j] - Dc) * w - q - m_r; /* r of cell e = 0 */
        int32_t *win = windows + (size_t)j * R * Wc;
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                if (edges[(size_t)y * epitch + x] != 255) continue;
                for (int a = 0; a < R; ++a) {
                    int64_t u = (int64_t)c * f - m_t + a;
                    int64_t h = floor_div(u, n_theta);
                    int t = (int)(u - h * n_theta);
                    int64_t r = floor_div((int64_t)x * C[t] + (int64_t)y * S[t] + 8192, 16384);
                    if (r < -D || r > D) continue;
                    int64_t ru = (h % 2 != 0) ? -r : r; /* the same line at row u */
                    int64_t e = ru - rlo;
                    if (e >= 0 && e < Wc) win[(size_t)a * Wc + (size_t)e] += 1;
                }
            }
        /* candidate: largest count in (a, e) order over cells inside [0, 2D] */
        int best = -1, bt = -1, bi = -1;
        for (int a = 0; a < R; ++a) {
            int64_t u = (int64_t)c * f - m_t + a;
            int64_t h = floor_div(u, n_theta);
            int t = (int)(u - h * n_theta);
            for (int e = 0; e < Wc; ++e) {
                int64_t ru = rlo + e;
                int64_t r = (h % 2 != 0) ? -ru : ru;
                if (r < -D || r > D) continue;
                int v = win[(size_t)a * Wc + (size_t)e];
                if (v > best) {
                    best = v;
                    bt = t;
                    bi = (int)(r + D);
                }
            }
        }
        cand[3 * j] = bt;
        cand[3 * j + 1] = bi;
        cand[3 * j + 2] = best;
    }

    /* final peaks among the candidates */
    size_t ncell = (size_t)n_theta * (size_t)n_r;
    int32_t *A = (int32_t *)calloc(ncell, sizeof(int32_t));
    if (!A) return -1;
    for (int j = 0; j < nc; ++j)
        if (cand[3 * j] >= 0 && cand[3 * j + 2] > 0)
            A[(size_t)cand[3 * j] * n_r + (size_t)cand[3 * j + 1]] = cand[3 * j + 2];
    int n = oracle_hough_peaks(A, n_theta, n_r, D, k, p[9], p[10], p[11], theta_idx, r_idx, votes);
    free(A);
    return n;
}

/* D = ceil(sqrt((W-1)^2 + (H-1)^2)) by integer search. */
int oracle_r_offset(int W, int H)
{
    int64_t q = (int64_t)(W - 1) * (W - 1) + (int64_t)(H - 1) * (H - 1);
    int64_t d = 0;
    while (d * d < q) ++d;
    return (int)d;
}
