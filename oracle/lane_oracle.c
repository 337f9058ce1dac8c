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
 * Returns the number of votes cast into acc; *dropped gets the rest. */
int64_t oracle_hough_vote(const uint8_t *edges, int W, int H, int epitch, const int16_t *C,
                          const int16_t *S, int n_theta, int r_offset, int n_r,
                          const uint8_t *tile_mask, int32_t *acc, int64_t *dropped)
{
    int tw = (W + 7) / 8;
    int64_t cast = 0, drop = 0;
    memset(acc, 0, sizeof(int32_t) * (size_t)n_theta * (size_t)n_r);
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            if (edges[(size_t)y * epitch + x] != 255) continue;
            int m = tile_mask ? tile_mask[(size_t)(y / 8) * tw + (x / 8)] : 0xFF;
            for (int k = 0; k < n_theta; ++k) {
                if (tile_mask && (m & oracle_band_bits(n_theta, k)) == 0) continue;
                int64_t v = (int64_t)x * C[k] + (int64_t)y * S[k];
                int64_t r = floor_div(v + 8192, 16384);
                int64_t i = r + r_offset;
                if (i >= 0 && i < n_r) {
                    acc[(size_t)k * n_r + (size_t)i] += 1;
                    ++cast;
                } else {
                    ++drop;
                }
            }
        }
    }
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

/* D = ceil(sqrt((W-1)^2 + (H-1)^2)) by integer search. */
int oracle_r_offset(int W, int H)
{
    int64_t q = (int64_t)(W - 1) * (W - 1) + (int64_t)(H - 1) * (H - 1);
    int64_t d = 0;
    while (d * d < q) ++d;
    return (int)d;
}
