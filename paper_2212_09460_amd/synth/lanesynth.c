/*
 * Seeded synthetic road frames and the Q14 trig table: the INPUTS shared by
 * the HIP path and the CPU oracle.  Nothing here computes any step of the
 * lane-detection method (no gradient, threshold, vote or peak); it only draws
 * pictures and tabulates cos/sin.
 *
 * The paper's own test image (a 512x512 gray road picture, Sec. 5, Fig. 9) is
 * not available, so these frames stand in for it: a noisy gray road with
 * bright straight lane bands converging to a vanishing point, optional thin
 * clutter segments and salt noise.
 *
 * Random numbers
 *   frame seed  = splitmix64 step of (base_seed ^ (config_id << 48) ^ index)
 *   stream      = xoshiro256** whose 4 state words are 4 successive
 *                 splitmix64 outputs started from the frame seed
 *   U[0,1)      = (next() >> 11) * 2^-53
 *   U{a..b}     = rejection sampling on next() (no modulo bias)
 *   N(0,1)      = Box-Muller, both outputs used, in double
 * Draw order inside one frame: scene parameters (vanishing point, lanes,
 * clutter), then background noise row-major, then clutter, lanes, salt.
 *
 * Build: plain C99, -ffp-contract=off so the double geometry is the same on
 * every x86-64 host with the same libm.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- PRNG -- */

static uint64_t sm64_next(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct { uint64_t s[4]; } xo256;

static uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t xo_next(xo256 *g)
{
    uint64_t *s = g->s;
    const uint64_t result = rotl64(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return result;
}

static void xo_seed(xo256 *g, uint64_t seed)
{
    uint64_t st = seed;
    for (int i = 0; i < 4; ++i) g->s[i] = sm64_next(&st);
}

static double u01(xo256 *g) { return (double)(xo_next(g) >> 11) * 0x1.0p-53; }

static double uab(xo256 *g, double a, double b) { return a + (b - a) * u01(g); }

/* uniform integer in [a, b] by rejection */
static int64_t uint_ab(xo256 *g, int64_t a, int64_t b)
{
    uint64_t n = (uint64_t)(b - a) + 1u;
    /* accept u < floor((2^64 - 1) / n) * n, so u % n is unbiased */
    uint64_t zone = (UINT64_MAX / n) * n;
    for (;;) {
        uint64_t u = xo_next(g);
        if (u < zone) return a + (int64_t)(u % n);
    }
}

uint64_t ls_frame_seed(uint64_t base_seed, int config_id, uint64_t index)
{
    uint64_t s = base_seed ^ ((uint64_t)(uint32_t)config_id << 48) ^ index;
    return sm64_next(&s);
}

/* ------------------------------------------------------------- drawing -- */

typedef struct {
    int W, H;
    int n_lanes;          /* straight lane bands toward the vanishing point */
    uint32_t dashed_mask; /* bit i set: lane i dashed (dash 40 px, gap 30 px) */
    int n_clutter;        /* thin random segments */
    double salt_p;        /* probability a pixel becomes 255 */
} ls_scene;

typedef struct {
    double x0, y0, x1, y1; /* segment end points, pixel-centre coordinates */
    double half_width;     /* pixels with |perpendicular distance| < this */
    int intensity;
    int dashed;
} seg_t;

/* Paint every pixel whose centre lies within the segment's band.  The
 * along-segment coordinate t (pixels from (x0,y0)) must satisfy 0 <= t <= L;
 * dashed segments are painted only where fmod(t, 70) < 40. */
static void paint_segment(uint8_t *img, int W, int H, int pitch, const seg_t *sg)
{
    double dx = sg->x1 - sg->x0, dy = sg->y1 - sg->y0;
    double L = sqrt(dx * dx + dy * dy);
    if (!(L > 0.0)) return;
    double ux = dx / L, uy = dy / L;
    double hw = sg->half_width;
    double minx = fmin(sg->x0, sg->x1) - hw - 1.0, maxx = fmax(sg->x0, sg->x1) + hw + 1.0;
    double miny = fmin(sg->y0, sg->y1) - hw - 1.0, maxy = fmax(sg->y0, sg->y1) + hw + 1.0;
    int xa = (int)floor(minx), xb = (int)ceil(maxx);
    int ya = (int)floor(miny), yb = (int)ceil(maxy);
    if (xa < 0) xa = 0;
    if (ya < 0) ya = 0;
    if (xb > W - 1) xb = W - 1;
    if (yb > H - 1) yb = H - 1;
    for (int y = ya; y <= yb; ++y) {
        for (int x = xa; x <= xb; ++x) {
            double px = (double)x - sg->x0, py = (double)y - sg->y0;
            double t = px * ux + py * uy;
            if (t < 0.0 || t > L) continue;
            double d = px * uy - py * ux;
            if (fabs(d) >= hw) continue;
            if (sg->dashed && fmod(t, 70.0) >= 40.0) continue;
            img[(size_t)y * pitch + x] = (uint8_t)sg->intensity;
        }
    }
}

/* Generate one frame into img[H][pitch].  Returns 0, or -1 on bad sizes. */
int ls_gen_frame(const ls_scene *sc, uint64_t seed, uint8_t *img, int pitch)
{
    const int W = sc->W, H = sc->H;
    if (W <= 0 || H <= 0 || pitch < W || sc->n_lanes < 0 || sc->n_lanes > 32 ||
        sc->n_clutter < 0)
        return -1;
    xo256 g;
    xo_seed(&g, seed);

    /* scene parameters */
    double vpx = W * 0.5 + uab(&g, -0.05, 0.05) * W;
    double vpy = uab(&g, 0.35, 0.45) * H;
    double spread = uab(&g, 0.25, 0.45) * W;
    seg_t lanes[32];
    for (int i = 0; i < sc->n_lanes; ++i) {
        double pos = sc->n_lanes == 1 ? 0.0 : (2.0 * i / (sc->n_lanes - 1) - 1.0);
        double xb = W * 0.5 + pos * spread;
        double yb = (double)(H - 1);
        lanes[i].x0 = xb;
        lanes[i].y0 = yb;
        lanes[i].x1 = xb + 0.9 * (vpx - xb);
        lanes[i].y1 = yb + 0.9 * (vpy - yb);
        lanes[i].half_width = 3.0;
        lanes[i].intensity = (int)uint_ab(&g, 200, 255);
        lanes[i].dashed = (sc->dashed_mask >> i) & 1u;
    }
    seg_t *clut = NULL;
    if (sc->n_clutter > 0) {
        clut = (seg_t *)malloc(sizeof(seg_t) * (size_t)sc->n_clutter);
        if (!clut) return -1;
        for (int i = 0; i < sc->n_clutter; ++i) {
            double cx = u01(&g) * W, cy = u01(&g) * H;
            double ang = u01(&g) * 3.14159265358979323846;
            double len = (double)uint_ab(&g, 10, 60);
            double hx = 0.5 * len * cos(ang), hy = 0.5 * len * sin(ang);
            clut[i].x0 = cx - hx;
            clut[i].y0 = cy - hy;
            clut[i].x1 = cx + hx;
            clut[i].y1 = cy + hy;
            clut[i].half_width = 1.0;
            clut[i].intensity = (int)uint_ab(&g, 120, 255);
            clut[i].dashed = 0;
        }
    }

    /* background: N(90, 12^2), rounded half up, clipped to 0..255 */
    {
        size_t n = (size_t)W * H, k = 0;
        while (k < n) {
            double u1 = 1.0 - u01(&g); /* (0, 1] */
            double u2 = u01(&g);
            double rad = sqrt(-2.0 * log(u1));
            double z[2] = {rad * cos(6.283185307179586476925 * u2),
                           rad * sin(6.283185307179586476925 * u2)};
            for (int j = 0; j < 2 && k < n; ++j, ++k) {
                double v = floor(90.0 + 12.0 * z[j] + 0.5);
                if (v < 0.0) v = 0.0;
                if (v > 255.0) v = 255.0;
                int y = (int)(k / (size_t)W), x = (int)(k % (size_t)W);
                img[(size_t)y * pitch + x] = (uint8_t)v;
            }
        }
    }
    for (int i = 0; i < sc->n_clutter; ++i) paint_segment(img, W, H, pitch, &clut[i]);
    for (int i = 0; i < sc->n_lanes; ++i) paint_segment(img, W, H, pitch, &lanes[i]);
    if (sc->salt_p > 0.0) {
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x)
                if (u01(&g) < sc->salt_p) img[(size_t)y * pitch + x] = 255;
    }
    free(clut);
    return 0;
}

/* Lane-line ground truth of a frame (the segments drawn), for reporting only.
 * out[i*4 + 0..3] = x0, y0, x1, y1 of lane i.  Returns the lane count. */
int ls_lane_segments(const ls_scene *sc, uint64_t seed, double *out)
{
    const int W = sc->W, H = sc->H;
    xo256 g;
    xo_seed(&g, seed);
    double vpx = W * 0.5 + uab(&g, -0.05, 0.05) * W;
    double vpy = uab(&g, 0.35, 0.45) * H;
    double spread = uab(&g, 0.25, 0.45) * W;
    for (int i = 0; i < sc->n_lanes; ++i) {
        double pos = sc->n_lanes == 1 ? 0.0 : (2.0 * i / (sc->n_lanes - 1) - 1.0);
        double xb = W * 0.5 + pos * spread, yb = (double)(H - 1);
        out[i * 4 + 0] = xb;
        out[i * 4 + 1] = yb;
        out[i * 4 + 2] = xb + 0.9 * (vpx - xb);
        out[i * 4 + 3] = yb + 0.9 * (vpy - yb);
        (void)uint_ab(&g, 200, 255);
    }
    return sc->n_lanes;
}

/* Draw a uniform integer in [a, b] from the stream of a given seed (used to
 * pick the per-frame lane count of mixed batches). */
int64_t ls_seed_uint(uint64_t seed, int64_t a, int64_t b)
{
    xo256 g;
    xo_seed(&g, seed ^ 0xA5A5A5A5A5A5A5A5ull);
    return uint_ab(&g, a, b);
}

/* One draw from U[0,1) of the stream of a seed (Poisson arrival clocks). */
void ls_seed_u01(uint64_t seed, int n, double *out)
{
    xo256 g;
    xo_seed(&g, seed);
    for (int i = 0; i < n; ++i) out[i] = u01(&g);
}

/* --------------------------------------------------------- trig table -- */

/* Q14 table: C[k] = round(cos(k*pi/n) * 2^14), S[k] = round(sin(k*pi/n) * 2^14),
 * rounding half away from zero, theta_k = k * 180deg / n for k in [0, n). */
int ls_trig_q14(int n_theta, int16_t *c, int16_t *s)
{
    if (n_theta <= 0) return -1;
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < n_theta; ++k) {
        double a = (double)k * pi / (double)n_theta;
        double cv = cos(a) * 16384.0, sv = sin(a) * 16384.0;
        double cr = cv >= 0 ? floor(cv + 0.5) : -floor(-cv + 0.5);
        double sr = sv >= 0 ? floor(sv + 0.5) : -floor(-sv + 0.5);
        c[k] = (int16_t)cr;
        s[k] = (int16_t)sr;
    }
    return 0;
}

/* -------------------------------------------------------------- CRC32 -- */

uint32_t ls_crc32(const uint8_t *p, size_t n)
{
    uint32_t crc = 0xFFFFFFFFu;
    for (size_t i = 0; i < n; ++i) {
        crc ^= p[i];
        for (int b = 0; b < 8; ++b) crc = (crc >> 1) ^ (0xEDB88320u & (0u - (crc & 1u)));
    }
    return ~crc;
}
