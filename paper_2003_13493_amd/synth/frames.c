/*
 * Seeded synthetic grayscale frames: the stand-in for the paper's EuRoC Machine
 * Hall camera images (Section III, evaluation), which are not available here.
 *
 * This module only synthesises input bytes.  It holds none of the detector's
 * arithmetic, so the CPU oracle and the GPU path can both be fed from it.
 *
 * Generators (published definitions, restated):
 *   - SplitMix64 (Steele, Lea, Flood 2014) expands a 64-bit seed into state;
 *   - xoshiro256** (Blackman, Vigna 2018) draws 64-bit words;
 *   - Lemire's multiply-shift method with rejection draws bounded integers;
 *   - Box-Muller turns two uniforms into two independent normals.
 *
 * Scene recipe: uniform background in [40,200]; then shapes painted in order,
 * even index an axis-aligned rectangle, odd index a triangle; an optional
 * linear brightness ramp of +-40 across the frame; then per-pixel Gaussian noise,
 * rounded half up and clamped to [0,255].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s[4]; int have_spare; double spare; } rng_t;

static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static void rng_seed(rng_t *r, uint64_t seed) {
    uint64_t x = seed;
    for (int i = 0; i < 4; ++i) r->s[i] = splitmix64(&x);
    r->have_spare = 0;
    r->spare = 0.0;
}

static inline uint64_t rotl64(uint64_t v, int k) { return (v << k) | (v >> (64 - k)); }

static uint64_t rng_next(rng_t *r) {
    uint64_t *s = r->s;
    const uint64_t out = rotl64(s[1] * 5, 7) * 9;
    const uint64_t sh = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= sh;
    s[3] = rotl64(s[3], 45);
    return out;
}

/* uniform double in [0,1) with 53 random bits */
static double rng_unit(rng_t *r) { return (double)(rng_next(r) >> 11) * (1.0 / 9007199254740992.0); }

/* uniform integer in [0, range) for 0 < range <= 2^32 (Lemire, with rejection) */
static uint32_t rng_below(rng_t *r, uint64_t range) {
    if (range <= 1) return 0;
    if (range > 0xFFFFFFFFULL) return (uint32_t)(rng_next(r) % range);
    uint32_t rg = (uint32_t)range;
    uint64_t m = (uint64_t)(uint32_t)(rng_next(r) >> 32) * rg;
    uint32_t lo = (uint32_t)m;
    if (lo < rg) {
        uint32_t thresh = (uint32_t)(-rg) % rg;
        while (lo < thresh) {
            m = (uint64_t)(uint32_t)(rng_next(r) >> 32) * rg;
            lo = (uint32_t)m;
        }
    }
    return (uint32_t)(m >> 32);
}

/* uniform integer in [lo, hi] inclusive */
static int rng_int(rng_t *r, int lo, int hi) {
    if (hi <= lo) return lo;
    return lo + (int)rng_below(r, (uint64_t)((int64_t)hi - lo + 1));
}

/* standard normal, Box-Muller, both outputs used */
static double rng_normal(rng_t *r) {
    if (r->have_spare) { r->have_spare = 0; return r->spare; }
    double u1 = 1.0 - rng_unit(r);           /* (0,1] so the log is finite */
    double u2 = rng_unit(r);
    double rad = sqrt(-2.0 * log(u1));
    double ang = 6.283185307179586 * u2;
    r->spare = rad * sin(ang);
    r->have_spare = 1;
    return rad * cos(ang);
}

static inline uint8_t clamp_round(double v) {
    double f = floor(v + 0.5);
    if (f < 0.0) return 0;
    if (f > 255.0) return 255;
    return (uint8_t)f;
}

static void paint_rect(uint8_t *img, int W, int H, int pitch, rng_t *r) {
    int wmax = W / 4 > 4 ? W / 4 : 4;
    int hmax = H / 4 > 4 ? H / 4 : 4;
    int w = rng_int(r, 4, wmax);
    int h = rng_int(r, 4, hmax);
    int x0 = rng_int(r, -(w / 2), W - 1);
    int y0 = rng_int(r, -(h / 2), H - 1);
    int v = rng_int(r, 0, 255);
    int xa = x0 < 0 ? 0 : x0, ya = y0 < 0 ? 0 : y0;
    int xb = x0 + w > W ? W : x0 + w, yb = y0 + h > H ? H : y0 + h;
    for (int y = ya; y < yb; ++y)
        memset(img + (size_t)y * pitch + xa, v, (size_t)(xb > xa ? xb - xa : 0));
}

static void paint_triangle(uint8_t *img, int W, int H, int pitch, rng_t *r) {
    double cx = rng_unit(r) * W, cy = rng_unit(r) * H;
    double rmax = (W < H ? W : H) / 6.0;
    if (rmax < 8.0) rmax = 8.0;
    double vx[3], vy[3];
    for (int i = 0; i < 3; ++i) {
        double rad = 8.0 + rng_unit(r) * (rmax - 8.0);
        double ang = 6.283185307179586 * rng_unit(r);
        vx[i] = cx + rad * cos(ang);
        vy[i] = cy + rad * sin(ang);
    }
    int v = rng_int(r, 0, 255);
    double bx0 = fmin(vx[0], fmin(vx[1], vx[2])), bx1 = fmax(vx[0], fmax(vx[1], vx[2]));
    double by0 = fmin(vy[0], fmin(vy[1], vy[2])), by1 = fmax(vy[0], fmax(vy[1], vy[2]));
    int xa = (int)floor(bx0) - 1, xb = (int)ceil(bx1) + 1;
    int ya = (int)floor(by0) - 1, yb = (int)ceil(by1) + 1;
    if (xa < 0) xa = 0;
    if (ya < 0) ya = 0;
    if (xb > W) xb = W;
    if (yb > H) yb = H;
    for (int y = ya; y < yb; ++y) {
        double py = y + 0.5;
        for (int x = xa; x < xb; ++x) {
            double px = x + 0.5;
            double e0 = (vx[1] - vx[0]) * (py - vy[0]) - (vy[1] - vy[0]) * (px - vx[0]);
            double e1 = (vx[2] - vx[1]) * (py - vy[1]) - (vy[2] - vy[1]) * (px - vx[1]);
            double e2 = (vx[0] - vx[2]) * (py - vy[2]) - (vy[0] - vy[2]) * (px - vx[2]);
            int neg = (e0 < 0) || (e1 < 0) || (e2 < 0);
            int pos = (e0 > 0) || (e1 > 0) || (e2 > 0);
            if (!(neg && pos)) img[(size_t)y * pitch + x] = (uint8_t)v;
        }
    }
}

/* Noise-free scene: background plus shapes.  Draw order: background, then
 * for each shape its geometry and fill value. */
void synth_scene(uint8_t *scene, int W, int H, int pitch, uint64_t seed, int nshapes) {
    rng_t r;
    rng_seed(&r, seed);
    int bg = rng_int(&r, 40, 200);
    for (int y = 0; y < H; ++y) memset(scene + (size_t)y * pitch, bg, (size_t)W);
    for (int i = 0; i < nshapes; ++i) {
        if ((i & 1) == 0) paint_rect(scene, W, H, pitch, &r);
        else paint_triangle(scene, W, H, pitch, &r);
    }
}

/* A full frame: scene, optional +-40 linear ramp in a seeded direction, then
 * N(0, sigma^2) noise per pixel, rounded half up and clamped.  Padding bytes
 * between width and pitch are left untouched. */
void synth_frame(uint8_t *out, int W, int H, int pitch, uint64_t seed, int nshapes,
                 double sigma, int gradient) {
    synth_scene(out, W, H, pitch, seed, nshapes);
    rng_t r;
    rng_seed(&r, seed ^ 0xA5A5A5A5DEADBEEFULL);
    double gc = 0.0, gs = 0.0;
    if (gradient) {
        double th = 6.283185307179586 * rng_unit(&r);
        double c = cos(th), s = sin(th);
        double nrm = fabs(c) + fabs(s);
        gc = 40.0 * c / nrm;
        gs = 40.0 * s / nrm;
    }
    double sx = W > 1 ? 2.0 / (W - 1) : 0.0, sy = H > 1 ? 2.0 / (H - 1) : 0.0;
    for (int y = 0; y < H; ++y) {
        uint8_t *row = out + (size_t)y * pitch;
        double v = y * sy - 1.0;
        for (int x = 0; x < W; ++x) {
            double base = row[x];
            if (gradient) base += gc * (x * sx - 1.0) + gs * v;
            double n = sigma > 0 ? sigma * rng_normal(&r) : 0.0;
            row[x] = clamp_round(base + n);
        }
    }
}

/* One camera frame from a larger resident scene: crop at (ox, oy), fresh noise. */
void synth_crop_noise(const uint8_t *scene, int SW, int SH, int spitch, int ox, int oy,
                      uint8_t *out, int W, int H, int pitch, uint64_t seed, double sigma) {
    rng_t r;
    rng_seed(&r, seed);
    for (int y = 0; y < H; ++y) {
        int sy = oy + y;
        if (sy < 0) sy = 0;
        if (sy >= SH) sy = SH - 1;
        for (int x = 0; x < W; ++x) {
            int sxx = ox + x;
            if (sxx < 0) sxx = 0;
            if (sxx >= SW) sxx = SW - 1;
            double n = sigma > 0 ? sigma * rng_normal(&r) : 0.0;
            out[(size_t)y * pitch + x] = clamp_round(scene[(size_t)sy * spitch + sxx] + n);
        }
    }
}

/* Fill padding bytes [W, pitch) of every row with seeded garbage. */
void synth_pad_garbage(uint8_t *img, int W, int H, int pitch, uint64_t seed) {
    rng_t r;
    rng_seed(&r, seed);
    for (int y = 0; y < H; ++y)
        for (int x = W; x < pitch; ++x) img[(size_t)y * pitch + x] = (uint8_t)(rng_next(&r) >> 56);
}

/* n integers uniform in [lo, hi], for drawing per-frame parameters */
void synth_ints(uint64_t seed, int n, int lo, int hi, int32_t *out) {
    rng_t r;
    rng_seed(&r, seed);
    for (int i = 0; i < n; ++i) out[i] = rng_int(&r, lo, hi);
}

/* n doubles uniform in [0, 1) */
void synth_units(uint64_t seed, int n, double *out) {
    rng_t r;
    rng_seed(&r, seed);
    for (int i = 0; i < n; ++i) out[i] = rng_unit(&r);
}

/* raw xoshiro256** words after SplitMix64 seeding (for pinning the generator) */
void synth_raw(uint64_t seed, int n, uint64_t *out) {
    rng_t r;
    rng_seed(&r, seed);
    for (int i = 0; i < n; ++i) out[i] = rng_next(&r);
}
