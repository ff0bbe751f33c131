/*
 * fastref.c — CPU oracle (TEST INFRASTRUCTURE ONLY; see fastref.h).
 *
 * Each function follows one passage of "Faster than FAST" (IROS 2020) and is
 * written as the plain definition: no tiling, no fusion, no lookup tables,
 * no bit tricks.  Readings taken where the paper is silent are marked READING.
 */
#include "fastref.h"

#include <stddef.h>
#include <stdlib.h>

/* The 16 points of the radius-3 Bresenham circle around the centre
 * (Section II-D), listed in cyclic order so that consecutive entries, and the
 * last and the first, are 8-neighbours.  The start point and direction do not
 * matter: any cyclic order gives the same arcs and the same sums. */
static const int CIRCLE_DX[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
static const int CIRCLE_DY[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};

static int plane_ok(const fastref_plane *p) {
    return p && p->data && p->width >= 1 && p->height >= 1 && p->pitch >= p->width;
}

static int px(const fastref_plane *p, int x, int y) {
    return p->data[(size_t)y * (size_t)p->pitch + (size_t)x];
}

/* Pyramid (Section II-B: the detector first builds subsampled copies of the
 * input; Section III-C: every level has half the resolution of the one below).
 * READING: the halving filter is the rounded 2x2 mean (a+b+c+d+2)>>2 applied to
 * the previous level (not to level 0 directly); odd trailing rows/columns are
 * dropped (floor). */
int fastref_pyr_build(fastref_plane *pyr, int levels) {
    if (!pyr || levels < 1 || levels > 8) return -1;
    for (int k = 0; k < levels; ++k) {
        if (!plane_ok(&pyr[k])) return -1;
        if (k > 0 && (pyr[k].width != pyr[k - 1].width / 2 ||
                      pyr[k].height != pyr[k - 1].height / 2))
            return -1;
    }
    for (int k = 1; k < levels; ++k) {
        const fastref_plane *src = &pyr[k - 1];
        fastref_plane *dst = &pyr[k];
        for (int y = 0; y < dst->height; ++y) {
            for (int x = 0; x < dst->width; ++x) {
                int a = px(src, 2 * x, 2 * y);
                int b = px(src, 2 * x + 1, 2 * y);
                int c = px(src, 2 * x, 2 * y + 1);
                int d = px(src, 2 * x + 1, 2 * y + 1);
                dst->data[(size_t)y * (size_t)dst->pitch + (size_t)x] =
                    (uint8_t)((a + b + c + d + 2) >> 2);
            }
        }
    }
    return 0;
}

/* Arc decision of the segment test (Section II-D): the centre is a corner when
 * a continuous arc of at least n circle pixels carries the same label.
 * READING: the arc is circular (it may wrap from the last point to the first).
 * Checked directly: try every start s and test the n positions s..s+n-1. */
int fastref_arc(uint32_t mask16, int n) {
    if (n < 1 || n > 16) return 0;
    for (int s = 0; s < 16; ++s) {
        int all = 1;
        for (int j = 0; j < n; ++j) {
            if (!((mask16 >> ((s + j) % 16)) & 1u)) { all = 0; break; }
        }
        if (all) return 1;
    }
    return 0;
}

/* Segment test and corner score at one pixel (Section II-D, Eq. (1)).
 * Labels: darker if I_p < I_c - t, brighter if I_c + t < I_p, else similar.
 * READING: brighter and darker arcs are tested separately (an arc mixing the
 * two labels does not count); pixels closer than 3 to any image edge are not
 * tested (score 0); the score is the whole-circle thresholded sum of the
 * winning side, max(sum_bright (p - c - t), sum_dark (c - p - t)), and 0 when
 * the test fails (Section II-D gives every score kind the value 0 there). */
static int outside_test_area(const fastref_plane *img, int x, int y) {
    return x < 3 || y < 3 || x > img->width - 4 || y > img->height - 4;
}

int fastref_score_at(const fastref_plane *img, int x, int y, int t, int n) {
    if (outside_test_area(img, x, y)) return 0;
    int c = px(img, x, y);
    uint32_t bright = 0, dark = 0;
    int sum_bright = 0, sum_dark = 0;
    for (int i = 0; i < 16; ++i) {
        int p = px(img, x + CIRCLE_DX[i], y + CIRCLE_DY[i]);
        if (p > c + t) {
            bright |= 1u << i;
            sum_bright += p - c - t;
        } else if (p < c - t) {
            dark |= 1u << i;
            sum_dark += c - p - t;
        }
    }
    int corner = fastref_arc(bright, n) || fastref_arc(dark, n);
    if (!corner) return 0;
    return sum_bright > sum_dark ? sum_bright : sum_dark;
}

/* Is circle point i on a continuous arc of at least n points of `mask`?
 * Direct check: some start s with i in s..s+n-1 (circularly) and all of
 * s..s+n-1 set. */
static int on_arc(uint32_t mask16, int n, int i) {
    for (int s = 0; s < 16; ++s) {
        int all = 1, covers = 0;
        for (int j = 0; j < n; ++j) {
            int q = (s + j) % 16;
            if (!((mask16 >> q) & 1u)) { all = 0; break; }
            if (q == i) covers = 1;
        }
        if (all && covers) return 1;
    }
    return 0;
}

/* The paper's other corner scores (Section II-D names three: SAD-B over the
 * whole circle, SAD-A over the contiguous arc, MT the maximum threshold for
 * which the point is still a corner).
 * READING, SAD-A: the thresholded sum of fastref_score_at restricted to the
 *   circle points that lie on a qualifying arc (a run of at least n points of
 *   one label), max over the two labels; 0 for a pixel that is not a corner.
 * READING, MT: d = the largest value such that some n consecutive circle points
 *   all differ from the centre by at least d in the same direction
 *   (brighter: p - c, darker: c - p).  The segment test with threshold t'
 *   passes exactly when d > t', so the maximum passing threshold is d - 1; the
 *   score is d (> t, at most 255) so that a corner never scores 0, and 0 if
 *   the test fails at t. */
int fastref_score_kind_at(const fastref_plane *img, int x, int y, int t, int n, int kind) {
    if (kind == FASTREF_SCORE_SADB) return fastref_score_at(img, x, y, t, n);
    if (outside_test_area(img, x, y)) return 0;
    int c = px(img, x, y);
    int v[16];
    uint32_t bright = 0, dark = 0;
    for (int i = 0; i < 16; ++i) {
        v[i] = px(img, x + CIRCLE_DX[i], y + CIRCLE_DY[i]);
        if (v[i] > c + t) bright |= 1u << i;
        else if (v[i] < c - t) dark |= 1u << i;
    }
    if (!fastref_arc(bright, n) && !fastref_arc(dark, n)) return 0;
    if (kind == FASTREF_SCORE_SADA) {
        int arc_bright = 0, arc_dark = 0;
        for (int i = 0; i < 16; ++i) {
            if (on_arc(bright, n, i)) arc_bright += v[i] - c - t;
            if (on_arc(dark, n, i)) arc_dark += c - v[i] - t;
        }
        return arc_bright > arc_dark ? arc_bright : arc_dark;
    }
    /* MT */
    int d = -256;
    for (int s = 0; s < 16; ++s) {
        int min_b = 256, min_d = 256;
        for (int j = 0; j < n; ++j) {
            int q = v[(s + j) % 16];
            if (q - c < min_b) min_b = q - c;
            if (c - q < min_d) min_d = c - q;
        }
        if (min_b > d) d = min_b;
        if (min_d > d) d = min_d;
    }
    return d > t ? d : 0;
}

int fastref_score_map_kind(const fastref_plane *img, int t, int n, int kind, uint16_t *score) {
    if (!plane_ok(img) || !score || t < 0 || t > 255 || n < 1 || n > 16) return -1;
    if (kind < FASTREF_SCORE_SADB || kind > FASTREF_SCORE_MT) return -1;
    for (int y = 0; y < img->height; ++y)
        for (int x = 0; x < img->width; ++x)
            score[(size_t)y * img->width + x] = (uint16_t)fastref_score_kind_at(img, x, y, t, n, kind);
    return 0;
}

int fastref_score_map(const fastref_plane *img, int t, int n, uint16_t *score) {
    return fastref_score_map_kind(img, t, n, FASTREF_SCORE_SADB, score);
}

/* Does candidate (sa, ia) rank above (sb, ib)?  Order: higher score first,
 * then smaller row-major index.  READING: the paper leaves NMS ties open; this
 * total order keeps exactly one pixel of any plateau of equal scores. */
static int ranks_above(int sa, long ia, int sb, long ib) {
    if (sa != sb) return sa > sb;
    return ia < ib;
}

/* Non-maxima suppression over the Moore neighbourhood of side 2r+1 (Section
 * I-B, where the paper calls the radius n; Section II-C: each thread checks
 * that its response is the maximum of its neighbourhood).  Neighbours outside
 * the map count as score 0. */
int fastref_nms_mask_radius(const uint16_t *score, int width, int height, int r, uint8_t *mask) {
    if (!score || !mask || width < 1 || height < 1 || r < 1 || r > 4) return -1;
    for (int y = 0; y < height; ++y) {
        for (int x = 0; x < width; ++x) {
            long idx = (long)y * width + x;
            int s = score[idx];
            int keep = s > 0;
            for (int dy = -r; dy <= r && keep; ++dy) {
                for (int dx = -r; dx <= r && keep; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    int qx = x + dx, qy = y + dy;
                    if (qx < 0 || qy < 0 || qx >= width || qy >= height) continue;
                    long qidx = (long)qy * width + qx;
                    if (!ranks_above(s, idx, score[qidx], qidx)) keep = 0;
                }
            }
            mask[idx] = (uint8_t)keep;
        }
    }
    return 0;
}

/* 3x3 non-maxima suppression (n = 1), the detector's default. */
int fastref_nms_mask(const uint16_t *score, int width, int height, uint8_t *mask) {
    return fastref_nms_mask_radius(score, width, height, 1, mask);
}

/* Grid-cell selection, "NMS-C" (Section II-B: one feature per cell, the one
 * with the highest score; Algorithm 1's last step) over all pyramid levels
 * with one shared grid (Section II-C: a level-k position scales up by 2^k to
 * the level-0 grid).
 * READING: cells are cell x cell level-0 pixels, partial cells at the right and
 * bottom edges are kept; ties across levels prefer the smaller level, ties
 * within a level the smaller row-major index; an empty cell gets the sentinel. */
int fastref_detect_grid_nms(const fastref_plane *pyr, int levels, int t, int n, int cell, int kind,
                            int radius, fastref_feature *out) {
    if (!pyr || !out || levels < 1 || levels > 8 || t < 0 || t > 255 || n < 1 || n > 16)
        return -1;
    if (kind < FASTREF_SCORE_SADB || kind > FASTREF_SCORE_MT || radius < 1 || radius > 4) return -1;
    if (cell < 1 || cell % (1 << (levels - 1)) != 0) return -1;
    for (int k = 0; k < levels; ++k) {
        if (!plane_ok(&pyr[k])) return -1;
        if (k > 0 && (pyr[k].width != pyr[k - 1].width / 2 ||
                      pyr[k].height != pyr[k - 1].height / 2))
            return -1;
    }
    const int W0 = pyr[0].width, H0 = pyr[0].height;
    const int gw = (W0 + cell - 1) / cell, gh = (H0 + cell - 1) / cell;
    long ncell = (long)gw * gh;
    for (long i = 0; i < ncell; ++i) {
        out[i].x = 0xFFFF;
        out[i].y = 0xFFFF;
        out[i].score = 0;
        out[i].level = 0xFF;
        out[i].reserved = 0;
    }
    for (int k = 0; k < levels; ++k) {
        const fastref_plane *img = &pyr[k];
        const int w = img->width, h = img->height;
        uint16_t *score = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)w * (size_t)h);
        uint8_t *mask = (uint8_t *)malloc((size_t)w * (size_t)h);
        if (!score || !mask) { free(score); free(mask); return -1; }
        fastref_score_map_kind(img, t, n, kind, score);
        fastref_nms_mask_radius(score, w, h, radius, mask);
        for (int y = 0; y < h; ++y) {
            for (int x = 0; x < w; ++x) {
                if (!mask[(size_t)y * w + x]) continue;
                int s = score[(size_t)y * w + x];
                long cx = ((long)x << k) / cell, cy = ((long)y << k) / cell;
                fastref_feature *f = &out[cy * gw + cx];
                int better;
                if (f->score == 0) better = 1;
                else if (s != f->score) better = s > f->score;
                else if (k != f->level) better = k < f->level;
                else better = ((long)y * w + x) < ((long)f->y * w + f->x);
                if (better) {
                    f->x = (uint16_t)x;
                    f->y = (uint16_t)y;
                    f->score = (uint16_t)s;
                    f->level = (uint8_t)k;
                    f->reserved = 0;
                }
            }
        }
        free(score);
        free(mask);
    }
    return 0;
}

int fastref_detect_grid_kind(const fastref_plane *pyr, int levels, int t, int n, int cell, int kind,
                             fastref_feature *out) {
    return fastref_detect_grid_nms(pyr, levels, t, n, cell, kind, 1, out);
}

int fastref_detect_grid(const fastref_plane *pyr, int levels, int t, int n, int cell,
                        fastref_feature *out) {
    return fastref_detect_grid_nms(pyr, levels, t, n, cell, FASTREF_SCORE_SADB, 1, out);
}
