/*
 * fastref — the CPU oracle for the FAST pyramid / NMS / grid-cell detector.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded C
 * implementation of what the detector computes, written from the definitions in
 * "Faster than FAST: GPU-Accelerated Frontend for High-Speed VIO" (Nagy, Foehn,
 * Scaramuzza, IROS 2020).  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header, table
 * or helper with the GPU library, and the product path never calls it.
 *
 * All arithmetic is exact integer arithmetic on uint8 images.
 * All pointers are host pointers owned by the caller.
 */
#ifndef FASTREF_H
#define FASTREF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    uint8_t *data;   /* row-major, row y starts at data + y*pitch */
    int32_t width;
    int32_t height;
    int32_t pitch;   /* bytes per row, >= width */
} fastref_plane;

typedef struct {
    uint16_t x, y;       /* level-local coordinates */
    uint16_t score;      /* corner score, >= 1 for a real feature */
    uint8_t level;       /* pyramid level the feature was found on */
    uint8_t reserved;    /* always 0 */
} fastref_feature;       /* empty cell: x = y = 0xFFFF, score 0, level 0xFF */

/* Status codes: 0 success, -1 invalid argument. */

/* Image pyramid (Section II-B; stage list of Section III-C): level k+1 halves
 * level k by the rounded 2x2 mean (a+b+c+d+2)>>2, successively from level k.
 * pyr[0] is the input; pyr[1..levels-1] must have floor-halved sizes and are
 * written.  Returns 0 or -1. */
int fastref_pyr_build(fastref_plane *pyr, int levels);

/* The contiguous-arc decision of the segment test (Section II-D): nonzero iff the
 * 16-bit circular mask holds a run of at least n consecutive set bits, 1<=n<=16. */
int fastref_arc(uint32_t mask16, int n);

/* Corner score of one pixel (Section II-D, Eq. (1)): 0 if (x,y) lies in the
 * 3-pixel border or fails the segment test with threshold t and arc length n;
 * otherwise max(sum over brighter circle pixels of (p-c-t), sum over darker
 * circle pixels of (c-p-t)). */
int fastref_score_at(const fastref_plane *img, int x, int y, int t, int n);

/* Score map of a whole plane: score[y*width + x], zeros in the border. */
int fastref_score_map(const fastref_plane *img, int t, int n, uint16_t *score);

/* Corner score kinds (Section II-D names three).  SADB is the score above.
 * SADA: the same thresholded sums over only the circle points on a continuous
 * arc of at least n points of one label.  MT: the largest d such that n
 * consecutive circle points all differ from the centre by at least d in one
 * direction (the test at threshold t' passes iff d > t'); the score is d, or 0
 * when the test fails at t. */
enum { FASTREF_SCORE_SADB = 0, FASTREF_SCORE_SADA = 1, FASTREF_SCORE_MT = 2 };

/* fastref_score_at / fastref_score_map with a score kind; -1 for a bad kind. */
int fastref_score_kind_at(const fastref_plane *img, int x, int y, int t, int n, int kind);
int fastref_score_map_kind(const fastref_plane *img, int t, int n, int kind, uint16_t *score);

/* 3x3 non-maxima suppression (Section I-B, n=1) of a width x height score map:
 * mask[y*width+x] = 1 iff score > 0 and the pixel beats all 8 neighbours by
 * (score descending, row-major index ascending). */
int fastref_nms_mask(const uint16_t *score, int width, int height, uint8_t *mask);

/* Grid-cell selection across levels (Section II-B and II-C, Algorithm 1):
 * pyr[0..levels-1] must already hold the pyramid.  out has ceil(W/cell) *
 * ceil(H/cell) slots, row-major; each holds the NMS survivor of greatest
 * (score, -level, -row-major index) whose level-0 position (x<<k, y<<k) falls
 * in the cell, or the empty sentinel. */
int fastref_detect_grid(const fastref_plane *pyr, int levels, int t, int n, int cell,
                        fastref_feature *out);

/* fastref_detect_grid with a score kind. */
int fastref_detect_grid_kind(const fastref_plane *pyr, int levels, int t, int n, int cell, int kind,
                             fastref_feature *out);

/* Non-maxima suppression over the (2r+1) x (2r+1) Moore neighbourhood, 1 <= r <= 4
 * (Section I-B; fastref_nms_mask is r = 1), same tie rule. */
int fastref_nms_mask_radius(const uint16_t *score, int width, int height, int r, uint8_t *mask);

/* fastref_detect_grid_kind with NMS over (2r+1) x (2r+1) neighbourhoods. */
int fastref_detect_grid_nms(const fastref_plane *pyr, int levels, int t, int n, int cell, int kind,
                            int radius, fastref_feature *out);

#ifdef __cplusplus
}
#endif
#endif
