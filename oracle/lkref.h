/* CPU oracle of the Lucas-Kanade feature tracker (TEST INFRASTRUCTURE ONLY).
 *
 * Pyramidal, approximated simultaneous inverse compositional Lucas-Kanade
 * (Section II-E): translation t = (tx, ty) (Eq. of the translational warp) with
 * affine illumination gain alpha and offset beta, in double precision.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark use
 * it; the GPU library shares no code with it. */
#ifndef LKREF_H
#define LKREF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One pyramid level in host memory: width x height uint8, row pitch in bytes. */
typedef struct {
    const uint8_t *data;
    int32_t width, height, pitch;
} lkref_plane;

/* Parameter sets of Table VI: translation always, plus the gain and/or offset. */
#define LKREF_GAIN 1
#define LKREF_OFFSET 2

/* Status of a track. */
#define LKREF_TRACKED 0
#define LKREF_TEMPLATE_OUTSIDE 1 /* a template patch (with its gradient margin) leaves a level */
#define LKREF_LOST_OUTSIDE 2     /* the warped patch left the current level */
#define LKREF_SINGULAR 3         /* the Hessian of a level is (numerically) singular */

/* Track one feature from the template pyramid `tpl` to the current pyramid
 * `img` (both `levels` levels with floor-halved sizes).
 * fx, fy:   the feature in the template, level-0 pixels (may be fractional).
 * q_in:     initial (tx, ty, alpha, beta), tx/ty in level-0 pixels.
 * mode:     LKREF_GAIN | LKREF_OFFSET bits; parameters not selected keep their
 *           input values.
 * patch:    patch side per level, even, 2..64 (16 on fine levels, 8 on coarse).
 * max_iter: iterations per level (>= 0); eps: a level stops once its step
 *           |delta t| < eps (level pixels).
 * Output: q_out (tx, ty, alpha, beta), the total number of iterations in
 * *iters.  Returns an LKREF_* status, or -1 for invalid arguments. */
int lkref_track(const lkref_plane *tpl, const lkref_plane *img, int levels, const int *patch, double fx,
                double fy, const double *q_in, int mode, int max_iter, double eps, double *q_out, int *iters);

#ifdef __cplusplus
}
#endif
#endif
