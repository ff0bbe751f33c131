/* CPU oracle of the Lucas-Kanade feature tracker (TEST INFRASTRUCTURE ONLY).
 *
 * Written from Section II-E: the approximated simultaneous inverse
 * compositional Lucas-Kanade tracker over an image pyramid, estimating the
 * translation t = (tx, ty) of the translational warp W(x, t) = x + t and the
 * affine illumination (alpha, beta).  Plain loops, double precision, one
 * feature at a time.
 *
 * Readings taken where the section is silent:
 *  - samples: bilinear interpolation of the uint8 levels; a sample (x, y) is
 *    usable when 0 <= x < width-1 and 0 <= y < height-1;
 *  - template gradients: central differences of the interpolated template,
 *    (T(x+1, y) - T(x-1, y)) / 2 and likewise in y;
 *  - the patch of side S around the level position p covers p + (i - S/2,
 *    j - S/2) for i, j = 0..S-1;
 *  - level k sees the feature at f / 2^k and the translation t / 2^k, and the
 *    translation found at level k seeds level k-1 doubled (coarse to fine);
 *    alpha and beta carry over unchanged (the pyramid keeps intensities);
 *  - the approximation of the section (the appearance barely changes, so the
 *    Hessian is computed once from its starting estimate): U(x) and the
 *    Hessian of a level use the alpha in force when the level starts and stay
 *    fixed over its iterations;
 *  - the template-side increment is composed inversely: t <- t - delta t,
 *    while the appearance parameters add, alpha <- alpha + delta alpha and
 *    beta <- beta + delta beta (the error term of Section II-E carries
 *    alpha + delta alpha and beta + delta beta);
 *  - a level stops after max_iter iterations or once |delta t| < eps;
 *  - a Hessian whose Cholesky pivot falls to 1e-6 of its diagonal entry or
 *    below counts as singular and the track as lost. */
#include "lkref.h"

#include <math.h>
#include <stddef.h>

/* usable bilinear sample position (its 2x2 neighbourhood is inside) */
static int usable(const lkref_plane *p, double x, double y) {
    return x >= 0.0 && y >= 0.0 && x < (double)(p->width - 1) && y < (double)(p->height - 1);
}

/* bilinear interpolation at a usable position */
static double bilinear(const lkref_plane *p, double x, double y) {
    const double fx = floor(x), fy = floor(y);
    const int x0 = (int)fx, y0 = (int)fy;
    const double ax = x - fx, ay = y - fy;
    const uint8_t *r0 = p->data + (size_t)y0 * (size_t)p->pitch + (size_t)x0;
    const uint8_t *r1 = r0 + p->pitch;
    const double top = (1.0 - ax) * r0[0] + ax * r0[1];
    const double bottom = (1.0 - ax) * r1[0] + ax * r1[1];
    return (1.0 - ay) * top + ay * bottom;
}

/* Solve the n x n symmetric system H d = b by Cholesky; 0 on success, 1 if a
 * pivot is not clearly positive. */
static int solve_spd(int n, double H[4][4], const double *b, double *d) {
    double L[4][4] = {{0}};
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = H[i][j];
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(s > 1e-6 * H[i][i])) return 1;
                L[i][i] = sqrt(s);
            } else {
                L[i][j] = s / L[j][j];
            }
        }
    }
    double y[4];
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
        y[i] = s / L[i][i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < n; ++k) s -= L[k][i] * d[k];
        d[i] = s / L[i][i];
    }
    return 0;
}

#define MAX_PATCH 64

int lkref_track(const lkref_plane *tpl, const lkref_plane *img, int levels, const int *patch, double fx,
                double fy, const double *q_in, int mode, int max_iter, double eps, double *q_out, int *iters) {
    if (!tpl || !img || !patch || !q_in || !q_out || !iters || levels < 1 || levels > 8 || max_iter < 0 ||
        (mode & ~(LKREF_GAIN | LKREF_OFFSET)))
        return -1;
    for (int k = 0; k < levels; ++k)
        if (patch[k] < 2 || patch[k] > MAX_PATCH || (patch[k] & 1) || !tpl[k].data || !img[k].data)
            return -1;

    /* the active parameters, in the order tx, ty, alpha, beta */
    int active[4], n = 0;
    active[n++] = 0;
    active[n++] = 1;
    if (mode & LKREF_GAIN) active[n++] = 2;
    if (mode & LKREF_OFFSET) active[n++] = 3;

    double tx = q_in[0], ty = q_in[1], alpha = q_in[2], beta = q_in[3];
    int total = 0;
    double T[MAX_PATCH * MAX_PATCH], U[MAX_PATCH * MAX_PATCH][4];
    int status = LKREF_TRACKED;

    for (int k = levels - 1; k >= 0; --k) {
        const double scale = ldexp(1.0, k);
        const lkref_plane *Tk = &tpl[k], *Ik = &img[k];
        const int S = patch[k], half = S / 2;
        const double px = fx / scale, py = fy / scale;
        double tkx = tx / scale, tky = ty / scale;

        /* template patch plus the one-pixel margin of its gradients */
        if (!usable(Tk, px - half - 1, py - half - 1) || !usable(Tk, px + half, py + half)) {
            status = LKREF_TEMPLATE_OUTSIDE;
            break;
        }

        /* U(x) of Section II-E with the alpha in force at the start of the level */
        const double g = 1.0 + alpha;
        double H[4][4] = {{0}};
        for (int j = 0; j < S; ++j) {
            for (int i = 0; i < S; ++i) {
                const double x = px + (i - half), y = py + (j - half);
                const double t = bilinear(Tk, x, y);
                const double gx = 0.5 * (bilinear(Tk, x + 1, y) - bilinear(Tk, x - 1, y));
                const double gy = 0.5 * (bilinear(Tk, x, y + 1) - bilinear(Tk, x, y - 1));
                double *u = U[j * S + i];
                u[0] = g * gx;
                u[1] = g * gy;
                u[2] = t;
                u[3] = 1.0;
                T[j * S + i] = t;
                for (int a = 0; a < n; ++a)
                    for (int b = 0; b < n; ++b) H[a][b] += u[active[a]] * u[active[b]];
            }
        }

        for (int it = 0; it < max_iter; ++it) {
            if (!usable(Ik, px - half + tkx, py - half + tky) ||
                !usable(Ik, px + half - 1 + tkx, py + half - 1 + tky)) {
                status = LKREF_LOST_OUTSIDE;
                break;
            }
            /* sum over the patch of U(x) [I(W(x, t)) - (1 + alpha) T(x) - beta] */
            double rhs[4] = {0, 0, 0, 0};
            for (int j = 0; j < S; ++j) {
                for (int i = 0; i < S; ++i) {
                    const double x = px + (i - half), y = py + (j - half);
                    const double r = bilinear(Ik, x + tkx, y + tky) - (1.0 + alpha) * T[j * S + i] - beta;
                    const double *u = U[j * S + i];
                    for (int a = 0; a < n; ++a) rhs[a] += u[active[a]] * r;
                }
            }
            double d[4] = {0, 0, 0, 0};
            if (solve_spd(n, H, rhs, d)) {
                status = LKREF_SINGULAR;
                break;
            }
            ++total;
            double dq[4] = {0, 0, 0, 0};
            for (int a = 0; a < n; ++a) dq[active[a]] = d[a];
            tkx -= dq[0];
            tky -= dq[1];
            alpha += dq[2];
            beta += dq[3];
            if (dq[0] * dq[0] + dq[1] * dq[1] < eps * eps) break;
        }
        tx = tkx * scale;
        ty = tky * scale;
        if (status != LKREF_TRACKED) break;
    }
    /* a lost track reports the estimate it had reached */
    q_out[0] = tx;
    q_out[1] = ty;
    q_out[2] = alpha;
    q_out[3] = beta;
    *iters = total;
    return status;
}
