// Lucas-Kanade feature tracking on gfx950 (Section II-E).
//
// The pyramidal, approximated simultaneous inverse compositional tracker:
// translation t = (tx, ty) plus affine illumination (alpha, beta), with the
// steepest-descent rows U(x) = [(1+alpha) dT/dx, (1+alpha) dT/dy, T(x), 1] and
// the Hessian H = sum U U^T fixed per level at the alpha the level starts with.
//
// One wave64 per feature, as the paper assigns one warp per feature: a 16x16
// patch is 4 pixels per lane, an 8x8 patch 1 pixel per lane, so every lane
// runs the same iterations and exits the same level.  The patch-wide sums
// (the 10 entries of H once per level, the 4-vector sum of U r per
// iteration) are DPP reductions across each row of 16 lanes whose four row
// sums every lane then reads in the same order, so every lane holds the same
// value and takes identical decisions.  Arithmetic is fp32.
//
// Every sample of a patch sits at p + t + (integer offset), so all of them
// share one fractional part: positions are split into an integer base and a
// fraction in [0, 1), which keeps the bilinear weights exact to fp32 at any
// frame size and makes the border tests integer comparisons.
#include <hip/hip_runtime.h>

#include "fg_internal.h"

namespace {

// Features (waves) per workgroup.  One spreads a small feature set over the
// most compute units (100 features: 100 CUs instead of 25), which measured
// 2-3% faster than four at 100 and at 10,000 features.
constexpr int TRACK_WAVES = 1;

// v plus its DPP-permuted copy (a register move, no LDS traffic)
template <int CTRL>
__device__ __forceinline__ float dpp_add(float v) {
    const int p = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false);
    return v + __builtin_bit_cast(float, p);
}

// Sum over the wave, the same value in every lane: within each row of 16
// lanes by swapping neighbours (quad_perm 1,0,3,2 and 2,3,0,1), halves of 8
// (row_half_mirror) and halves of the row (row_mirror), then the four row
// sums read out in a fixed order.
__device__ __forceinline__ float wave_sum(float v) {
    v = dpp_add<0xB1>(v);
    v = dpp_add<0x4E>(v);
    v = dpp_add<0x141>(v);
    v = dpp_add<0x140>(v);
    const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 0));
    const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16));
    const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
    const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 48));
    return (r0 + r1) + (r2 + r3);
}

__device__ __forceinline__ float uniform(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// Bilinear sample at integer base (x0, y0) plus the shared fraction (ax, ay).
__device__ __forceinline__ float bilinear(const uint8_t *p, int pitch, int x0, int y0, float ax, float ay) {
    const uint8_t *r0 = p + (ptrdiff_t)y0 * pitch + x0;
    const float a = r0[0], b = r0[1], c = r0[pitch], d = r0[pitch + 1];
    const float top = (1.0f - ax) * a + ax * b;
    const float bottom = (1.0f - ax) * c + ax * d;
    return (1.0f - ay) * top + ay * bottom;
}

// A position split into an integer part and a fraction in [0, 1).
struct Split {
    int i;
    float f;
};

__device__ __forceinline__ Split split(int base, float frac_plus) {
    const float fl = floorf(frac_plus);
    return Split{base + (int)fl, frac_plus - fl};
}

template <int S>
__device__ void track_level(const fg_track_args &A, int k, float pxf, int pxi, float pyf, int pyi, float &tkx,
                            float &tky, float &alpha, float &beta, int &total, int &status) {
    constexpr int NP = S * S / 64;   // pixels per lane
    constexpr int HALF = S / 2;
    const int lane = threadIdx.x & 63;
    const uint8_t *T = A.tpl[k];
    const uint8_t *I = A.img[k];
    const int tp = A.tpitch[k], ip = A.ipitch[k], W = A.w[k], H = A.h[k];

    // template patch plus the gradient margin: x in [p-HALF-1, p+HALF] usable
    if (pxi - HALF - 1 < 0 || pyi - HALF - 1 < 0 || pxi + HALF > W - 2 || pyi + HALF > H - 2) {
        status = FAST_TRACK_TEMPLATE_OUTSIDE;
        return;
    }
    const float g = 1.0f + alpha;
    float tv[NP], ux[NP], uy[NP];
    float h00 = 0, h01 = 0, h02 = 0, h03 = 0, h11 = 0, h12 = 0, h13 = 0, h22 = 0, h23 = 0, h33 = 0;
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        const int pix = lane + 64 * m;
        const int ox = pix % S - HALF, oy = pix / S - HALF;
        const int x0 = pxi + ox, y0 = pyi + oy;
        const float t = bilinear(T, tp, x0, y0, pxf, pyf);
        const float gx = 0.5f * (bilinear(T, tp, x0 + 1, y0, pxf, pyf) - bilinear(T, tp, x0 - 1, y0, pxf, pyf));
        const float gy = 0.5f * (bilinear(T, tp, x0, y0 + 1, pxf, pyf) - bilinear(T, tp, x0, y0 - 1, pxf, pyf));
        tv[m] = t;
        ux[m] = g * gx;
        uy[m] = g * gy;
        h00 += ux[m] * ux[m];
        h01 += ux[m] * uy[m];
        h02 += ux[m] * t;
        h03 += ux[m];
        h11 += uy[m] * uy[m];
        h12 += uy[m] * t;
        h13 += uy[m];
        h22 += t * t;
        h23 += t;
        h33 += 1.0f;
    }
    const bool gain = A.mode & FAST_TRACK_GAIN, offset = A.mode & FAST_TRACK_OFFSET;
    // Inactive parameters get an identity row and column and a zero right-hand
    // side, so their increment is 0 and the active block factors as it would
    // on its own.
    float M[4][4];
    M[0][0] = wave_sum(h00);
    M[1][0] = wave_sum(h01);
    M[1][1] = wave_sum(h11);
    M[2][0] = gain ? wave_sum(h02) : 0.0f;
    M[2][1] = gain ? wave_sum(h12) : 0.0f;
    M[2][2] = gain ? wave_sum(h22) : 1.0f;
    M[3][0] = offset ? wave_sum(h03) : 0.0f;
    M[3][1] = offset ? wave_sum(h13) : 0.0f;
    M[3][2] = gain && offset ? wave_sum(h23) : 0.0f;
    M[3][3] = offset ? wave_sum(h33) : 1.0f;
    // Cholesky factor, with the reciprocals of its diagonal kept so the
    // per-iteration solve has no divisions; singular when a pivot falls to
    // 1e-6 of its diagonal entry
    float L[4][4] = {}, inv[4];
    bool singular = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            float s = M[i][j];
#pragma unroll
            for (int q = 0; q < j; ++q) s -= L[i][q] * L[j][q];
            if (i == j) {
                singular |= !(s > 1e-6f * M[i][i]);
                L[i][i] = sqrtf(fmaxf(s, 0.0f));
                inv[i] = L[i][i] > 0.0f ? 1.0f / L[i][i] : 0.0f;
            } else {
                L[i][j] = s * inv[j];
            }
        }
    }

    for (int it = 0; it < A.max_iter; ++it) {
        // a non-finite or huge estimate is outside (keeps the integer parts small)
        if (!(fabsf(pxf + tkx) < 65536.0f && fabsf(pyf + tky) < 65536.0f)) {
            status = FAST_TRACK_LOST_OUTSIDE;
            return;
        }
        const Split sx = split(pxi, pxf + tkx), sy = split(pyi, pyf + tky);
        // warped patch: x in [p+t-HALF, p+t+HALF-1] usable
        if (sx.i - HALF < 0 || sy.i - HALF < 0 || sx.i + HALF - 1 > W - 2 || sy.i + HALF - 1 > H - 2) {
            status = FAST_TRACK_LOST_OUTSIDE;
            return;
        }
        float b0 = 0, b1 = 0, b2 = 0, b3 = 0;
#pragma unroll
        for (int m = 0; m < NP; ++m) {
            const int pix = lane + 64 * m;
            const int ox = pix % S - HALF, oy = pix / S - HALF;
            const float r = bilinear(I, ip, sx.i + ox, sy.i + oy, sx.f, sy.f) - (1.0f + alpha) * tv[m] - beta;
            b0 += ux[m] * r;
            b1 += uy[m] * r;
            b2 += tv[m] * r;
            b3 += r;
        }
        if (singular) {
            status = FAST_TRACK_SINGULAR;
            return;
        }
        float rhs[4] = {wave_sum(b0), wave_sum(b1), gain ? wave_sum(b2) : 0.0f, offset ? wave_sum(b3) : 0.0f};
        float y[4], d[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float s = rhs[i];
#pragma unroll
            for (int q = 0; q < i; ++q) s -= L[i][q] * y[q];
            y[i] = s * inv[i];
        }
#pragma unroll
        for (int i = 3; i >= 0; --i) {
            float s = y[i];
#pragma unroll
            for (int q = i + 1; q < 4; ++q) s -= L[q][i] * d[q];
            d[i] = s * inv[i];
        }
        ++total;
        tkx = uniform(tkx - d[0]);
        tky = uniform(tky - d[1]);
        alpha = uniform(alpha + d[2]);
        beta = uniform(beta + d[3]);
        if (d[0] * d[0] + d[1] * d[1] < A.eps * A.eps) break;
    }
}

__global__ void __launch_bounds__(64 * TRACK_WAVES) track_kernel(fg_track_args A) {
    // the wave's feature, provably uniform: its loads become scalar loads and
    // the tests and loops on its position become scalar branches
    const int f = __builtin_amdgcn_readfirstlane(blockIdx.x * TRACK_WAVES + (int)(threadIdx.x >> 6));
    if (f >= A.nfeat) return;   // whole waves leave together
    const float fx = A.feats[2 * f], fy = A.feats[2 * f + 1];
    float tx = A.q[4 * f], ty = A.q[4 * f + 1], alpha = A.q[4 * f + 2], beta = A.q[4 * f + 3];
    int total = 0, status = FAST_TRACK_OK;
    for (int k = A.levels - 1; k >= 0; --k) {
        const float scale = ldexpf(1.0f, k);
        const float px = fx / scale, py = fy / scale;   // exact: a power-of-two divide
        if (!(px >= 0.0f && py >= 0.0f && px < 65536.0f && py < 65536.0f)) {   // also NaN
            status = FAST_TRACK_TEMPLATE_OUTSIDE;
            break;
        }
        const float pxfl = floorf(px), pyfl = floorf(py);
        const int pxi = (int)pxfl, pyi = (int)pyfl;
        const float pxf = px - pxfl, pyf = py - pyfl;
        float tkx = tx / scale, tky = ty / scale;
        if (k < 2)
            track_level<16>(A, k, pxf, pxi, pyf, pyi, tkx, tky, alpha, beta, total, status);
        else
            track_level<8>(A, k, pxf, pxi, pyf, pyi, tkx, tky, alpha, beta, total, status);
        if (status == FAST_TRACK_TEMPLATE_OUTSIDE) break;
        tx = tkx * scale;
        ty = tky * scale;
        if (status != FAST_TRACK_OK) break;
    }
    if ((threadIdx.x & 63) == 0) {
        A.q[4 * f] = tx;
        A.q[4 * f + 1] = ty;
        A.q[4 * f + 2] = alpha;
        A.q[4 * f + 3] = beta;
        A.status[f] = status;
        if (A.iters) A.iters[f] = total;
    }
}

}  // namespace

hipError_t fg_launch_track(const fg_track_args &A, hipStream_t s) {
    if (A.nfeat <= 0) return hipSuccess;
    const int blocks = (A.nfeat + TRACK_WAVES - 1) / TRACK_WAVES;
    hipLaunchKernelGGL(track_kernel, dim3(blocks), dim3(64 * TRACK_WAVES), 0, s, A);
    return hipGetLastError();
}
