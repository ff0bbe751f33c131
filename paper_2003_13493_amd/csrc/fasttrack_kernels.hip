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

// Track feature f of A from its initial estimate (A.q, or zero when
// zero_init) and write the estimate, status and iteration count.
__device__ void track_feature(const fg_track_args &A, int f, bool zero_init) {
    const float fx = A.feats[2 * f], fy = A.feats[2 * f + 1];
    float tx = 0.0f, ty = 0.0f, alpha = 0.0f, beta = 0.0f;
    if (!zero_init) {
        tx = A.q[4 * f];
        ty = A.q[4 * f + 1];
        alpha = A.q[4 * f + 2];
        beta = A.q[4 * f + 3];
    }
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

__global__ void __launch_bounds__(64 * TRACK_WAVES) track_kernel(fg_track_args A) {
    // the wave's feature, provably uniform: its loads become scalar loads and
    // the tests and loops on its position become scalar branches
    const int f = __builtin_amdgcn_readfirstlane(blockIdx.x * TRACK_WAVES + (int)(threadIdx.x >> 6));
    if (f >= A.nfeat) return;   // whole waves leave together
    track_feature(A, f, false);
}

// ---------------------------------------------------------------------------
// The detect-and-track loop of many camera streams (Section III-D's tracker
// evaluation, one step per stream), with every feature list resident in
// device memory.
//
// track_batch_kernel: one wave per feature slot of every job; a slot past the
// job's live count (read from device memory) leaves at once.  Every track
// starts from a zero estimate.

// Atomic load of a counter another launch wrote (not through the scalar cache).
__device__ __forceinline__ int load_count(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(64) track_batch_kernel(const fg_fe_job *__restrict__ jobs, int njobs) {
    const int b = (int)blockIdx.x;
    // the job whose slot range holds b: the last one with feat_base <= b
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].feat_base <= b) lo = mid;
        else hi = mid - 1;
    }
    const fg_fe_job &J = jobs[lo];
    const int f = b - J.feat_base;
    if (!J.has_prev || f >= J.capacity) return;
    const int n = __builtin_amdgcn_readfirstlane(load_count(J.count));
    if (f >= n) return;
    track_feature(J.A, f, true);
}

// frontend_update_kernel: one workgroup per job, after its tracking.
//   1. the tracked features (status OK) move by their estimate and are kept
//      in order; the others are dropped;
//   2. when fewer than redetect_below remain, the cells holding a kept
//      feature are marked taken, and the strongest cell winners of the other
//      cells (score descending, then cell index ascending) are appended up to
//      the capacity, at their level-0 positions (x << level, y << level);
//   3. the live count and (tracked, redetected, live) are written.
constexpr int FE_THREADS = 256;
constexpr int FE_MAX_SCORE = 4096;   // scores are at most 4080
static_assert(FAST_MAX_TRACKS <= 1024 && FAST_MAX_GRID_CELLS <= 65536, "LDS sizes below");

// Inclusive prefix sum over the workgroup of one int per thread; `tot`
// receives the total.  Uses wave DPP scans and one LDS word per wave.
__device__ int block_scan(int v, int *wsum, int &tot) {
    int x = v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int before = 0;
    tot = 0;
#pragma unroll
    for (int w = 0; w < FE_THREADS / 64; ++w) {
        const int s = wsum[w];
        before += w < wave ? s : 0;
        tot += s;
    }
    return x + before;
}

__global__ void __launch_bounds__(FE_THREADS) frontend_update_kernel(const fg_fe_job *__restrict__ jobs) {
    __shared__ float2 kept[FAST_MAX_TRACKS];
    __shared__ uint32_t taken[FAST_MAX_GRID_CELLS / 32];
    __shared__ int hist[FE_MAX_SCORE];
    __shared__ uint32_t sel[FAST_MAX_TRACKS];
    __shared__ int wsum[FE_THREADS / 64];
    __shared__ int s_nsel, s_all, s_sstar, s_at;
    const fg_fe_job &J = jobs[blockIdx.x];
    const int tid = threadIdx.x;
    const int cap = J.capacity;
    const int n = J.has_prev ? min(load_count(J.count), cap) : 0;
    // 1. keep the tracked features, in order, at their new positions
    int live = 0;
    for (int base = 0; base < n; base += FE_THREADS) {
        const int i = base + tid;
        const bool keep = i < n && J.A.status[i] == FAST_TRACK_OK;
        float2 p = make_float2(0.0f, 0.0f);
        if (keep) p = make_float2(J.A.feats[2 * i] + J.A.q[4 * i], J.A.feats[2 * i + 1] + J.A.q[4 * i + 1]);
        int tot;
        const int incl = block_scan(keep ? 1 : 0, wsum, tot);
        if (keep) kept[live + incl - 1] = p;
        live += tot;
    }
    // every thread has read the count and the kept list is complete before
    // anyone reads the list or thread 0 rewrites the count
    __syncthreads();
    const int tracked = live;
    const bool redetect = live < J.redetect_below;
    const int ncells = J.gw * J.gh;
    int nsel = 0;
    if (redetect && live < cap) {
        // 2a. taken cells and the score histogram of the free winners
        for (int i = tid; i < (ncells + 31) / 32; i += FE_THREADS) taken[i] = 0u;
        for (int i = tid; i < FE_MAX_SCORE; i += FE_THREADS) hist[i] = 0;
        if (tid == 0) {
            s_all = 1;
            s_sstar = 1;
            s_at = 0;
            s_nsel = 0;
        }
        __syncthreads();
        for (int i = tid; i < live; i += FE_THREADS) {
            const float2 p = kept[i];
            const long cx = (long)floorf(p.x / (float)J.cell), cy = (long)floorf(p.y / (float)J.cell);
            const long c = cy * J.gw + cx;
            if (c >= 0 && c < ncells) atomicOr(&taken[c >> 5], 1u << (c & 31));
        }
        __syncthreads();
        for (int i = tid; i < ncells; i += FE_THREADS) {
            const int sc = J.slots[i].score;
            if (sc > 0 && !((taken[i >> 5] >> (i & 31)) & 1u)) atomicAdd(&hist[sc], 1);
        }
        __syncthreads();
        // 2b. the score s* at which the count of free winners from the top
        // reaches k = capacity - live: every winner above s* is taken, and the
        // first ones in cell order at s*.  Thread i sums the 16 bins from
        // score 4095 - 16 i down; a scan over threads counts from the top.
        const int k = cap - live;
        constexpr int PER = FE_MAX_SCORE / FE_THREADS;
        const int top = FE_MAX_SCORE - 1 - tid * PER;
        int mine = 0;
        for (int j = 0; j < PER; ++j) mine += hist[top - j];
        int tot;
        const int incl = block_scan(mine, wsum, tot);
        const int excl = incl - mine;
        if (tot > k && excl < k && incl >= k) {   // exactly one thread
            int acc = excl;
            for (int j = 0; j < PER; ++j) {
                const int h = hist[top - j];
                if (acc + h >= k) {
                    s_sstar = top - j;
                    s_at = k - acc;
                    s_all = 0;
                    break;
                }
                acc += h;
            }
        }
        __syncthreads();
        const bool take_all = s_all != 0;
        const int sstar = s_sstar, at = s_at;
        // 2c. gather the chosen winners' keys (score << 16 | 0xFFFF - cell):
        // every free winner above s* (or every one), and the first `at` at
        // s* in cell order
        int eq_seen = 0;
        for (int base = 0; base < ncells; base += FE_THREADS) {
            const int i = base + tid;
            int sc = 0;
            if (i < ncells) {
                sc = J.slots[i].score;
                if ((taken[i >> 5] >> (i & 31)) & 1u) sc = 0;
            }
            const bool hi = sc > 0 && (take_all || sc > sstar);
            const bool eq = !take_all && sc > 0 && sc == sstar;
            int tot;
            const int incl = block_scan(eq ? 1 : 0, wsum, tot);
            const bool pick = hi || (eq && eq_seen + incl <= at);
            eq_seen += tot;
            if (pick) {
                const int slot = atomicAdd(&s_nsel, 1);
                sel[slot] = ((uint32_t)sc << 16) | (0xFFFFu - (uint32_t)i);
            }
        }
        __syncthreads();
        nsel = s_nsel;
        // 2d. order them: bitonic sort, descending, over the next power of two
        int m = 1;
        while (m < nsel) m <<= 1;
        for (int i = nsel + tid; i < m; i += FE_THREADS) sel[i] = 0u;
        __syncthreads();
        for (int size = 2; size <= m; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int i = tid; i < m; i += FE_THREADS) {
                    const int j = i ^ stride;
                    if (j > i) {
                        const uint32_t a = sel[i], b = sel[j];
                        const bool desc = (i & size) == 0;
                        if (desc ? a < b : a > b) {
                            sel[i] = b;
                            sel[j] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
    }
    // 3. write the list back: kept features, then the new ones (the list is
    // the job's own output; the tracking arguments only read it)
    float *const feats = const_cast<float *>(J.A.feats);
    for (int i = tid; i < live; i += FE_THREADS) {
        feats[2 * i] = kept[i].x;
        feats[2 * i + 1] = kept[i].y;
    }
    for (int r = tid; r < nsel; r += FE_THREADS) {
        const int cellidx = (int)(0xFFFFu - (sel[r] & 0xFFFFu));
        const fast_feature w = J.slots[cellidx];
        feats[2 * (live + r)] = (float)((int)w.x << w.level);
        feats[2 * (live + r) + 1] = (float)((int)w.y << w.level);
    }
    if (tid == 0) {
        *J.count = live + nsel;
        J.info[0] = tracked;
        J.info[1] = redetect ? 1 : 0;
        J.info[2] = live + nsel;
        J.info[3] = 0;
    }
}

}  // namespace

hipError_t fg_launch_frontend(const fg_fe_job *jobs_dev, int njobs, int total_slots, hipStream_t s) {
    if (total_slots > 0) {
        hipLaunchKernelGGL(track_batch_kernel, dim3(total_slots), dim3(64), 0, s, jobs_dev, njobs);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(frontend_update_kernel, dim3(njobs), dim3(FE_THREADS), 0, s, jobs_dev);
    return hipGetLastError();
}

hipError_t fg_launch_track(const fg_track_args &A, hipStream_t s) {
    if (A.nfeat <= 0) return hipSuccess;
    const int blocks = (A.nfeat + TRACK_WAVES - 1) / TRACK_WAVES;
    hipLaunchKernelGGL(track_kernel, dim3(blocks), dim3(64 * TRACK_WAVES), 0, s, A);
    return hipGetLastError();
}
