// Device code of libfastgrid: pyramid, FAST score, 3x3 NMS and per-cell
// arg-max over all pyramid levels ("Faster than FAST", Sections II-B to II-D).
//
// Work decomposition: a workgroup owns a square region of whole grid cells.
// For every level it walks the region's level-k footprint in sub-tiles,
// stages each sub-tile (plus a 4-pixel halo: 3 for the circle, 1 for the NMS
// neighbours) in LDS, scores it, suppresses non-maxima, and folds survivors
// into one 32-bit key per cell with an LDS atomicMax.  The key orders
// candidates by (score desc, level asc, row-major index asc), so a single max
// is the cell's answer, independent of the order threads arrive in.
#include "fg_internal.h"

namespace {

constexpr int SUB = 64;                 // sub-tile side (level-k pixels)
constexpr int HALO = 4;                 // 3 (circle) + 1 (NMS neighbour)
constexpr int TILE_W = SUB + 2 * HALO;  // 72
constexpr int TILE_P = 80;              // LDS row pitch of the pixel tile
constexpr int SC_W = SUB + 2;           // scores: sub-tile plus 1-pixel ring
constexpr int SC_P = 68;
constexpr int MAX_RCELLS = 32;          // cells per region side
constexpr int MAX_KEYS = MAX_RCELLS * MAX_RCELLS;

// Circle of radius 3 (Section II-D), cyclic order.
__constant__ int8_t c_dx[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
__constant__ int8_t c_dy[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};

// Circular run of >= n set bits in a 16-bit mask: AND shifted copies of the
// doubled mask, doubling the covered length each step.
__device__ __forceinline__ bool has_arc(uint32_t m, int n) {
    uint32_t r = m | (m << 16);
    int have = 1;
    while (have * 2 <= n) {
        r &= r >> have;
        have *= 2;
    }
    if (have < n) r &= r >> (n - have);
    return (r & 0xFFFFu) != 0;
}

// Score of the pixel at tile position (lx, ly); caller guarantees the 7x7
// stencil lies inside the tile and the pixel is outside the 3-pixel border.
__device__ __forceinline__ uint32_t fast_score(const uint8_t *tile, int lx, int ly, int t,
                                               int n) {
    const int c = tile[ly * TILE_P + lx];
    const int hi = c + t, lo = c - t;
    uint32_t bm = 0, dm = 0;
    int sb = 0, sd = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int p = tile[(ly + c_dy[i]) * TILE_P + lx + c_dx[i]];
        const int db = p - hi, dd = lo - p;
        bm |= (db > 0 ? 1u : 0u) << i;
        dm |= (dd > 0 ? 1u : 0u) << i;
        sb += db > 0 ? db : 0;
        sd += dd > 0 ? dd : 0;
    }
    if (!has_arc(bm, n) && !has_arc(dm, n)) return 0;
    return (uint32_t)(sb > sd ? sb : sd);
}

// Cell key: (score << 19) | ((7 - level) << 16) | (0xFFFF - local index).
__device__ __forceinline__ uint32_t make_key(uint32_t score, int level, uint32_t local) {
    return (score << 19) | ((uint32_t)(7 - level) << 16) | (0xFFFFu - local);
}

__device__ void detect_region(const fg_job &J, int region, uint8_t *tile, uint16_t *sc,
                              uint32_t *keys) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int rxi = region % J.rx, ryi = region / J.rx;
    const int ncx = min(J.rcells, J.gw - rxi * J.rcells);
    const int ncy = min(J.rcells, J.gh - ryi * J.rcells);
    for (int i = tid; i < ncx * ncy; i += nthr) keys[i] = 0;

    for (int k = 0; k < J.levels; ++k) {
        const int W = J.w[k], H = J.h[k], P = J.pitch[k];
        const uint8_t *img = J.lvl[k];
        const int cw = J.cell >> k;
        const int x0 = rxi * J.rcells * cw, y0 = ryi * J.rcells * cw;
        const int x1 = min(x0 + ncx * cw, W), y1 = min(y0 + ncy * cw, H);
        for (int sy = y0; sy < y1; sy += SUB) {
            for (int sx = x0; sx < x1; sx += SUB) {
                const int ex = min(sx + SUB, x1), ey = min(sy + SUB, y1);
                const int tw = ex - sx + 2 * HALO, th = ey - sy + 2 * HALO;
                __syncthreads();
                for (int i = tid; i < tw * th; i += nthr) {
                    const int lx = i % tw, ly = i / tw;
                    const int gx = sx - HALO + lx, gy = sy - HALO + ly;
                    uint8_t v = 0;
                    if (gx >= 0 && gx < W && gy >= 0 && gy < H) v = img[(size_t)gy * P + gx];
                    tile[ly * TILE_P + lx] = v;
                }
                __syncthreads();
                const int sw = ex - sx + 2, sh = ey - sy + 2;
                for (int i = tid; i < sw * sh; i += nthr) {
                    const int lx = i % sw, ly = i / sw;
                    const int gx = sx - 1 + lx, gy = sy - 1 + ly;
                    uint32_t s = 0;
                    if (gx >= 3 && gx <= W - 4 && gy >= 3 && gy <= H - 4)
                        s = fast_score(tile, lx + HALO - 1, ly + HALO - 1, J.t, J.n);
                    sc[ly * SC_P + lx] = (uint16_t)s;
                }
                __syncthreads();
                const int iw = ex - sx, ih = ey - sy;
                for (int i = tid; i < iw * ih; i += nthr) {
                    const int lx = i % iw, ly = i / iw;
                    const uint16_t *c = sc + (ly + 1) * SC_P + (lx + 1);
                    const uint32_t s = c[0];
                    if (s == 0) continue;
                    // earlier neighbours in row-major order must be strictly
                    // lower; later ones lower or equal
                    const bool keep = s > c[-SC_P - 1] && s > c[-SC_P] && s > c[-SC_P + 1] &&
                                      s > c[-1] && s >= c[1] && s >= c[SC_P - 1] &&
                                      s >= c[SC_P] && s >= c[SC_P + 1];
                    if (!keep) continue;
                    const int gx = sx + lx, gy = sy + ly;
                    const int ox = gx - x0, oy = gy - y0;
                    const int ci = (oy / cw) * ncx + (ox / cw);
                    const uint32_t local = (uint32_t)((oy % cw) * cw + (ox % cw));
                    atomicMax(&keys[ci], make_key(s, k, local));
                }
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < ncx * ncy; i += nthr) {
        const int cx = rxi * J.rcells + i % ncx, cy = ryi * J.rcells + i / ncx;
        const uint32_t key = keys[i];
        fast_feature f;
        if (key == 0) {
            f.x = 0xFFFF;
            f.y = 0xFFFF;
            f.score = 0;
            f.level = 0xFF;
        } else {
            const int level = 7 - (int)((key >> 16) & 7u);
            const uint32_t local = 0xFFFFu - (key & 0xFFFFu);
            const int cw = J.cell >> level;
            f.x = (uint16_t)(((cx * J.cell) >> level) + (int)(local % (uint32_t)cw));
            f.y = (uint16_t)(((cy * J.cell) >> level) + (int)(local / (uint32_t)cw));
            f.score = (uint16_t)(key >> 19);
            f.level = (uint8_t)level;
        }
        f.reserved = 0;
        J.out[(size_t)cy * J.gw + cx] = f;
    }
}

// Bijective block -> item map that gives each XCD (blocks are dealt to the 8
// XCDs round-robin) a contiguous run of items, so neighbouring regions share
// halo lines in the same L2.
__device__ __forceinline__ int xcd_item(int b, int n) {
    const int q = n >> 3, r = n & 7;
    const int xcd = b & 7, local = b >> 3;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

__global__ void __launch_bounds__(1024) detect_plain_kernel(fg_job J) {
    __shared__ uint8_t tile[TILE_W * TILE_P];
    __shared__ uint16_t sc[SC_W * SC_P];
    __shared__ uint32_t keys[MAX_KEYS];
    detect_region(J, xcd_item(blockIdx.x, gridDim.x), tile, sc, keys);
}

__global__ void __launch_bounds__(1024) detect_batch_kernel(const fg_job *__restrict__ jobs,
                                                            int njobs, int total,
                                                            unsigned *counter) {
    __shared__ uint8_t tile[TILE_W * TILE_P];
    __shared__ uint16_t sc[SC_W * SC_P];
    __shared__ uint32_t keys[MAX_KEYS];
    __shared__ int s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(&counter[0], 1u);
        __syncthreads();
        const int item = s_item;
        if (item >= total) break;
        int lo = 0, hi = njobs - 1;   // last job with region_base <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].region_base <= item) lo = mid;
            else hi = mid - 1;
        }
        const fg_job J = jobs[lo];
        detect_region(J, item - J.region_base, tile, sc, keys);
    }
    // The last workgroup out re-arms the queue for the next launch.
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned done = atomicAdd(&counter[1], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&counter[0], 0u);
            atomicExch(&counter[1], 0u);
        }
    }
}

// Pyramid level k from level k-1 (one output pixel per thread).
__global__ void pyr_kernel(const uint8_t *__restrict__ src, int sp, uint8_t *__restrict__ dst,
                           int dw, int dh, int dp) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (x >= dw || y >= dh) return;
    const uint8_t *r0 = src + (size_t)(2 * y) * sp + 2 * x;
    const uint8_t *r1 = r0 + sp;
    dst[(size_t)y * dp + x] = (uint8_t)((r0[0] + r0[1] + r1[0] + r1[1] + 2) >> 2);
}

__global__ void pyr_batch_kernel(const fg_job *__restrict__ jobs, int k) {
    const fg_job &J = jobs[blockIdx.z];
    if (k >= J.levels) return;
    const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    const int dw = J.w[k], dh = J.h[k];
    if (x >= dw || y >= dh) return;
    const int sp = J.pitch[k - 1];
    const uint8_t *r0 = J.lvl[k - 1] + (size_t)(2 * y) * sp + 2 * x;
    const uint8_t *r1 = r0 + sp;
    J.lvl[k][(size_t)y * J.pitch[k] + x] = (uint8_t)((r0[0] + r0[1] + r1[0] + r1[1] + 2) >> 2);
}

}  // namespace

void fg_job_layout(fg_job &j, const fg_launch &L) {
    j.gw = (j.w[0] + j.cell - 1) / j.cell;
    j.gh = (j.h[0] + j.cell - 1) / j.cell;
    int rc = L.region / j.cell;
    if (rc < 1) rc = 1;
    if (rc > MAX_RCELLS) rc = MAX_RCELLS;
    j.rcells = rc;
    j.rx = (j.gw + rc - 1) / rc;
    j.ry = (j.gh + rc - 1) / rc;
}

hipError_t fg_launch_pyramid(const fg_job &j, hipStream_t s) {
    for (int k = 1; k < j.levels; ++k) {
        dim3 grid((j.w[k] + 255) / 256, j.h[k]);
        hipLaunchKernelGGL(pyr_kernel, grid, dim3(256), 0, s, j.lvl[k - 1], j.pitch[k - 1],
                           j.lvl[k], j.w[k], j.h[k], j.pitch[k]);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t fg_launch_plain(const fg_job &j, const fg_launch &L, hipStream_t s) {
    hipError_t e = fg_launch_pyramid(j, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(detect_plain_kernel, dim3(j.rx * j.ry), dim3(L.block), 0, s, j);
    return hipGetLastError();
}

hipError_t fg_launch_batch(const fg_job *jobs_dev, int njobs, int total, int max_levels,
                           int max_w1, int max_h1, unsigned *counter, const fg_launch &L,
                           hipStream_t s) {
    int mw = max_w1, mh = max_h1;
    for (int k = 1; k < max_levels; ++k) {
        dim3 grid((mw + 255) / 256, mh, njobs);
        hipLaunchKernelGGL(pyr_batch_kernel, grid, dim3(256), 0, s, jobs_dev, k);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        mw = (mw >> 1) > 0 ? (mw >> 1) : 1;
        mh = (mh >> 1) > 0 ? (mh >> 1) : 1;
    }
    int blocks = L.num_cu * L.blocks_per_cu;
    if (blocks > total) blocks = total;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(detect_batch_kernel, dim3(blocks), dim3(L.block), 0, s, jobs_dev, njobs,
                       total, counter);
    return hipGetLastError();
}
