// Device code of libfastgrid: pyramid, FAST score, 3x3 NMS and per-cell
// arg-max over all pyramid levels ("Faster than FAST", Sections II-B to II-D).
//
// Work decomposition
// ------------------
// A workgroup owns a region of whole grid cells (a multiple of 16 level-0
// pixels wide and tall) and walks it in 64x64 level-0 sub-tiles.  For pyramids
// of up to 3 levels the sub-tile is loaded once with a 4*2^(L-1)-pixel halo and
// the deeper levels are built from it in LDS (one pass over HBM: level 0 read
// once, levels 1.. written once).  Deeper pyramids are built by a separate
// kernel and each level's sub-tile is loaded with a 4-pixel halo.
//
// Detection of a sub-tile scores every pixel of its area plus a 1-pixel ring
// at every level:
//
//   P1 compass test, 8 pixels per lane in packed 16-bit lanes.  An arc of N
//      circle pixels contains floor(N/4) consecutive compass points (circle
//      indices 0, 4, 8, 12) of its label.  The 8-pixel groups of all levels
//      are dealt to the waves round-robin in rounds of 64.
//   P2 compaction of the survivors into a wave-private LDS list (ballot +
//      mbcnt over groups, then a DPP prefix scan over pixels).
//   P3 8-point test, one survivor per lane: the arc also contains floor(N/2)
//      consecutive even circle points of its label.  In-place compaction.
//   P4 full segment test and score (Section II-D, Eq. (1)) into the level's
//      score map (the sub-tile area plus its ring).
//   P5 after one workgroup barrier, 3x3 NMS (Section I-B, n=1) of the
//      sub-tile's own pixels and an LDS atomicMax of a 32-bit key per cell:
//      (score << 19) | ((7-level) << 16) | (0xFFFF - row-major index inside
//      the cell), which orders candidates by (score desc, level asc, index
//      asc), so the cell's answer does not depend on thread order.
//
// P1-P4 need no workgroup barrier.  Both filters are necessary conditions of
// the segment test, so a pixel they reject has score 0; the cascade never
// changes a result.
#include <type_traits>

#include "fg_internal.h"

namespace {

constexpr int SUB = FG_SUB;             // sub-tile side at level 0
constexpr int MAX_FUSED = FG_MAX_FUSED;   // levels built in LDS from one load

// All level tiles share one LDS row pitch, so circle offsets are constants.
// Band A (rows 0..95): level 0 of a fused sub-tile, or the current level of an
// unfused one.  Band B (rows 96..143): level 1 at byte 8, level 2 at byte 68.
// For a sub-tile whose origin is a multiple of 16 pixels, the compass groups
// of every level then start 4 bytes past a multiple of 8, so the row words
// around a group are two aligned 8-byte reads (load8<true>).
constexpr int LP = 112;
constexpr int T0 = 16;
constexpr int T1 = 96 * LP + 8;
constexpr int T2 = 96 * LP + 68;
constexpr int TILE_BYTES = 144 * LP;
static_assert(T0 % 16 == 0 && LP % 16 == 0, "16-byte tile stores in band A");
static_assert(T1 % 8 == 0 && T2 % 4 == 0, "8-byte reads when halving level 1");
static_assert(LP % 8 == 0 && T0 % 8 == 0 && T1 % 8 == 0 && T2 % 8 == 4, "aligned compass row reads");
static_assert(TILE_BYTES <= 16384, "entries hold 14-bit LDS offsets");
// Score maps: a level's sub-tile area plus a 1-pixel ring.
constexpr int M0_ROWS = SUB + 2, M0_P = SUB + 4;
constexpr int M1_ROWS = SUB / 2 + 2, M1_P = M0_P;
constexpr int M2_ROWS = SUB / 4 + 2, M2_P = M0_P;
constexpr int MP = M0_P;   // one pitch for every level's score map
constexpr int MAX_RCELLS = 16;
constexpr int MAX_KEYS = MAX_RCELLS * MAX_RCELLS;
// Groups of 8 pixels scored per sub-tile, at most: every level's area plus a
// 1-pixel ring, in whole groups (66 x 9 + 34 x 5 + 18 x 3 for three levels).
constexpr int MAX_GROUPS = 66 * 9 + 34 * 5 + 18 * 3;
constexpr uint16_t NO_ENTRY = 0xFFFF;

constexpr int OFF_M0 = TILE_BYTES;
// levels 1 and 2 share a band of M1_ROWS rows: level 1 in columns 0..35,
// level 2 in columns 40..59
constexpr int OFF_M1 = OFF_M0 + M0_ROWS * MP * 2;
constexpr int OFF_M2 = OFF_M1 + 40 * 2;
constexpr int OFF_KEYS = (OFF_M1 + M1_ROWS * MP * 2 + 15) & ~15;
static_assert(SUB / 2 + 4 <= 40 && 40 + SUB / 4 + 4 <= MP && M2_ROWS <= M1_ROWS, "level 1 and 2 maps share a band");
constexpr int OFF_KEYS2 = OFF_KEYS + MAX_KEYS * 4;   // second buffer for the pipelined kernel
constexpr int OFF_WAVES = OFF_KEYS2 + MAX_KEYS * 4;
static_assert(OFF_WAVES % 16 == 0, "aligned scratch");

// Per-wave scratch for V waves.  Compass rounds are dealt to the waves in
// turn, so a wave sees at most ceil(MAX_GROUPS / 64V) rounds of 64 groups:
// its group list holds that many words (64 per round) and its pixel list
// eight pixels per group plus one spare slot per lane.
__host__ __device__ constexpr int blist_cap(int waves) {
    return (MAX_GROUPS + 64 * waves - 1) / (64 * waves) * 64;
}
__host__ __device__ constexpr int list_cap(int waves) { return 8 * blist_cap(waves); }
__host__ __device__ constexpr int wave_bytes(int waves) {
    return (blist_cap(waves) * 4 + (list_cap(waves) + 64) * 2 + 15) & ~15;
}

}  // namespace

size_t fg_smem_bytes(int block) { return (size_t)OFF_WAVES + (size_t)(block / 64) * wave_bytes(block / 64); }

namespace {

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Image planes and outputs reach the kernels as generic pointers inside job
// structs.  Accessing them through global-address-space pointers makes the
// compiler emit global (not flat) loads and stores, which are counted by
// vmcnt only: outstanding HBM traffic then never holds up an LDS wait.
#define GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ T gload(const void *p) {
    return *(const GLOBAL T *)p;
}
template <class T>
__device__ __forceinline__ void gstore(void *p, T v) {
    *(GLOBAL T *)p = v;
}

__device__ __forceinline__ s16x2 as_s16x2(uint32_t v) { return __builtin_bit_cast(s16x2, v); }
__device__ __forceinline__ uint32_t as_u32(s16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ s16x2 vmax(s16x2 a, s16x2 b) { return __builtin_elementwise_max(a, b); }
__device__ __forceinline__ s16x2 vmin(s16x2 a, s16x2 b) { return __builtin_elementwise_min(a, b); }

// Two bytes of the 8-byte value {hi, lo} zero-extended into 16-bit lanes.
__device__ __forceinline__ s16x2 pair(uint32_t hi, uint32_t lo, uint32_t sel) {
    return as_s16x2(__builtin_amdgcn_perm(hi, lo, sel));
}

// floor(a / b) for 0 <= a < 2^21 and b >= 1 with the approximate reciprocal:
// (a + 0.5) / b lies at least 0.5 / b from an integer, and the relative error
// of rcp and of the product (< 2^-22) keeps the estimate closer than that.
__device__ __forceinline__ int div_small(int a, int b) {
    return (int)(((float)a + 0.5f) * __builtin_amdgcn_rcpf((float)b));
}

// An LDS pointer the compiler cannot see through.  Reads at constant
// non-negative offsets from it then share one address register and carry the
// offsets in the instructions' (unsigned) immediate fields, instead of the
// compiler folding the base into each address and adding negative offsets
// with separate instructions.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(3))) T *lds_base(const T *p) {
    const __attribute__((address_space(3))) T *q = (const __attribute__((address_space(3))) T *)p;
    asm("" : "+v"(q));
    return q;
}

__device__ __forceinline__ int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Orders this wave's LDS accesses across its lanes (LDS executes one wave's
// operations in order; this keeps the compiler from reordering them).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Inclusive prefix sum over the 64 lanes: shifts within rows of 16 lanes,
// then the row totals are broadcast into the following rows.
__device__ __forceinline__ int wave_scan(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return x;
}

// Bit i of the result is set iff bits i..i+n-1 of m are all set (1 <= n <=
// 16): runs of 2, 4, 8, 16 by doubling while they fit in n, then the
// remainder.  The shift amounts depend on n only (uniform, so they are scalar
// and hoisted out of the callers' loops); a step that does not apply shifts by
// 0, so the code has no branches.
__device__ __forceinline__ uint32_t runs(uint32_t m, int n) {
    const int s1 = n >= 2 ? 1 : 0, s2 = n >= 4 ? 2 : 0, s4 = n >= 8 ? 4 : 0, s8 = n >= 16 ? 8 : 0;
    m &= m >> s1;
    m &= m >> s2;
    m &= m >> s4;
    m &= m >> s8;
    return m & (m >> (n - 1 - s1 - s2 - s4 - s8));
}

// The same for n <= 8.
__device__ __forceinline__ uint32_t runs8(uint32_t m, int n) {
    const int s1 = n >= 2 ? 1 : 0, s2 = n >= 4 ? 2 : 0, s4 = n >= 8 ? 4 : 0;
    m &= m >> s1;
    m &= m >> s2;
    m &= m >> s4;
    return m & (m >> (n - 1 - s1 - s2 - s4));
}

// Compass test of two pixels in packed 16-bit lanes; per lane >= 0 iff the
// pixel may be a corner.  K = floor(N/4) consecutive points of (N, E, S, W)
// must all be brighter than c+t (darker than c-t); the weakest value over the
// best run is compared with the centre.
template <int K>
__device__ __forceinline__ s16x2 compass(s16x2 C, s16x2 N, s16x2 E, s16x2 S, s16x2 W, s16x2 T1) {
    s16x2 need_hi, need_lo;
    if constexpr (K == 1) {
        need_hi = vmax(vmax(N, S), vmax(E, W));
        need_lo = vmin(vmin(N, S), vmin(E, W));
    } else if constexpr (K == 2) {
        // adjacent pairs (N,E) (E,S) (S,W) (W,N): (N or S) and (E or W)
        need_hi = vmin(vmax(N, S), vmax(E, W));
        need_lo = vmax(vmin(N, S), vmin(E, W));
    } else if constexpr (K == 3) {
        // any 3 of the 4 are consecutive: second smallest / second largest
        const s16x2 lo1 = vmin(N, S), hi1 = vmax(N, S), lo2 = vmin(E, W), hi2 = vmax(E, W);
        need_hi = vmin(vmax(lo1, lo2), vmin(hi1, hi2));
        need_lo = vmax(vmin(hi1, hi2), vmax(lo1, lo2));
    } else {
        need_hi = vmin(vmin(N, S), vmin(E, W));
        need_lo = vmax(vmax(N, S), vmax(E, W));
    }
    return vmax(need_hi - C, C - need_lo) - T1;
}

// Circle of radius 3 (Section II-D) in cyclic order, as LDS byte offsets.
#define CIRC(j) (CDY[j] * LP + CDX[j])
// Offset of a pixel from the top-left corner of its circle's bounding box.
constexpr int CORNER = 3 * LP + 3;
constexpr int CDX[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
constexpr int CDY[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};

// Bits i .. i+n-1 (circularly, 0 <= i < 16) set for every bit i of `starts`
// (a 16-bit mask): the circle points covered by the arcs starting there.
__device__ __forceinline__ uint32_t arc_cover(uint32_t starts, int n) {
    uint32_t c = starts;
    int have = 1;
    while (have * 2 <= n) {
        c |= c << have;
        have *= 2;
    }
    if (have < n) c |= c << (n - have);
    return (c | (c >> 16)) & 0xFFFFu;
}

// w[i] <- min(w[i], w[(i + k) & 15]) for both 16-bit halves.
template <int K>
__device__ __forceinline__ void window_step(s16x2 (&w)[16]) {
    s16x2 u[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) u[i] = vmin(w[i], w[(i + K) & 15]);
#pragma unroll
    for (int i = 0; i < 16; ++i) w[i] = u[i];
}

template <int K>
__device__ __forceinline__ void rotate(s16x2 (&w)[16]) {
    s16x2 u[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) u[i] = w[(i + K) & 15];
#pragma unroll
    for (int i = 0; i < 16; ++i) w[i] = u[i];
}

// Maximum-threshold score from the 16 circle values: the largest d such that
// n consecutive points all exceed the centre by at least d (low half: v - c)
// or fall below it by at least d (high half: c - v).  Window minima by
// doubling (uniform steps), the remainder by a barrel rotation, so every
// register index is static.
__device__ __forceinline__ int max_threshold(const uint32_t (&v)[16], uint32_t cv, int n) {
    s16x2 w[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) w[i] = s16x2{(short)((int)v[i] - (int)cv), (short)((int)cv - (int)v[i])};
    int have = 1;
    if (n >= 2) { window_step<1>(w); have = 2; }
    if (n >= 4) { window_step<2>(w); have = 4; }
    if (n >= 8) { window_step<4>(w); have = 8; }
    if (n >= 16) { window_step<8>(w); have = 16; }
    const int r = n - have;   // 0 <= r < have
    if (r) {
        s16x2 u[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) u[i] = w[i];
        if (r & 1) rotate<1>(u);
        if (r & 2) rotate<2>(u);
        if (r & 4) rotate<4>(u);
#pragma unroll
        for (int i = 0; i < 16; ++i) w[i] = vmin(w[i], u[i]);
    }
    s16x2 m = w[0];
#pragma unroll
    for (int i = 1; i < 16; ++i) m = vmax(m, w[i]);
    return m.x > m.y ? m.x : m.y;
}

// Corner score kinds (Section II-D): FAST_SCORE_SADB sums over the whole
// circle, FAST_SCORE_SADA over the points on a qualifying arc, FAST_SCORE_MT
// is the maximum threshold at which the test still passes (plus one).
// Segment test and score of the pixel at p; 0 if the test fails.  The sums
// accumulate max(v - (c+t), 0) and max((c-t) - v, 0), each one saturating
// unsigned subtraction.
template <int KIND>
__device__ __forceinline__ uint32_t full_score(const uint8_t *p, int t, int n) {
    // every read is at a non-negative constant offset from the circle's
    // top-left corner, so all 17 share one address register
    const auto q = lds_base(p - CORNER);
    const uint32_t cv = q[CORNER];
    const uint32_t hi = cv + (uint32_t)t;
    const uint32_t lo = (int)cv - t > 0 ? cv - (uint32_t)t : 0u;   // darker needs v < c-t; none if c-t <= 0
    uint32_t v[16];
    uint32_t bm = 0, dm = 0, sb = 0, sd = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        v[j] = q[CORNER + CIRC(j)];
        bm = __builtin_amdgcn_alignbit(bm, hi - v[j], 31);   // sign: v > c+t; point j at bit 15-j
        dm = __builtin_amdgcn_alignbit(dm, v[j] - lo, 31);   // sign: v < c-t
    }
    if constexpr (KIND == FAST_SCORE_SADB) {
        // the sums in 16-bit lanes, points j and j+8 side by side: each lane
        // sums 8 terms of at most 255, so nothing saturates but the terms
        const u16x2 hi2 = {(unsigned short)hi, (unsigned short)hi}, lo2 = {(unsigned short)lo, (unsigned short)lo};
        u16x2 b2 = {0, 0}, d2 = {0, 0};
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const u16x2 p = __builtin_bit_cast(u16x2, v[j] | (v[j + 8] << 16));
            b2 += __builtin_elementwise_sub_sat(p, hi2);
            d2 += __builtin_elementwise_sub_sat(lo2, p);
        }
        sb = (uint32_t)b2.x + b2.y;
        sd = (uint32_t)d2.x + d2.y;
    }
    const uint32_t b2 = bm | (bm << 16), d2 = dm | (dm << 16);
    const uint32_t rb = runs(b2, n) & 0xFFFFu, rd = runs(d2, n) & 0xFFFFu;
    if ((rb | rd) == 0) return 0;
    if constexpr (KIND == FAST_SCORE_MT) return (uint32_t)max_threshold(v, cv, n);
    if constexpr (KIND == FAST_SCORE_SADA) {
        const uint32_t cb = arc_cover(rb, n), cd = arc_cover(rd, n);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            sb += __builtin_elementwise_sub_sat(v[j], hi) & (0u - ((cb >> (15 - j)) & 1u));
            sd += __builtin_elementwise_sub_sat(lo, v[j]) & (0u - ((cd >> (15 - j)) & 1u));
        }
    }
    return sb > sd ? sb : sd;
}

// One pyramid level of the current sub-tile as staged in LDS (uniform).
struct Geo {
    int tbase;           // LDS offset of tile (0,0)
    int tx, ty;          // level coordinates of tile (0,0)
    int W, H;            // level size
    int sx, sy, ex, ey;  // sub-tile area at this level (NMS targets), clipped
    int moff, mp;        // score map: LDS offset and pitch (u16) of [sx-1, ex+1) x [sy-1, ey+1)
    int gc0, ncolg;      // first group column (tile coords) and groups per row (even)
    int k;               // level index
};

struct Params {
    int t, n, kc, k8;    // threshold, arc length, floor(N/4), floor(N/2)
    int kind;            // corner score kind (FAST_SCORE_*)
    // score-map mode (smap[0] != null): the passes write each level's area
    // scores to smap[l] (pitch spitch[l] elements) instead of running NMS;
    // index l follows the levels handed to run_passes
    uint16_t *smap[3];
    int spitch[3];
    int cell;            // level-0 cell side
    int rx0, ry0;        // region origin in level-0 pixels
    int ncx;             // cells across the region
};

__device__ __forceinline__ void set_groups(Geo &g) {
    const int c_first = g.sx - 1 - g.tx;
    g.gc0 = c_first & ~3;
    g.ncolg = (g.ex + 1 - g.tx - g.gc0 + 3) >> 2;
    g.ncolg += g.ncolg & 1;   // whole pairs of groups
}

__device__ __forceinline__ bool has_area(const Geo &g) { return g.ex > g.sx && g.ey > g.sy; }

__device__ __forceinline__ int sel3(int l, int a, int b, int c) { return l == 0 ? a : (l == 1 ? b : c); }

// Scored area of one level in a sub-tile: rows [r0, r0 + nrows) of the tile
// band, groups of 8 pixels from column gc0, ppr groups per row; pixels
// outside [c_lo, c_hi] x [r_lo, r_hi] (tile coordinates) are not testable.
struct Seg {
    int tbase, r0, nrows, gc0, ppr, n;   // n = nrows * ppr groups
    int c_lo, c_hi, r_lo, r_hi;
};

__device__ __forceinline__ Seg make_seg(const Geo &g, bool on) {
    Seg q;
    q.tbase = g.tbase;
    q.r0 = g.sy - 1 - g.ty;
    q.nrows = on ? g.ey - g.sy + 2 : 0;
    q.gc0 = g.gc0;
    q.ppr = g.ncolg >> 1;
    q.n = q.nrows * q.ppr;
    q.c_lo = max(g.sx - 1, 3) - g.tx;
    q.c_hi = min(g.ex, g.W - 4) - g.tx;
    q.r_lo = max(q.r0, 3 - g.ty);
    q.r_hi = min(q.r0 + q.nrows - 1, g.H - 4 - g.ty);
    return q;
}

// The groups of all levels of a sub-tile form one sequence: level 0's rows
// first, then level 1's, then level 2's.  A group's entry is the LDS offset of
// its first pixel | level << 14, or NO_GROUP past the end.
constexpr uint32_t NO_GROUP = 0xFFFFu;
// Any offset whose 8 pixels and compass points lie inside the tile; a lane
// with no group reads there and discards the result.
constexpr uint32_t SAFE_OFF = T0 + 3 * LP + 4;
static_assert(SAFE_OFF % 8 == 4, "aligned compass row reads at SAFE_OFF");

struct GroupSeq {
    int b1, b2, total;   // first group of level 1, of level 2; group count
};

__device__ __forceinline__ GroupSeq group_seq(const Seg &s0, const Seg &s1, const Seg &s2) {
    GroupSeq q;
    q.b1 = s0.n;
    q.b2 = s0.n + s1.n;
    q.total = s0.n + s1.n + s2.n;
    return q;
}

__device__ __forceinline__ uint32_t group_entry(const Seg &s0, const Seg &s1, const Seg &s2,
                                                const GroupSeq &q, int i) {
    const uint32_t lvl = i < q.b1 ? 0u : (i < q.b2 ? 1u : 2u);
    const int local = i - (lvl == 0 ? 0 : (lvl == 1 ? q.b1 : q.b2));
    const int ppr = max(sel3(lvl, s0.ppr, s1.ppr, s2.ppr), 1);
    // row = floor((local + 0.5) / ppr), exact with the approximate reciprocal
    // since local < 1024 and ppr <= 9
    const int row = (int)(((float)local + 0.5f) * __builtin_amdgcn_rcpf((float)ppr)), pp = local - row * ppr;
    const uint32_t off = (uint32_t)(sel3(lvl, s0.tbase, s1.tbase, s2.tbase) +
                                    (sel3(lvl, s0.r0, s1.r0, s2.r0) + row) * LP +
                                    sel3(lvl, s0.gc0, s1.gc0, s2.gc0) + 8 * pp);
    return i < q.total ? off | (lvl << 14) : NO_GROUP;
}

// Group entries of one lane for the (at most four) compass rounds it takes
// when four or more waves share a sub-tile, two 16-bit entries per word.
// Regions with the same staged geometry have the same entries, so the
// pipelined kernel keeps them across regions; `key` names the geometry
// (-1: not reusable).
struct GroupCache {
    uint32_t e01, e23;
    int key;
};

// The words a compass test of 8 pixels reads: the 16 bytes around the group
// on its own row (4 before, 4 after) and 8 bytes three rows above and below.
// With A8 every group starts 4 bytes past a multiple of 8 (see the tile
// layout), and the row is read as two aligned 8-byte words.
struct Px8 {
    uint32_t D0, D1, D2, D3, N0, N1, S0, S1;
};

template <bool A8>
__device__ __forceinline__ Px8 load8(const uint8_t *smem, uint32_t off) {
    // every read at a non-negative offset from the word 4 bytes before the
    // group's pixel three rows up
    const auto b = lds_base((const uint32_t *)(smem + off - 3 * LP - 4));
    constexpr int R3 = 3 * LP / 4;   // three rows, in words
    Px8 x;
    if constexpr (A8) {
        // b is 8-aligned here (LP and the group's offset - 4 are)
        const auto b2 = (const __attribute__((address_space(3))) u32x2 *)b;
        const u32x2 lo = b2[R3 / 2], hi = b2[R3 / 2 + 1];
        x.D0 = lo.x;
        x.D1 = lo.y;
        x.D2 = hi.x;
        x.D3 = hi.y;
    } else {
        x.D0 = b[R3];
        x.D1 = b[R3 + 1];
        x.D2 = b[R3 + 2];
        x.D3 = b[R3 + 3];
    }
    x.N0 = b[1];
    x.N1 = b[2];
    x.S0 = b[2 * R3 + 1];
    x.S1 = b[2 * R3 + 2];
    return x;
}

// Compass test of the 8 pixels of x: bit j <- pixel 2j, bit 4+j <- pixel
// 2j+1 (set = may be a corner).
template <int K>
__device__ __forceinline__ uint32_t compass8(const Px8 &x, s16x2 T1) {
    if constexpr (K > 0) {
        const uint32_t r01 = as_u32(compass<K>(
            pair(x.D1, x.D1, 0x0c010c00u), pair(x.N0, x.N0, 0x0c010c00u), pair(x.D2, x.D1, 0x0c040c03u),
            pair(x.S0, x.S0, 0x0c010c00u), pair(x.D1, x.D0, 0x0c020c01u), T1));
        const uint32_t r23 = as_u32(compass<K>(
            pair(x.D1, x.D1, 0x0c030c02u), pair(x.N0, x.N0, 0x0c030c02u), pair(x.D2, x.D1, 0x0c060c05u),
            pair(x.S0, x.S0, 0x0c030c02u), pair(x.D1, x.D0, 0x0c040c03u), T1));
        const uint32_t r45 = as_u32(compass<K>(
            pair(x.D2, x.D2, 0x0c010c00u), pair(x.N1, x.N1, 0x0c010c00u), pair(x.D3, x.D2, 0x0c040c03u),
            pair(x.S1, x.S1, 0x0c010c00u), pair(x.D2, x.D1, 0x0c020c01u), T1));
        const uint32_t r67 = as_u32(compass<K>(
            pair(x.D2, x.D2, 0x0c030c02u), pair(x.N1, x.N1, 0x0c030c02u), pair(x.D3, x.D2, 0x0c060c05u),
            pair(x.S1, x.S1, 0x0c030c02u), pair(x.D2, x.D1, 0x0c040c03u), T1));
        // sign bit of each 16-bit lane = rejected; bit j <- pixel 2j,
        // bit 4+j <- pixel 2j+1
        const uint32_t sg = ((r01 >> 15) & 0x10001u) | ((r23 >> 14) & 0x20002u) |
                            ((r45 >> 13) & 0x40004u) | ((r67 >> 12) & 0x80008u);
        return ~(sg | (sg >> 12)) & 0xFFu;
    } else {
        return 0xFFu;
    }
}

// LDS offset a lane with entry e reads (a safe one for NO_GROUP).
__device__ __forceinline__ uint32_t entry_off(uint32_t e) { return e != NO_GROUP ? (e & 0x3FFFu) : SAFE_OFF; }

// Bits b with lo <= b < hi (0 <= lo <= hi <= 4).
__device__ __forceinline__ uint32_t bit_range(int lo, int hi) { return (1u << hi) - (1u << lo); }

// P1+P2: compass test of every scored pixel of every level, 8 pixels per
// lane in packed 16-bit lanes.  The groups of all levels form one sequence
// dealt to the waves round-robin in rounds of 64, so every wave does the
// same share whatever the level sizes; a wave tests two rounds at a time so
// that the LDS reads of one overlap the arithmetic of the other.  Groups with
// a survivor are compacted into the wave's group list (ballot + mbcnt; word =
// level << 22 | LDS offset of the group << 8 | survivor mask), which is then
// expanded into the wave's pixel list, keeping testable pixels only; an entry
// is (level << 14) | LDS offset of the pixel.  Returns the wave's pixel count.
// With `cached` (four or more waves), the group entries are e01 and e23
// (GroupCache).
template <int K, bool A8>
__device__ int collect(const uint8_t *smem, const Seg &s0, const Seg &s1, const Seg &s2, int t,
                       bool cached, uint32_t e01, uint32_t e23, uint32_t *blist, uint16_t *list) {
    const int lane = lane_id(), wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), nwaves = blockDim.x >> 6;
    const GroupSeq q = group_seq(s0, s1, s2);
    const s16x2 T1 = {(short)(t + 1), (short)(t + 1)};
    const int stride = nwaves * 64;
    int nb = 0;
    // survivors go to nb + (survivors below the lane); the other lanes write
    // past them, inside the round's own 64 words, where a later round
    // overwrites them, so the stores need no branch
    auto push = [&](uint32_t e, uint32_t sv) {
        const uint64_t bal = __ballot(sv != 0);
        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        const int cnt = __popcll(bal);
        blist[sv ? nb + rank : nb + cnt + lane - rank] = (e << 8) | sv;
        nb += cnt;
    };
    for (int r = 0;; r += 2) {
        const int i0 = wave * 64 + r * stride;
        if (i0 >= q.total) break;
        uint32_t ea, eb;
        if (cached) {
            const uint32_t w = r == 0 ? e01 : e23;
            ea = w & 0xFFFFu;
            eb = w >> 16;
        } else {
            ea = group_entry(s0, s1, s2, q, i0 + lane);
            eb = group_entry(s0, s1, s2, q, i0 + stride + lane);
        }
        const Px8 xa = load8<A8>(smem, entry_off(ea));
        if (i0 + stride < q.total) {
            // two rounds: both rounds' LDS reads are issued before either is
            // evaluated
            const Px8 xb = load8<A8>(smem, entry_off(eb));
            const uint32_t sva = compass8<K>(xa, T1) & (0u - (uint32_t)(ea != NO_GROUP));
            const uint32_t svb = compass8<K>(xb, T1) & (0u - (uint32_t)(eb != NO_GROUP));
            push(ea, sva);
            push(eb, svb);
        } else {
            push(ea, compass8<K>(xa, T1) & (0u - (uint32_t)(ea != NO_GROUP)));
        }
    }
    wave_sync();
    int count = 0;
    const int spare = list_cap(nwaves) + lane;
    for (int j0 = 0; j0 < nb; j0 += 64) {
        const int j = j0 + lane;
        const uint32_t w = j < nb ? blist[j] : 0u;
        const uint32_t l = w >> 22;
        const int off0 = (int)((w >> 8) & 0x3FFFu);
        const int rel = off0 - sel3(l, s0.tbase, s1.tbase, s2.tbase);
        const int r = (int)(((uint32_t)rel * 18725u) >> 21);   // rel / LP
        const int c0 = rel - r * LP;
        const bool row_ok = r >= sel3(l, s0.r_lo, s1.r_lo, s2.r_lo) && r <= sel3(l, s0.r_hi, s1.r_hi, s2.r_hi);
        // pixel p of the group (column c0 + p) is testable iff lo <= p < hi;
        // bit b of the mask is pixel 2b (b < 4) or 2(b-4)+1
        const int lo = min(max(sel3(l, s0.c_lo, s1.c_lo, s2.c_lo) - c0, 0), 8);
        const int hi = max(min(max(sel3(l, s0.c_hi, s1.c_hi, s2.c_hi) - c0 + 1, 0), 8), lo);
        const uint32_t valid = bit_range((lo + 1) >> 1, (hi + 1) >> 1) | (bit_range(lo >> 1, hi >> 1) << 4);
        const uint32_t m = row_ok ? (w & valid) : 0u;
        const int cnt = __builtin_popcount(m);
        const int incl = wave_scan(cnt);
        const int pos = count + incl - cnt;
        count += __builtin_amdgcn_readlane(incl, 63);
        const uint32_t base = (l << 14) | (uint32_t)off0;
        // a kept pixel goes to pos + (kept pixels before it); the others write
        // to the lane's spare slot, so the loop has no branches
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int at = (m >> b) & 1u ? pos + __builtin_popcount(m & ((1u << b) - 1u)) : spare;
            list[at] = (uint16_t)(base + (uint32_t)(((b & 3) << 1) | (b >> 2)));
        }
    }
    return count;
}

// Entries of this lane's compass rounds when at least four waves share the
// sub-tile (at most four rounds: MAX_GROUPS <= 4 * 256).
__device__ __forceinline__ void group_cache_fill(GroupCache &c, const Seg &s0, const Seg &s1, const Seg &s2) {
    const int lane = lane_id(), wave = threadIdx.x >> 6, stride = (blockDim.x >> 6) * 64;
    const GroupSeq q = group_seq(s0, s1, s2);
    const int i = wave * 64 + lane;
    c.e01 = group_entry(s0, s1, s2, q, i) | (group_entry(s0, s1, s2, q, i + stride) << 16);
    c.e23 = group_entry(s0, s1, s2, q, i + 2 * stride) | (group_entry(s0, s1, s2, q, i + 3 * stride) << 16);
}
static_assert(MAX_GROUPS <= 4 * 256, "four compass rounds per wave with four or more waves");

// P3: keep entries that pass the 8-point test, compacted in place.  A lane
// past the end reads a stale slot (the list has a spare slot per lane beyond
// its capacity, and n1 <= capacity), tests the pixel at SAFE_OFF instead and
// is masked off; entries that fail go to the lane's spare slot.  The pass
// therefore has no branches.
__device__ int pass_even8(const uint8_t *smem, int t, int k8, uint16_t *list, int n1) {
    const int lane = lane_id();
    const int spare = list_cap(blockDim.x >> 6) + lane;
    int n2 = 0;
    for (int i0 = 0; i0 < n1; i0 += 64) {
        const int i = i0 + lane;
        const uint16_t e = list[i];
        const bool valid = i < n1 && e != NO_ENTRY;
        const auto q = lds_base(smem + (valid ? (e & 0x3FFFu) : SAFE_OFF) - CORNER);
        const int cv = q[CORNER];
        const int hi = cv + t, lo = cv - t;
        uint32_t bm = 0, dm = 0;
#pragma unroll
        for (int j = 0; j < 16; j += 2) {
            const int v = q[CORNER + CIRC(j)];
            bm = __builtin_amdgcn_alignbit(bm, (uint32_t)(hi - v), 31);
            dm = __builtin_amdgcn_alignbit(dm, (uint32_t)(v - lo), 31);
        }
        // bright arcs in bits 0-15, dark arcs in bits 16-31, each 8-point
        // mask doubled for the circular wrap: a run of k8 <= 8 starting at
        // bit 0-7 (16-23) stays below bit 15 (31)
        const uint32_t w = (bm | (dm << 16)) * 0x101u;
        const bool pass = valid && (k8 == 0 || (runs8(w, k8) & 0x00FF00FFu) != 0);
        const uint64_t bal = __ballot(pass);
        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        list[pass ? n2 + rank : spare] = e;
        n2 += __popcll(bal);
        wave_sync();
    }
    return n2;
}


// Row and column inside the LDS tile band of an entry's offset.
__device__ __forceinline__ void tile_rc(uint32_t off, int &row, int &col) {
    row = (int)((off * 18725u) >> 21);   // off / LP, exact for off < 16384
    col = (int)off - row * LP;
}

// Per-level constants for mapping an entry to its score map and cell.
struct LevelMap {
    int mp, mbias;       // map index = row * mp + col + mbias (row, col in the tile band)
    int rlo, rhi;        // band rows of the sub-tile area: [rlo, rhi)
    int clo, chi;        // band columns of the sub-tile area: [clo, chi)
    int xo, yo;          // cell-relative position = (col + xo, row + yo)
    int cw;              // cell side at this level
    float inv_cw;        // ~1/cw: floor((v + 0.5) * inv_cw) = v / cw for 0 <= v < 2^12
};

__device__ __forceinline__ LevelMap level_map(const Geo &g, int band_row, int band_col, int ra,
                                             int rb, const Params &P) {
    LevelMap m;
    const int ybias = g.ty - band_row, xbias = g.tx - band_col;   // level y = row + ybias
    m.mp = g.mp;
    m.mbias = (g.moff >> 1) + (ybias - (g.sy - 1)) * g.mp + (xbias - (g.sx - 1));
    m.rlo = ra - ybias;
    m.rhi = rb - ybias;
    m.clo = g.sx - xbias;
    m.chi = g.ex - xbias;
    m.xo = xbias - (P.rx0 >> g.k);
    m.yo = ybias - (P.ry0 >> g.k);
    m.cw = P.cell >> g.k;
    m.inv_cw = __builtin_amdgcn_rcpf((float)max(m.cw, 1));
    return m;
}

// Write the scores of level g's sub-tile area from its LDS score map to a
// global map (row y at dst + y * pitch elements).
__device__ void store_scores(const uint8_t *smem, const Geo &g, uint16_t *dst, int pitch) {
    const int w = g.ex - g.sx, h = g.ey - g.sy;
    if (w <= 0 || h <= 0) return;
    const uint16_t *m = (const uint16_t *)smem + (g.moff >> 1);
    for (int i = threadIdx.x; i < w * h; i += blockDim.x) {
        const int yy = div_small(i, w), xx = i - yy * w;
        gstore<uint16_t>(dst + (ptrdiff_t)(g.sy + yy) * pitch + (g.sx + xx), m[(yy + 1) * g.mp + xx + 1]);
    }
}

// Detect levels g0..g(nl-1) of the staged sub-tile (score maps zeroed) and
// fold the survivors into the region's cell keys.  P1-P4 run on every wave
// without workgroup barriers; one barrier makes all scores visible before
// NMS.
struct NoHook {
    __device__ void operator()() const {}
};

// `before` runs on every thread just before the barrier that separates
// scoring from NMS, `after` just after it (the pipelined kernel uses them to
// publish its next work item and to reuse the level-0 tile, which NMS no
// longer reads).
//
// `cache` (workgroups of four or more waves only) keeps the compass group
// entries across calls whose staged geometry has the same `cache_key`
// (-1: recompute).
template <class Before = NoHook, class After = NoHook>
__device__ void run_passes(uint8_t *smem, const Geo &g0, const Geo &g1, const Geo &g2, int nl,
                           const Params &P, uint32_t *keys, GroupCache *cache = nullptr, int cache_key = -1,
                           Before before = Before(), After after = After()) {
    const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    uint8_t *scratch = smem + OFF_WAVES + wave * wave_bytes(nwaves);
    uint32_t *blist = (uint32_t *)scratch;
    uint16_t *list = (uint16_t *)(scratch + blist_cap(nwaves) * 4);
    const Seg s0 = make_seg(g0, has_area(g0));
    const Seg s1 = make_seg(g1, nl > 1 && has_area(g1));
    const Seg s2 = make_seg(g2, nl > 2 && has_area(g2));
    if (cache && (cache_key < 0 || __builtin_amdgcn_readfirstlane(cache->key) != cache_key)) {
        group_cache_fill(*cache, s0, s1, s2);
        cache->key = cache_key;
    }
    const uint32_t ce01 = cache ? cache->e01 : 0u, ce23 = cache ? cache->e23 : 0u;
    // every level's groups start 4 bytes past a multiple of 8 (uniform): true
    // for fused sub-tiles, whose origins are on the 16-pixel grid; the single
    // deeper levels of process_subtile_upper may start elsewhere
    const bool a8 = ((s0.tbase + s0.gc0) & 7) == 4 && (!s1.n || ((s1.tbase + s1.gc0) & 7) == 4) &&
                    (!s2.n || ((s2.tbase + s2.gc0) & 7) == 4);
    int n1 = 0;
    auto run_collect = [&](auto aligned) {
        constexpr bool A = decltype(aligned)::value;
        switch (P.kc) {
            case 0: n1 = collect<0, A>(smem, s0, s1, s2, P.t, cache != nullptr, ce01, ce23, blist, list); break;
            case 1: n1 = collect<1, A>(smem, s0, s1, s2, P.t, cache != nullptr, ce01, ce23, blist, list); break;
            case 2: n1 = collect<2, A>(smem, s0, s1, s2, P.t, cache != nullptr, ce01, ce23, blist, list); break;
            case 3: n1 = collect<3, A>(smem, s0, s1, s2, P.t, cache != nullptr, ce01, ce23, blist, list); break;
            default: n1 = collect<4, A>(smem, s0, s1, s2, P.t, cache != nullptr, ce01, ce23, blist, list); break;
        }
    };
    if (a8)
        run_collect(std::true_type());
    else
        run_collect(std::false_type());
    wave_sync();
    // the later passes run at a raised wave priority: a wave that is further
    // through its sub-tile issues first, so workgroups reach their barriers
    // sooner (the waves sharing a SIMD belong to different workgroups)
    __builtin_amdgcn_s_setprio(1);
    const int n2 = pass_even8(smem, P.t, P.k8, list, n1);
    const LevelMap m0 = level_map(g0, 0, T0, g0.sy, g0.ey, P);
    const LevelMap m1 = level_map(g1, 96, T1 - 96 * LP, g1.sy, g1.ey, P);
    const LevelMap m2 = level_map(g2, 96, T2 - 96 * LP, g2.sy, g2.ey, P);
    uint16_t *maps = (uint16_t *)smem;
    const int lane = lane_id();
    // P4: full segment test and score into the level's score map (one loop
    // per score kind, so each compiles to straight-line code)
    auto score_pass = [&](auto kind) {
        for (int i = lane; i < n2; i += 64) {
            const uint16_t e = list[i];
            const uint32_t s = full_score<decltype(kind)::value>(smem + (e & 0x3FFF), P.t, P.n);
            if (s) {
                const int l = e >> 14;
                int row, col;
                tile_rc(e & 0x3FFF, row, col);
                maps[row * MP + col + sel3(l, m0.mbias, m1.mbias, m2.mbias)] =
                    (uint16_t)s;
            }
        }
    };
    switch (P.kind) {
        case FAST_SCORE_SADA: score_pass(std::integral_constant<int, FAST_SCORE_SADA>()); break;
        case FAST_SCORE_MT: score_pass(std::integral_constant<int, FAST_SCORE_MT>()); break;
        default: score_pass(std::integral_constant<int, FAST_SCORE_SADB>()); break;
    }
    before();
    __syncthreads();   // every level's scores, ring included, are in the maps
    after();
    if (P.smap[0]) {   // score-map mode: the sub-tile's own scores, no NMS
        store_scores(smem, g0, P.smap[0], P.spitch[0]);
        if (nl > 1) store_scores(smem, g1, P.smap[1], P.spitch[1]);
        if (nl > 2) store_scores(smem, g2, P.smap[2], P.spitch[2]);
        __builtin_amdgcn_s_setprio(0);
        return;
    }
    // P5: 3x3 NMS of the sub-tile's own pixels, then the cell keys.  A lane
    // issues its nine score reads together, so the test costs one LDS round
    // trip; a ring pixel (its own sub-tile suppresses it) reads around a
    // fixed entry of the level-0 map instead and is masked off.
    for (int i = lane; i < n2; i += 64) {
        const uint16_t e = list[i];
        const int l = e >> 14;
        int row, col;
        tile_rc(e & 0x3FFF, row, col);
        const bool own = (row >= sel3(l, m0.rlo, m1.rlo, m2.rlo)) & (row < sel3(l, m0.rhi, m1.rhi, m2.rhi)) &
                         (col >= sel3(l, m0.clo, m1.clo, m2.clo)) & (col < sel3(l, m0.chi, m1.chi, m2.chi));
        constexpr int mp = MP;
        // q: the upper-left neighbour
        const auto q = lds_base(maps + (own ? row * mp + col + sel3(l, m0.mbias, m1.mbias, m2.mbias) : OFF_M0 / 2 + mp + 1) -
                                mp - 1);
        const uint32_t s = q[mp + 1];
        // earlier neighbours in row-major order must be strictly lower,
        // later ones lower or equal
        const uint32_t earlier = max(max((uint32_t)q[0], (uint32_t)q[1]), max((uint32_t)q[2], (uint32_t)q[mp]));
        const uint32_t later =
            max(max((uint32_t)q[mp + 2], (uint32_t)q[2 * mp]), max((uint32_t)q[2 * mp + 1], (uint32_t)q[2 * mp + 2]));
        if (!(own & (s != 0) & (s > earlier) & (s >= later))) continue;
        const int cw = sel3(l, m0.cw, m1.cw, m2.cw);
        const int ox = col + sel3(l, m0.xo, m1.xo, m2.xo);
        const int oy = row + sel3(l, m0.yo, m1.yo, m2.yo);
        // exact: v + 0.5 is at least 0.5 / cw from a multiple of cw, far above
        // the error of the approximate reciprocal for v < 2^12
        const float inv = l == 0 ? m0.inv_cw : (l == 1 ? m1.inv_cw : m2.inv_cw);
        const int cy = (int)(((float)oy + 0.5f) * inv), cx = (int)(((float)ox + 0.5f) * inv);
        const uint32_t local = (uint32_t)((oy - cy * cw) * cw + (ox - cx * cw));
        const uint32_t key = (s << 19) | ((uint32_t)(7 - (g0.k + l)) << 16) | (0xFFFFu - local);
        atomicMax(&keys[cy * P.ncx + cx], key);
    }
    __builtin_amdgcn_s_setprio(0);
}

// Stage level pixels [tx, tx+tw) x [ty, ty+th) into an LDS tile with 16-byte
// loads (tx % 16 == 0, so no chunk straddles the pitch; tw <= 128).  Chunks
// outside the plane are zero and never used as pixel values.  Thread i owns
// chunk column i % 8 of rows i/8 + j * (block/8); the first four of its rows
// are loaded into registers (TileRegs) before any store.
struct TileRegs {
    u32x4 v[4];
};

__device__ __forceinline__ void tile_issue(TileRegs &R, const uint8_t *img, int H, int P, int tx, int ty,
                                           int tw, int th) {
    const int ch = threadIdx.x & 7;
    const int gx = tx + 16 * ch;
    const bool col_ok = ch < (tw >> 4) && gx >= 0 && gx < P;
    const int r0 = threadIdx.x >> 3, dr = blockDim.x >> 3;
    // row pointers advance by a uniform stride: one 64-bit multiply per thread
    const uint8_t *row = img + (ptrdiff_t)(ty + r0) * P + gx;
    const ptrdiff_t step = (ptrdiff_t)dr * P;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int r = r0 + j * dr, gy = ty + r;
        R.v[j] = u32x4{0u, 0u, 0u, 0u};
        if (r < th && col_ok && gy >= 0 && gy < H) R.v[j] = gload<u32x4>(row);
        row += step;
    }
}

__device__ __forceinline__ void tile_commit(uint8_t *tile, const TileRegs &R, int tw, int th) {
    const int ch = threadIdx.x & 7;
    if (ch >= (tw >> 4)) return;
    const int r0 = threadIdx.x >> 3, dr = blockDim.x >> 3;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int r = r0 + j * dr;
        if (r < th) *(u32x4 *)(tile + r * LP + 16 * ch) = R.v[j];
    }
}

__device__ void load_tile(uint8_t *tile, const uint8_t *img, int H, int P, int tx, int ty, int tw,
                          int th) {
    TileRegs R;
    tile_issue(R, img, H, P, tx, ty, tw, th);
    tile_commit(tile, R, tw, th);
    const int ch = threadIdx.x & 7;
    if (ch >= (tw >> 4)) return;
    const int gx = tx + 16 * ch;
    const bool col_ok = gx >= 0 && gx < P;
    const int dr = blockDim.x >> 3;
    for (int r = (threadIdx.x >> 3) + 4 * dr; r < th; r += dr) {   // small workgroups only
        const int gy = ty + r;
        u32x4 w = u32x4{0u, 0u, 0u, 0u};
        if (col_ok && gy >= 0 && gy < H) w = gload<u32x4>(img + (size_t)gy * P + gx);
        *(u32x4 *)(tile + r * LP + 16 * ch) = w;
    }
}

// Four pyramid pixels from two rows of eight: (a+b+c+d+2)>>2 per 2x2 block.
// Bytes 0, 2 and bytes 1, 3 of each word go to 16-bit lanes with one v_perm
// each; a block's sum is at most 4 * 255 + 2, so no lane carries into the
// next.  After the shift by 2 each lane's result is its low byte (the bits
// shifted in from the lane above land in the byte the final v_perm skips).
__device__ __forceinline__ uint32_t halve4(uint2 a, uint2 b) {
    auto even = [](uint32_t x) { return __builtin_amdgcn_perm(0u, x, 0x0c020c00u); };
    auto odd = [](uint32_t x) { return __builtin_amdgcn_perm(0u, x, 0x0c030c01u); };
    const uint32_t s0 = even(a.x) + odd(a.x) + even(b.x) + odd(b.x) + 0x00020002u;
    const uint32_t s1 = even(a.y) + odd(a.y) + even(b.y) + odd(b.y) + 0x00020002u;
    return __builtin_amdgcn_perm(s1 >> 2, s0 >> 2, 0x06040200u);
}

// Levels 1 and 2 of a fused tile in one pass (tw a multiple of 16): a task
// reads a 16 x 4 block of level 0 and writes the 8 x 2 level-1 block and the
// 4 x 1 level-2 block it covers, each by successive (a+b+c+d+2)>>2 rounding.
// With an odd number of level-1 rows the last one has tasks of its own.
__device__ void halve_two(const uint8_t *l0, uint8_t *l1, uint8_t *l2, int tw, int th, bool need_l2) {
    const int wpr = tw >> 4, rows2 = th >> 2;
    const int tasks = wpr * rows2 + (((th >> 1) & 1) ? wpr : 0);
    for (int i = threadIdx.x; i < tasks; i += blockDim.x) {
        const int y2 = div_small(i, wpr), x4 = i - y2 * wpr;
        const uint8_t *s = l0 + (4 * y2) * LP + 16 * x4;
        if (y2 < rows2) {
            const u32x4 a = *(const u32x4 *)s, b = *(const u32x4 *)(s + LP);
            const u32x4 c = *(const u32x4 *)(s + 2 * LP), d = *(const u32x4 *)(s + 3 * LP);
            const uint32_t r0a = halve4(make_uint2(a.x, a.y), make_uint2(b.x, b.y));
            const uint32_t r0b = halve4(make_uint2(a.z, a.w), make_uint2(b.z, b.w));
            const uint32_t r1a = halve4(make_uint2(c.x, c.y), make_uint2(d.x, d.y));
            const uint32_t r1b = halve4(make_uint2(c.z, c.w), make_uint2(d.z, d.w));
            *(uint2 *)(l1 + (2 * y2) * LP + 8 * x4) = make_uint2(r0a, r0b);
            *(uint2 *)(l1 + (2 * y2 + 1) * LP + 8 * x4) = make_uint2(r1a, r1b);
            if (need_l2) *(uint32_t *)(l2 + y2 * LP + 4 * x4) = halve4(make_uint2(r0a, r0b), make_uint2(r1a, r1b));
        } else {
            // last level-1 row, 2 * rows2, from level-0 rows 4 * rows2 and 4 * rows2 + 1
            const u32x4 a = *(const u32x4 *)s, b = *(const u32x4 *)(s + LP);
            *(uint2 *)(l1 + (2 * y2) * LP + 8 * x4) =
                make_uint2(halve4(make_uint2(a.x, a.y), make_uint2(b.x, b.y)),
                           halve4(make_uint2(a.z, a.w), make_uint2(b.z, b.w)));
        }
    }
}

// Copy the sub-tile's own pixels of an LDS level to the pyramid plane
// (sx % 4 == 0, ex - sx <= 32).  The last word of a row is written byte by
// byte when it would cross the level width.
__device__ void store_level(const uint8_t *tile, int tx, int ty, uint8_t *img, int P, int sx, int sy,
                            int ex, int ey) {
    const int w = threadIdx.x & 7;               // 8 word slots per row
    const int x = sx + 4 * w;
    if (x >= ex) return;
    for (int y = sy + (threadIdx.x >> 3); y < ey; y += blockDim.x >> 3) {
        const uint8_t *s = tile + (y - ty) * LP + (x - tx);
        uint8_t *d = img + (size_t)y * P + x;
        if (x + 4 <= ex) {
            gstore<uint32_t>(d, *(const uint32_t *)s);
        } else {
            for (int q = 0; q < ex - x; ++q) gstore<uint8_t>(d + q, s[q]);
        }
    }
}

// Zero [p, p+bytes) with 16-byte stores (p and bytes multiples of 16).
__device__ void zero_lds(uint8_t *p, int bytes) {
    for (int i = threadIdx.x; i < (bytes >> 4); i += blockDim.x) ((uint4 *)p)[i] = make_uint4(0, 0, 0, 0);
}

// Level-k area of the level-0 sub-tile at (sx0, sy0), clipped to the region
// end (xr1, yr1 at level 0) and the level size.
__device__ __forceinline__ void level_area(const fg_job &J, int k, int sx0, int sy0, int xr1,
                                           int yr1, Geo &g) {
    g.k = k;
    g.W = J.w[k];
    g.H = J.h[k];
    g.sx = sx0 >> k;
    g.sy = sy0 >> k;
    g.ex = min(min((sx0 + SUB) >> k, xr1 >> k), g.W);
    g.ey = min(min((sy0 + SUB) >> k, yr1 >> k), g.H);
}

// Levels 0 .. fused_levels(J)-1 are detected from one level-0 load; levels
// beyond (jobs with more than MAX_FUSED levels) are detected afterwards by
// the upper-level pass.
__device__ __forceinline__ int fused_levels(const fg_job &J) { return min(J.levels, MAX_FUSED); }

// Level-0 tile of a fused sub-tile: the sub-tile plus a 4*2^(F-1) halo (F
// fused levels), with the left edge rounded down to 16 pixels.
struct Stage {
    int tx, ty, tw, th;
};

__device__ __forceinline__ Stage fused_stage(const fg_job &J, int sx0, int sy0, int xr1, int yr1) {
    const int H0 = 4 << (fused_levels(J) - 1);
    Stage st;
    st.tx = (sx0 - H0) & ~15;
    st.ty = sy0 - H0;
    st.tw = ((min(sx0 + SUB, xr1) + H0 + 15) & ~15) - st.tx;
    st.th = min(sy0 + SUB, yr1) + H0 - st.ty;
    return st;
}

// Describe levels 0 .. F-1 of a fused sub-tile staged as `st`.
__device__ void describe_fused(const fg_job &J, int sx0, int sy0, int xr1, int yr1, const Stage &st, Geo &g0,
                               Geo &g1, Geo &g2) {
    level_area(J, 0, sx0, sy0, xr1, yr1, g0);
    g0.tbase = T0;
    g0.tx = st.tx;
    g0.ty = st.ty;
    g0.moff = OFF_M0;
    g0.mp = M0_P;
    set_groups(g0);
    g1 = g0;
    g2 = g0;
    const int nl = fused_levels(J);
    if (nl > 1) {
        level_area(J, 1, sx0, sy0, xr1, yr1, g1);
        g1.tbase = T1;
        g1.tx = st.tx >> 1;
        g1.ty = st.ty >> 1;
        g1.moff = OFF_M1;
        g1.mp = M1_P;
        set_groups(g1);
    }
    if (nl > 2) {
        level_area(J, 2, sx0, sy0, xr1, yr1, g2);
        g2.tbase = T2;
        g2.tx = st.tx >> 2;
        g2.ty = st.ty >> 2;
        g2.moff = OFF_M2;
        g2.mp = M2_P;
        set_groups(g2);
    }
}

// With level 0 of a fused sub-tile in LDS: build levels 1.. in LDS, describe
// every level, and write levels 1.. of the sub-tile to their planes.
__device__ void build_fused(const fg_job &J, int sx0, int sy0, int xr1, int yr1, const Stage &st,
                            uint8_t *smem, Geo &g0, Geo &g1, Geo &g2) {
    describe_fused(J, sx0, sy0, xr1, yr1, st, g0, g1, g2);
    const int nl = fused_levels(J);
    if (nl > 1) {
        __syncthreads();
        halve_two(smem + T0, smem + T1, smem + T2, st.tw, st.th, nl > 2);
    }
    __syncthreads();
    if (nl > 1 && has_area(g1))
        store_level(smem + T1, g1.tx, g1.ty, J.lvl[1], J.pitch[1], g1.sx, g1.sy, g1.ex, g1.ey);
    if (nl > 2 && has_area(g2))
        store_level(smem + T2, g2.tx, g2.ty, J.lvl[2], J.pitch[2], g2.sx, g2.sy, g2.ex, g2.ey);
}

// One level-0 sub-tile of a region: stage levels 0 .. F-1, detect, fold into
// keys.
__device__ void process_subtile(const fg_job &J, int sx0, int sy0, int xr1, int yr1,
                                const Params &P, uint8_t *smem) {
    // one load with a 4*2^(F-1) halo; levels 1 .. F-1 built in LDS
    const Stage st = fused_stage(J, sx0, sy0, xr1, yr1);
    __syncthreads();
    load_tile(smem + T0, J.lvl[0], J.h[0], J.pitch[0], st.tx, st.ty, st.tw, st.th);
    zero_lds(smem + OFF_M0, OFF_KEYS - OFF_M0);
    Geo g0, g1, g2;
    build_fused(J, sx0, sy0, xr1, yr1, st, smem, g0, g1, g2);
    run_passes(smem, g0, g1, g2, fused_levels(J), P, (uint32_t *)(smem + OFF_KEYS));
}

// Levels MAX_FUSED .. L-1 of one level-0 sub-tile (already built in their
// planes): one level at a time, loaded with a 4-pixel halo.
__device__ void process_subtile_upper(const fg_job &J, int sx0, int sy0, int xr1, int yr1,
                                      const Params &P, uint8_t *smem) {
    for (int k = MAX_FUSED; k < J.levels; ++k) {
        Geo g;
        level_area(J, k, sx0, sy0, xr1, yr1, g);
        if (!has_area(g)) continue;
        const int tx = (g.sx - 4) & ~15, ty = g.sy - 4;
        const int tw = ((g.ex + 4 + 15) & ~15) - tx, th = g.ey + 4 - ty;
        __syncthreads();
        load_tile(smem + T0, J.lvl[k], g.H, J.pitch[k], tx, ty, tw, th);
        zero_lds(smem + OFF_M0, (M0_ROWS * M0_P * 2 + 15) & ~15);
        __syncthreads();
        g.tbase = T0;
        g.tx = tx;
        g.ty = ty;
        g.moff = OFF_M0;
        g.mp = M0_P;
        set_groups(g);
        Params Pk = P;
        if (P.smap[0]) {
            Pk.smap[0] = J.smap[k];
            Pk.spitch[0] = J.smap_pitch[k];
        }
        run_passes(smem, g, g, g, 1, Pk, (uint32_t *)(smem + OFF_KEYS));
    }
}

// A region of a job: its cells and its level-0 extent.
struct Region {
    int rxi, ryi;        // region column and row
    int ncx, ncy;        // cells across and down (clipped at the grid edge)
    int xr1, yr1;        // level-0 end of the region (clipped at the image)
    Params P;
};

__device__ __forceinline__ Region region_of(const fg_job &J, int region) {
    Region R;
    R.ryi = region < (1 << 21) ? div_small(region, J.rx) : region / J.rx;
    R.rxi = region - R.ryi * J.rx;
    R.ncx = min(J.rcells, J.gw - R.rxi * J.rcells);
    R.ncy = min(J.rcells, J.gh - R.ryi * J.rcells);
    R.P.t = J.t;
    R.P.n = J.n;
    R.P.kind = J.score;
    R.P.smap[0] = R.P.smap[1] = R.P.smap[2] = nullptr;
    R.P.spitch[0] = R.P.spitch[1] = R.P.spitch[2] = 0;
    R.P.kc = J.n >> 2;
    R.P.k8 = J.n >> 1;
    R.P.cell = J.cell;
    R.P.rx0 = R.rxi * J.rcells * J.cell;
    R.P.ry0 = R.ryi * J.rcells * J.cell;
    R.P.ncx = R.ncx;
    R.xr1 = min(R.P.rx0 + R.ncx * J.cell, J.w[0]);
    R.yr1 = min(R.P.ry0 + R.ncy * J.cell, J.h[0]);
    return R;
}

__device__ __forceinline__ void keys_clear(uint32_t *keys, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) keys[i] = 0;
}

// Decode the region's cell keys into output slots.
__device__ void keys_write(const fg_job &J, const Region &R, const uint32_t *keys, int tid = threadIdx.x,
                           int nthreads = blockDim.x) {
    for (int i = tid; i < R.ncx * R.ncy; i += nthreads) {
        const int qy = div_small(i, R.ncx);   // i < MAX_KEYS
        const int cx = R.rxi * J.rcells + i - qy * R.ncx, cy = R.ryi * J.rcells + qy;
        const uint32_t key = keys[i];
        // fast_feature {x, y, score, level, reserved} as one little-endian word
        uint64_t f;
        if (key == 0) {
            f = 0x00FF0000FFFFFFFFull;
        } else {
            const int level = 7 - (int)((key >> 16) & 7u);
            const uint32_t local = 0xFFFFu - (key & 0xFFFFu);
            const int cw = J.cell >> level;
            const int ly = div_small((int)local, cw);   // local < cw * cw <= 2^16
            const uint32_t x = (uint32_t)(((cx * J.cell) >> level) + (int)local - ly * cw);
            const uint32_t y = (uint32_t)(((cy * J.cell) >> level) + ly);
            f = (uint64_t)(x | (y << 16)) | ((uint64_t)(key >> 19) << 32) | ((uint64_t)level << 48);
        }
        gstore<uint64_t>(J.out + (size_t)cy * J.gw + cx, f);
    }
}

__device__ void detect_region(const fg_job &J, int region, uint8_t *smem) {
    const Region R = region_of(J, region);
    uint32_t *keys = (uint32_t *)(smem + OFF_KEYS);
    __syncthreads();   // previous region's slot writes have read the keys
    keys_clear(keys, R.ncx * R.ncy);
    for (int sy0 = R.P.ry0; sy0 < R.yr1; sy0 += SUB)
        for (int sx0 = R.P.rx0; sx0 < R.xr1; sx0 += SUB)
            process_subtile(J, sx0, sy0, R.xr1, R.yr1, R.P, smem);
    __syncthreads();
    keys_write(J, R, keys);
}

// Cell keys of a region from the slots an earlier pass wrote (the inverse
// of keys_write).
__device__ void keys_from_slots(const fg_job &J, const Region &R, uint32_t *keys) {
    for (int i = threadIdx.x; i < R.ncx * R.ncy; i += blockDim.x) {
        const int qy = div_small(i, R.ncx);
        const int cx = R.rxi * J.rcells + i - qy * R.ncx, cy = R.ryi * J.rcells + qy;
        const uint64_t f = gload<uint64_t>(J.out + (size_t)cy * J.gw + cx);
        const uint32_t score = (uint32_t)(f >> 32) & 0xFFFFu;
        uint32_t key = 0;
        if (score) {
            const int level = (int)((f >> 48) & 0xFFu);
            const int cw = J.cell >> level;
            const int lx = (int)(f & 0xFFFFu) - ((cx * J.cell) >> level);
            const int ly = (int)((f >> 16) & 0xFFFFu) - ((cy * J.cell) >> level);
            key = (score << 19) | ((uint32_t)(7 - level) << 16) | (0xFFFFu - (uint32_t)(ly * cw + lx));
        }
        keys[i] = key;
    }
}

// Levels MAX_FUSED .. L-1 of a region, merged into the slots of levels below.
__device__ void detect_region_upper(const fg_job &J, int region, uint8_t *smem) {
    const Region R = region_of(J, region);
    uint32_t *keys = (uint32_t *)(smem + OFF_KEYS);
    __syncthreads();
    keys_from_slots(J, R, keys);
    for (int sy0 = R.P.ry0; sy0 < R.yr1; sy0 += SUB)
        for (int sx0 = R.P.rx0; sx0 < R.xr1; sx0 += SUB)
            process_subtile_upper(J, sx0, sy0, R.xr1, R.yr1, R.P, smem);
    __syncthreads();
    keys_write(J, R, keys);
}

// Threads that own a quad of a fused level-0 tile (at most 96 rows of 4).
constexpr int QUAD_THREADS = 8 * (96 / 4);
static_assert(SUB + 2 * (4 << (MAX_FUSED - 1)) <= 96, "fused tiles have at most 96 level-0 rows");

// Tile staging of the pipelined kernel: thread i owns the 16-byte chunk
// column i % 8 of level-0 tile rows 4(i/8) .. 4(i/8)+3 (workgroups of at
// least 256 threads cover a fused tile), so it holds whole 16 x 4 blocks and
// builds the 8 x 2 level-1 and 4 x 1 level-2 pixels they cover in registers.
//
// The loads go through a buffer resource over the plane rows the tile covers
// (H * P bytes of a plane are addressable): a row above or below the plane
// reads zero through the buffer's range check.  A chunk left or right of the
// plane is not loaded and keeps stale register values.  No pixel outside the
// plane is ever used as a pixel value (it is never testable, never inside a
// testable pixel's circle, and never written to a level plane), so the tile
// needs no zeros there.  Chunks a thread does not own keep stale values too,
// which quad_commit never reads.
__device__ __forceinline__ void quad_issue(TileRegs &R, const uint8_t *img, int H, int P, const Stage &st) {
    const int ch = threadIdx.x & 7, q = threadIdx.x >> 3;
    const int gx = st.tx + 16 * ch;
    if (ch >= (st.tw >> 4) || 4 * q >= st.th || gx < 0 || gx >= P) return;
    const int y0 = max(st.ty, 0), y1 = min(st.ty + st.th, H);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(img + (ptrdiff_t)y0 * P), (short)0, max(y1 - y0, 0) * P, 0x00020000);
    int off = (st.ty + 4 * q - y0) * P + gx;   // negative: out of range, reads zero
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        R.v[j] = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
        off += P;
    }
}

// Write the n-pixel piece w (n = 4 or 8, little-endian) of row y of a plane,
// starting at column x (a multiple of n), clipped to [sx, ex) x [sy, ey).
__device__ __forceinline__ void store_piece(uint8_t *plane, int P, int y, int x, uint64_t w, int n,
                                            const Geo &g) {
    if (y < g.sy || y >= g.ey || x + n <= g.sx || x >= g.ex) return;
    uint8_t *d = plane + (ptrdiff_t)y * P + x;
    if (x >= g.sx && x + n <= g.ex) {
        if (n == 8)
            gstore<uint64_t>(d, w);
        else
            gstore<uint32_t>(d, (uint32_t)w);
    } else {
        for (int i = 0; i < n; ++i)
            if (x + i >= g.sx && x + i < g.ex) gstore<uint8_t>(d + i, (uint8_t)(w >> (8 * i)));
    }
}

// Commit a quad-staged level-0 tile to LDS, build levels 1 and 2 of it into
// LDS from registers, and write the sub-tile's own level-1 and level-2 pixels
// to their planes.  A quad's rows past the tile (at most three, still inside
// the 96 level-0 rows of the LDS tile) are committed too: nothing reads them,
// and the level rows they feed lie past the level tiles.
__device__ void quad_commit(uint8_t *smem, const TileRegs &R, const Stage &st, const fg_job &J, const Geo &g1,
                            const Geo &g2) {
    const int ch = threadIdx.x & 7, q = threadIdx.x >> 3;
    if (ch >= (st.tw >> 4) || 4 * q >= st.th) return;
    uint8_t *t0 = smem + T0 + 4 * q * LP + 16 * ch;
#pragma unroll
    for (int j = 0; j < 4; ++j) *(u32x4 *)(t0 + j * LP) = R.v[j];
    const int nl = fused_levels(J);
    if (nl < 2) return;
    const u32x4 a = R.v[0], b = R.v[1], c = R.v[2], d = R.v[3];
    const uint32_t r0a = halve4(make_uint2(a.x, a.y), make_uint2(b.x, b.y));
    const uint32_t r0b = halve4(make_uint2(a.z, a.w), make_uint2(b.z, b.w));
    const uint32_t r1a = halve4(make_uint2(c.x, c.y), make_uint2(d.x, d.y));
    const uint32_t r1b = halve4(make_uint2(c.z, c.w), make_uint2(d.z, d.w));
    *(uint2 *)(smem + T1 + (2 * q) * LP + 8 * ch) = make_uint2(r0a, r0b);
    *(uint2 *)(smem + T1 + (2 * q + 1) * LP + 8 * ch) = make_uint2(r1a, r1b);
    const int x1 = (st.tx >> 1) + 8 * ch, y1 = (st.ty >> 1) + 2 * q;
    store_piece(J.lvl[1], J.pitch[1], y1, x1, (uint64_t)r0b << 32 | r0a, 8, g1);
    store_piece(J.lvl[1], J.pitch[1], y1 + 1, x1, (uint64_t)r1b << 32 | r1a, 8, g1);
    if (nl < 3) return;
    const uint32_t l2 = halve4(make_uint2(r0a, r0b), make_uint2(r1a, r1b));
    *(uint32_t *)(smem + T2 + q * LP + 4 * ch) = l2;
    store_piece(J.lvl[2], J.pitch[2], (st.ty >> 2) + q, (st.tx >> 2) + 4 * ch, l2, 4, g2);
}

// Issue the level-0 tile loads of a single-fused-sub-tile region.
__device__ __forceinline__ void region_prefetch(const fg_job &J, int region, TileRegs &T) {
    const Region R = region_of(J, region);
    quad_issue(T, J.lvl[0], J.h[0], J.pitch[0], fused_stage(J, R.P.rx0, R.P.ry0, R.xr1, R.yr1));
}

// Commit a prefetched region's tile and build its levels 1-2 (quad_commit).
__device__ __forceinline__ void region_commit(uint8_t *smem, const fg_job &J, int region, const TileRegs &T) {
    const Region R = region_of(J, region);
    const Stage st = fused_stage(J, R.P.rx0, R.P.ry0, R.xr1, R.yr1);
    Geo g0, g1, g2;
    describe_fused(J, R.P.rx0, R.P.ry0, R.xr1, R.yr1, st, g0, g1, g2);
    quad_commit(smem, T, st, J, g1, g2);
}

// Bijective block -> item map that gives each XCD (blocks are dealt to the 8
// XCDs round-robin) a contiguous run of items, so neighbouring regions share
// halo lines in the same L2.
__device__ __forceinline__ int xcd_item(int b, int n) {
    const int q = n >> 3, r = n & 7;
    const int xcd = b & 7, local = b >> 3;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// Score-map mode of a region: levels 0 .. F-1 from one load, no cell keys.
__device__ void scores_region(const fg_job &J, int region, uint8_t *smem) {
    const Region R = region_of(J, region);
    Params P = R.P;
    for (int l = 0; l < MAX_FUSED; ++l) {
        P.smap[l] = J.smap[l < J.levels ? l : 0];
        P.spitch[l] = J.smap_pitch[l < J.levels ? l : 0];
    }
    for (int sy0 = P.ry0; sy0 < R.yr1; sy0 += SUB)
        for (int sx0 = P.rx0; sx0 < R.xr1; sx0 += SUB) process_subtile(J, sx0, sy0, R.xr1, R.yr1, P, smem);
}

// Score-map mode of levels MAX_FUSED.. of a region.
__device__ void scores_region_upper(const fg_job &J, int region, uint8_t *smem) {
    const Region R = region_of(J, region);
    Params P = R.P;
    P.smap[0] = J.smap[MAX_FUSED];   // non-null selects the mode; each level sets its own
    for (int sy0 = P.ry0; sy0 < R.yr1; sy0 += SUB)
        for (int sx0 = P.rx0; sx0 < R.xr1; sx0 += SUB) process_subtile_upper(J, sx0, sy0, R.xr1, R.yr1, P, smem);
}

// Standalone NMS over (2r+1) x (2r+1) neighbourhoods and the cell arg-max
// across levels, from global score maps (J.smap).  One workgroup per region;
// each level's part of the region is walked in 64 x 64 tiles staged in LDS
// with an r-pixel halo (zero outside the map).  Every tile pixel gets the
// rank (score << 16) | (0xFFFF - its row-major index in the tile) (0 for
// score 0): ranks are unique, and a higher rank means a higher score or, on
// a tie, an earlier pixel, so a pixel survives exactly when its rank is the
// maximum of its window.  The window maximum is separable: a row pass, then
// a column pass, 2(2r+1) comparisons per pixel.
constexpr int NMS_TILE = SUB + 2 * 4;
constexpr int NMS_HMAX_OFF = NMS_TILE * NMS_TILE * 4;
constexpr int NMS_KEYS_OFF = NMS_HMAX_OFF + NMS_TILE * SUB * 4;
size_t nms_smem_bytes() { return (size_t)NMS_KEYS_OFF + MAX_KEYS * 4; }

__global__ void __launch_bounds__(512) nms_grid_kernel(fg_job J, int radius) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const int region = xcd_item(blockIdx.x, gridDim.x);
    const Region R = region_of(J, region);
    uint32_t *rank = (uint32_t *)smem;
    uint32_t *hmax = (uint32_t *)(smem + NMS_HMAX_OFF);
    uint32_t *keys = (uint32_t *)(smem + NMS_KEYS_OFF);
    keys_clear(keys, R.ncx * R.ncy);
    const int r = radius;
    for (int k = 0; k < J.levels; ++k) {
        const int x0 = R.P.rx0 >> k, y0 = R.P.ry0 >> k;
        const int x1 = min(R.xr1 >> k, J.w[k]), y1 = min(R.yr1 >> k, J.h[k]);
        const int cw = J.cell >> k;
        const uint16_t *map = J.smap[k];
        const int mp = J.smap_pitch[k];
        for (int ty0 = y0; ty0 < y1; ty0 += SUB) {
            for (int tx0 = x0; tx0 < x1; tx0 += SUB) {
                const int tw = min(SUB, x1 - tx0), th = min(SUB, y1 - ty0);
                const int TW = tw + 2 * r, TH = th + 2 * r;
                __syncthreads();   // the previous tile has been read
                for (int i = threadIdx.x; i < TW * TH; i += blockDim.x) {
                    const int yy = div_small(i, TW), xx = i - yy * TW;
                    const int gx = tx0 - r + xx, gy = ty0 - r + yy;
                    const uint32_t sc = gx >= 0 && gx < J.w[k] && gy >= 0 && gy < J.h[k]
                                            ? gload<uint16_t>(map + (ptrdiff_t)gy * mp + gx) : 0u;
                    rank[i] = sc ? (sc << 16) | (0xFFFFu - (uint32_t)i) : 0u;
                }
                __syncthreads();
                // row pass: the maximum over columns xx-r .. xx+r of every row
                for (int i = threadIdx.x; i < tw * TH; i += blockDim.x) {
                    const int yy = div_small(i, tw), xx = i - yy * tw;
                    const uint32_t *q = rank + yy * TW + xx;   // columns xx .. xx+2r
                    uint32_t m = q[0];
                    for (int d = 1; d <= 2 * r; ++d) m = max(m, q[d]);
                    hmax[i] = m;
                }
                __syncthreads();
                // column pass over the tile's own pixels, then the cell keys
                for (int i = threadIdx.x; i < tw * th; i += blockDim.x) {
                    const int yy = div_small(i, tw), xx = i - yy * tw;
                    const uint32_t own = rank[(yy + r) * TW + xx + r];
                    if (own == 0) continue;
                    uint32_t m = 0;
                    for (int d = 0; d <= 2 * r; ++d) m = max(m, hmax[(yy + d) * tw + xx]);
                    if (m != own) continue;
                    const uint32_t sc = own >> 16;
                    const int ox = tx0 + xx - x0, oy = ty0 + yy - y0;
                    const int cx = div_small(ox, cw), cy = div_small(oy, cw);
                    const uint32_t local = (uint32_t)((oy - cy * cw) * cw + (ox - cx * cw));
                    const uint32_t key = (sc << 19) | ((uint32_t)(7 - k) << 16) | (0xFFFFu - local);
                    atomicMax(&keys[cy * R.ncx + cx], key);
                }
            }
        }
    }
    __syncthreads();
    keys_write(J, R, keys);
}

__global__ void __launch_bounds__(512) score_plain_kernel(fg_job J) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    scores_region(J, xcd_item(blockIdx.x, gridDim.x), smem);
}

__global__ void __launch_bounds__(512) score_upper_plain_kernel(fg_job J) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    scores_region_upper(J, xcd_item(blockIdx.x, gridDim.x), smem);
}

__global__ void __launch_bounds__(512) detect_plain_kernel(fg_job J) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    detect_region(J, xcd_item(blockIdx.x, gridDim.x), smem);
}

// Levels MAX_FUSED.. of one frame, one region per block.
__global__ void __launch_bounds__(512) detect_upper_plain_kernel(fg_job J) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    detect_region_upper(J, xcd_item(blockIdx.x, gridDim.x), smem);
}

// Levels MAX_FUSED.. of the batch's deep jobs, one listed region per block.
__global__ void __launch_bounds__(512) detect_upper_batch_kernel(const fg_job *__restrict__ jobs,
                                                                 const fg_item *__restrict__ items) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const fg_item it = items[blockIdx.x];
    detect_region_upper(jobs[it.job], (int)it.region, smem);
}

// Persistent batched detectors.  Work items are regions of all jobs (items[]
// gives each one's job and region, row by row within a job, whole regions
// first and clipped ones last), split over FG_QUEUES queues.  The list is
// cut into runs of FG_QUEUE_RUN consecutive items dealt round-robin: queue c
// holds runs c, c + 8, c + 16, ... and then, past the last full round of
// runs, items c, c + 8, ... of the remainder, so the queues stay within one
// run of each other.  Workgroup g uses queue g % 8; it starts with that
// queue's positions g / 8 and g / 8 + n (n workgroups on the queue) and then
// takes position 2n + k for its k-th ticket of the queue's counter.  Eight
// heads on separate cache lines keep the tickets from queueing behind each
// other.  Workgroups are placed on the XCDs round-robin, so one queue's
// workgroups share one XCD and its L2: a run's regions lie side by side in
// their frame and share the cache lines of their tiles, which a run of one
// region (neighbours on eight different L2s) fetches again from memory.
struct Queue {
    unsigned *head;
    int c, n, first;    // queue index, its workgroups, this workgroup's first position
};

__device__ __forceinline__ Queue queue_of(unsigned *counter) {
    Queue q;
    const int G = (int)gridDim.x;
    q.c = (int)(blockIdx.x % FG_QUEUES);
    q.first = (int)(blockIdx.x / FG_QUEUES);
    q.n = (G - q.c + FG_QUEUES - 1) / FG_QUEUES;
    q.head = counter + q.c * FG_QUEUE_STRIDE;
    return q;
}

// Item at queue position pos, or total past the end.
__device__ __forceinline__ int queue_item(const Queue &q, long long pos, int total) {
    const long long runs = total / (FG_QUEUES * FG_QUEUE_RUN);   // full rounds of runs
    const long long in_runs = runs * FG_QUEUE_RUN;               // positions per queue inside them
    const long long it = pos < in_runs
                             ? ((pos / FG_QUEUE_RUN) * FG_QUEUES + q.c) * FG_QUEUE_RUN + pos % FG_QUEUE_RUN
                             : in_runs * FG_QUEUES + q.c + (long long)FG_QUEUES * (pos - in_runs);
    return it < total ? (int)it : total;
}

// A ticket of the queue.  The ticket's value is first needed after the
// passes of a whole region, so no wait may follow the atomic at once (the
// library is built without the atomic optimiser, whose wave-level rewrite
// reads the result right after the atomic).
__device__ __forceinline__ unsigned queue_ticket(const Queue &q) {
    return __hip_atomic_fetch_add(q.head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The last workgroup out re-arms the queues for the next launch (every ticket
// a workgroup drew has been resolved by then).
__device__ __forceinline__ void queue_exit(unsigned *counter) {
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned done = atomicAdd(&counter[FG_EXIT_WORD], 1u);
        if (done == gridDim.x - 1) {
            for (int c = 0; c < FG_QUEUES; ++c) atomicExch(&counter[c * FG_QUEUE_STRIDE], 0u);
            atomicExch(&counter[FG_EXIT_WORD], 0u);
        }
    }
}

// Pipelined kernel, for batches whose regions are all single fused sub-tiles
// and workgroups of at least 256 threads (32 quads of tile rows cover a
// fused tile).  Per region there are three workgroup barriers:
//   [A] the previous region's NMS is done; this region's levels 0-2 are in
//       LDS: write the previous region's slots, clear the score maps and
//       this region's cell keys (two key buffers alternate);
//   [B] draw the ticket of the region after next, run the compass, 8-point
//       and scoring passes; thread 0 resolves the ticket;
//   [C] the scores are complete and the tiles are no longer read: commit
//       the next region's level-0 tile (loaded into registers one region
//       earlier) to LDS, build its levels 1-2 from the registers into LDS
//       and their planes, start loading the tile after it, then run NMS into
//       the keys.
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 4)))
detect_batch_kernel(const fg_job *__restrict__ jobs, const fg_item *__restrict__ items, int total,
                    unsigned *counter) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    // s_next[b] carries the item after next from thread 0 to the workgroup;
    // the two buffers alternate, so a value is never overwritten before every
    // wave has read it.
    __shared__ int s_next[2];
    const Queue q = queue_of(counter);
    int item = queue_item(q, q.first, total);
    if (item >= total) {   // a queue with fewer items than workgroups
        queue_exit(counter);
        return;
    }
    int next = queue_item(q, q.first + (long long)q.n, total);
    fg_item il = items[item];
    fg_item in = next < total ? items[next] : fg_item{0u, 0u};
    TileRegs T;
    region_prefetch(jobs[il.job], (int)il.region, T);
    region_commit(smem, jobs[il.job], (int)il.region, T);
    if (next < total) region_prefetch(jobs[in.job], (int)in.region, T);
    fg_item prev{0u, 0u};
    bool have_prev = false;
    int b = 0;
    GroupCache gcache{0u, 0u, -1};
    while (item < total) {
        const fg_job &J = jobs[il.job];   // uniform: read through the scalar cache
        const Region R = region_of(J, (int)il.region);
        const Stage st = fused_stage(J, R.P.rx0, R.P.ry0, R.xr1, R.yr1);
        uint32_t *keys = (uint32_t *)(smem + (b ? OFF_KEYS2 : OFF_KEYS));
        __syncthreads();   // [A]
        zero_lds(smem + OFF_M0, OFF_KEYS - OFF_M0);
        keys_clear(keys, R.ncx * R.ncy);
        Geo g0, g1, g2;
        describe_fused(J, R.P.rx0, R.P.ry0, R.xr1, R.yr1, st, g0, g1, g2);
        __syncthreads();   // [B]
        // thread 0 only, read only where it was set; left without a value
        // elsewhere so that no copy of the atomic's result (which would wait
        // for it at once) is needed where the branch rejoins
        unsigned ticket;
        // (the first lane of the last wave: wave 0 already carries the extra
        // compass round of a full region, so it sets the region's pace)
        if (threadIdx.x == blockDim.x - 64 && next < total) ticket = queue_ticket(q);
        int after = total;
        // the staged geometry depends only on the fused level count and the
        // region's size once its origin is 16-aligned across and 4-aligned down
        const int gkey = (R.P.rx0 & 15) == 0 && (R.P.ry0 & 3) == 0
                             ? fused_levels(J) | (R.xr1 - R.P.rx0) << 2 | (R.yr1 - R.P.ry0) << 9
                             : -1;
        run_passes(
            smem, g0, g1, g2, fused_levels(J), R.P, keys, &gcache, gkey,
            [&]() {
                if (threadIdx.x == blockDim.x - 64)
                    s_next[b] = next < total ? queue_item(q, 2LL * q.n + ticket, total) : total;
            },
            [&]() {   // after [C]
                after = __builtin_amdgcn_readfirstlane(s_next[b]);
                if (next < total) {
                    region_commit(smem, jobs[in.job], (int)in.region, T);
                    if (after < total) {
                        const fg_item ia = items[after];
                        region_prefetch(jobs[ia.job], (int)ia.region, T);
                    }
                }
                // the previous region's slots, written by the threads the
                // tile commit leaves idle (quads past level-0 row 96); its
                // keys buffer is next cleared after the next [A]
                if (have_prev && threadIdx.x >= QUAD_THREADS) {
                    const fg_job &Jp = jobs[prev.job];
                    keys_write(Jp, region_of(Jp, (int)prev.region),
                               (const uint32_t *)(smem + (b ? OFF_KEYS : OFF_KEYS2)), threadIdx.x - QUAD_THREADS,
                               blockDim.x - QUAD_THREADS);
                }
            });
        prev = il;
        have_prev = true;
        item = next;
        il = in;
        next = after;
        in = after < total ? items[after] : fg_item{0u, 0u};
        b ^= 1;
    }
    __syncthreads();
    if (have_prev) {   // the last region used the buffer before the final flip of b
        const fg_job &Jp = jobs[prev.job];
        keys_write(Jp, region_of(Jp, (int)prev.region), (const uint32_t *)(smem + (b ? OFF_KEYS : OFF_KEYS2)));
    }
    queue_exit(counter);
}

// Generic persistent kernel: any region size and workgroup size, one region
// at a time.
__global__ void __launch_bounds__(512) detect_batch_generic_kernel(const fg_job *__restrict__ jobs,
                                                                   const fg_item *__restrict__ items,
                                                                   int total, unsigned *counter) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    __shared__ int s_item;
    const Queue q = queue_of(counter);
    for (int k = 0;; ++k) {
        __syncthreads();   // every wave has read the previous s_item
        if (threadIdx.x == 0) {
            long long pos = q.first + (long long)k * q.n;
            if (k >= 2) pos = 2LL * q.n + queue_ticket(q);
            s_item = queue_item(q, pos, total);
        }
        __syncthreads();
        const int item = s_item;
        if (item >= total) break;
        const fg_item it = items[item];
        detect_region(jobs[it.job], (int)it.region, smem);
    }
    queue_exit(counter);
}

// Pyramid level k from level k-1, four output pixels per thread.
__device__ __forceinline__ void pyr_row_words(const uint8_t *src, int sp, uint8_t *dst, int dp,
                                              int dw, int y, int w) {
    const int x = 4 * w;
    const uint8_t *s0 = src + (size_t)(2 * y) * sp + 2 * x;
    const uint8_t *s1 = s0 + sp;
    uint8_t *d = dst + (size_t)y * dp + x;
    if (x + 4 <= dw) {
        const u32x2 a = gload<u32x2>(s0), b = gload<u32x2>(s1);
        gstore<uint32_t>(d, halve4(make_uint2(a.x, a.y), make_uint2(b.x, b.y)));
    } else {
        for (int q = 0; q < dw - x; ++q)
            gstore<uint8_t>(d + q, (uint8_t)((gload<uint8_t>(s0 + 2 * q) + gload<uint8_t>(s0 + 2 * q + 1) +
                                              gload<uint8_t>(s1 + 2 * q) + gload<uint8_t>(s1 + 2 * q + 1) + 2) >>
                                             2));
    }
}

__global__ void pyr_kernel(const uint8_t *__restrict__ src, int sp, uint8_t *__restrict__ dst,
                           int dw, int dh, int dp) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (4 * w >= dw || y >= dh) return;
    pyr_row_words(src, sp, dst, dp, dw, y, w);
}

__global__ void pyr_batch_kernel(const fg_job *__restrict__ jobs, int k) {
    const fg_job &J = jobs[blockIdx.z];
    if (k >= J.levels || k < MAX_FUSED) return;
    const int w = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
    if (4 * w >= J.w[k] || y >= J.h[k]) return;
    pyr_row_words(J.lvl[k - 1], J.pitch[k - 1], J.lvl[k], J.pitch[k], J.w[k], y, w);
}

}  // namespace

void fg_job_layout(fg_job &j, const fg_launch &L) {
    j.gw = (j.w[0] + j.cell - 1) / j.cell;
    j.gh = (j.h[0] + j.cell - 1) / j.cell;
    // cells per region side: a multiple of 16/gcd(cell,16), so regions and
    // sub-tiles start on 16-pixel boundaries
    int g = 16;
    while (j.cell % g) g >>= 1;
    const int m = 16 / g;
    int rc = L.region / j.cell;
    rc = (rc + m - 1) / m * m;
    if (rc < m) rc = m;
    if (rc > MAX_RCELLS) rc = MAX_RCELLS / m * m;
    j.rcells = rc;
    j.rx = (j.gw + rc - 1) / rc;
    j.ry = (j.gh + rc - 1) / rc;
}

hipError_t fg_launch_pyramid(const fg_job &j, hipStream_t s) {
    for (int k = 1; k < j.levels; ++k) {
        dim3 grid(((j.w[k] + 3) / 4 + 63) / 64, j.h[k]);
        hipLaunchKernelGGL(pyr_kernel, grid, dim3(64), 0, s, j.lvl[k - 1], j.pitch[k - 1], j.lvl[k],
                           j.w[k], j.h[k], j.pitch[k]);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t fg_launch_plain(const fg_job &j, const fg_launch &L, hipStream_t s) {
    hipLaunchKernelGGL(detect_plain_kernel, dim3(j.rx * j.ry), dim3(L.block),
                       fg_smem_bytes(L.block), s, j);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || j.levels <= MAX_FUSED) return e;
    // deeper levels: built from the fused pass's last level, then detected
    for (int k = MAX_FUSED; k < j.levels; ++k) {
        dim3 grid(((j.w[k] + 3) / 4 + 63) / 64, j.h[k]);
        hipLaunchKernelGGL(pyr_kernel, grid, dim3(64), 0, s, j.lvl[k - 1], j.pitch[k - 1], j.lvl[k],
                           j.w[k], j.h[k], j.pitch[k]);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(detect_upper_plain_kernel, dim3(j.rx * j.ry), dim3(L.block),
                       fg_smem_bytes(L.block), s, j);
    return hipGetLastError();
}

hipError_t fg_launch_score_maps(const fg_job &j, const fg_launch &L, hipStream_t s) {
    hipLaunchKernelGGL(score_plain_kernel, dim3(j.rx * j.ry), dim3(L.block), fg_smem_bytes(L.block), s, j);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || j.levels <= MAX_FUSED) return e;
    for (int k = MAX_FUSED; k < j.levels; ++k) {
        dim3 grid(((j.w[k] + 3) / 4 + 63) / 64, j.h[k]);
        hipLaunchKernelGGL(pyr_kernel, grid, dim3(64), 0, s, j.lvl[k - 1], j.pitch[k - 1], j.lvl[k],
                           j.w[k], j.h[k], j.pitch[k]);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(score_upper_plain_kernel, dim3(j.rx * j.ry), dim3(L.block), fg_smem_bytes(L.block),
                       s, j);
    return hipGetLastError();
}

hipError_t fg_launch_nms_grid(const fg_job &j, int radius, hipStream_t s) {
    hipLaunchKernelGGL(nms_grid_kernel, dim3(j.rx * j.ry), dim3(256), nms_smem_bytes(), s, j, radius);
    return hipGetLastError();
}

hipError_t fg_launch_batch(const fg_job *jobs_dev, const fg_item *items, int njobs, int total,
                           int total_upper, int max_levels, int max_w1, int max_h1, bool all_single,
                           unsigned *counter, const fg_launch &L, hipStream_t s) {
    int blocks = L.num_cu * L.blocks_per_cu;
    if (blocks > total) blocks = total;
    if (blocks < 1) blocks = 1;
    if (all_single && L.block >= 256)
        hipLaunchKernelGGL(detect_batch_kernel, dim3(blocks), dim3(L.block), fg_smem_bytes(L.block), s,
                           jobs_dev, items, total, counter);
    else
        hipLaunchKernelGGL(detect_batch_generic_kernel, dim3(blocks), dim3(L.block), fg_smem_bytes(L.block), s,
                           jobs_dev, items, total, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || total_upper == 0) return e;
    int mw = max_w1, mh = max_h1;
    for (int k = 2; k < max_levels; ++k) {
        mw = (mw >> 1) > 0 ? (mw >> 1) : 1;
        mh = (mh >> 1) > 0 ? (mh >> 1) : 1;
        if (k < MAX_FUSED) continue;
        dim3 grid(((mw + 3) / 4 + 63) / 64, mh, njobs);
        hipLaunchKernelGGL(pyr_batch_kernel, grid, dim3(64), 0, s, jobs_dev, k);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(detect_upper_batch_kernel, dim3(total_upper), dim3(L.block), fg_smem_bytes(L.block),
                       s, jobs_dev, items + total);
    return hipGetLastError();
}
