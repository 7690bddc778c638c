// Internal declarations shared by the HIP translation units of libekm.
// Device helpers: Morton codes, conservative FP32 error bounds, exact
// fixed-point decomposition of coordinates, wave-level reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <array>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/ekm.h"

namespace ekm {

constexpr int WAVE = 64;
constexpr int MAX_LEAF = 64;     // a leaf fits one wave
constexpr int GROUP_LEAVES = 8;  // most consecutive leaves sharing one centroid-tree descent (one wave)
constexpr int DEFAULT_G_2D = 6;  // default leaves per group in 2D (3D: GROUP_LEAVES); measured on 1e6 hotspot points
// Leaves with more candidates than this go to the per-leaf pass.  At the
// main pass's list capacity, only leaves whose candidate list does not fit
// are deferred (measured: deferring crowded leaves cost more in the extra
// pass than it saved in the main one); the small-list test mode lowers it.
constexpr int HEAVY_M = 256;
// Workgroups of the per-leaf pass (one per CU): workgroup b of W takes the
// deferred leaves b, b + W, ... of the step's list.  Many leaves are
// deferred only with many centroids per cloud (crowded candidate lists):
// then every CU takes part; otherwise a quarter of them, which keeps the
// usually empty pass short.
inline int heavy_blocks(int64_t kmax) { return kmax >= 8192 ? 256 : 64; }
// Waves per workgroup of the indexed main pass (one group per wave; in 2D the
// waves claim units of work from a shared list, and 8 of them balance long
// units better than 4; the 3D kernel keeps 4, its registers allow no more).
template <int D>
constexpr int MAIN_WAVES = D == 2 ? 8 : 4;
inline int main_waves(int d) { return d == 2 ? MAIN_WAVES<2> : MAIN_WAVES<3>; }
constexpr int TREE_BUCKET = 8;   // centroids per centroid-tree leaf bucket
constexpr int TREE_MAX_LEVELS = 8;
constexpr int TREE_START_MAX = 512; // nodes a descent evaluates at its first level
constexpr int NSTAT = 12;      // per-block statistics slots (see StatSlot); even (read as pairs)
constexpr int MAX_FIX_BITS = 94;
constexpr int FIX64_BITS = 56;  // per-point fixed-point values of this size sum over a wave within int64

enum StatSlot {
    ST_CHANGED = 0,
    ST_EVALS = 1,
    ST_SINGLE = 2,        // points in leaves with a single candidate (batch-assigned)
    ST_RECHECK = 3,
    ST_CANDS = 4,
    ST_FALLBACK_PTS = 5,  // points decided by the scan of all k centroids (no candidate list fitted)
    ST_KEEP_LEAF_PTS = 6, // points of leaves kept whole by the inter bound (Eq. (5))
    ST_KEEP_PTS = 7,      // points kept by the per-point inter bound (Eq. (4))
    ST_DEFERRED = 8,      // leaves handed to the per-leaf pass
    ST_GROUP_OVF = 9,     // groups whose candidate list did not fit (searched leaf by leaf)
    ST_GROUP_SKIP = 10,   // groups with every leaf kept: no centroid-tree descent
    ST_REGION_PTS = 11,   // points of groups (regions) whose candidate list held one centroid
};

// Device-side loop control of a context (ctl[]): the step kernels of a
// kmeans_run return at once when CTL_STOP is set, so a run can be launched
// in chunks of steps (as graphs) without the host waiting for each step.
enum CtlSlot {
    CTL_STOP = 0,      // nonzero: the run is over (stable, or max_iter steps done)
    CTL_RUN_ITERS = 1, // steps done by the current run
    CTL_STEPS = 2,     // steps done by the context (0: no previous centroids)
    CTL_MAX_ITER = 3,  // the current run's max_iter (a large value outside runs)
    CTL_STABLE = 4,    // the current run stops when the assignment is stable
    CTL_N = 8,
};
constexpr int RUN_CHUNK = 8;  // steps per launch group (graph) of kmeans_run
constexpr int RUN_AHEAD = 3;  // launch groups kmeans_run keeps queued while it waits for an earlier one
constexpr int HIST_ROWS = 1024; // per-step statistics rows a context holds from the start

// Common cluster of a leaf's points (leaf_own): a centroid id when every
// point of the leaf is assigned to it, else one of these.
constexpr int OWN_MIXED = -1; // points of several clusters
constexpr int OWN_NONE = -2;  // not assigned yet (before the first step)

// ------------------------------------------------------------------------
// Morton codes on a 2^b grid per dimension over the data bounding box.
// 2D: 16 bits per dimension (32-bit key); 3D: 10 bits per dimension (30-bit).
// ------------------------------------------------------------------------
__host__ __device__ inline uint32_t spread2(uint32_t v)
{
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}
__host__ __device__ inline uint32_t spread3(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
inline constexpr int morton_bits(int d) { return d == 2 ? 16 : 10; }
inline constexpr int key_bits(int d) { return d == 2 ? 32 : 30; }

struct Grid {
    float lo[3];
    float scale[3]; // cells per unit length
};

__device__ inline uint32_t quantize(float v, float lo, float scale, int bits)
{
    float q = floorf((v - lo) * scale);
    float top = (float)((1u << bits) - 1u);
    q = fminf(fmaxf(q, 0.0f), top); // NaN-free inputs only
    return (uint32_t)q;
}

template <int D>
__device__ inline uint32_t morton_key(const float *p, const Grid &g)
{
    if (D == 2)
        return spread2(quantize(p[0], g.lo[0], g.scale[0], 16)) |
               (spread2(quantize(p[1], g.lo[1], g.scale[1], 16)) << 1);
    return spread3(quantize(p[0], g.lo[0], g.scale[0], 10)) |
           (spread3(quantize(p[1], g.lo[1], g.scale[1], 10)) << 1) |
           (spread3(quantize(p[2], g.lo[2], g.scale[2], 10)) << 2);
}

// ------------------------------------------------------------------------
// Conservative FP32 decisions.
//
// For an FP32 point x and an FP64 centroid c with c' = fl32(c):
//   D' = exact sum (x_i - c'_i)^2,  s = FP32 evaluation of D' (<= d+2
//   roundings per term, so |s - D'| <= gamma D' + tau with gamma ~ (d+2)u,
//   tau covering underflow),  |sqrt(D') - sqrt(D)| <= ||c - c'|| <= e,
//   and the canonical FP64 D64 is within (d+2)w of the exact D.
// All these relative errors are far below MARGIN = 2^-16, which also covers
// the FP32 sqrt and the few roundings of the tests themselves.
// ------------------------------------------------------------------------
constexpr float MARGIN_UP = 1.0f + 0x1p-16f;
constexpr float MARGIN_DN = 1.0f - 0x1p-16f;
constexpr float TAU = 0x1p-120f;

// Upper bound on sqrt(D64) given FP32 s (of the centroid that will be chosen).
__device__ inline float dist_hi(float s, float e) { return sqrtf(s + TAU) * MARGIN_UP + e; }
// Lower bound on sqrt(D64) given FP32 s.
__device__ inline float dist_lo(float s, float e) { return sqrtf(fmaxf(s - TAU, 0.0f)) * MARGIN_DN - e; }

// A bound T on FP32 squared distances with: dist_lo(s, e) <= h implies
// s <= T (T is loose on purpose; it only has to keep every such s).
__device__ inline float lo_inverse(float h, float e)
{
    const float r = (h + e) * MARGIN_UP * MARGIN_UP;
    return r * r * MARGIN_UP + TAU;
}

// True when the FP32 best (s1) is certainly the FP64 argmin against every
// centroid whose FP32 value is >= s2.
__device__ inline bool margin_safe(float s1, float s2, float e) { return dist_lo(s2, e) > dist_hi(s1, e); }

// Pruning threshold on FP32 squared box distances from an exact-distance
// bound: when every point of the box is within exact distance R of some
// existing centroid (not necessarily the same one), any centroid whose FP32
// min-distance to the box exceeds prune_threshold_r(R, e) is strictly
// farther (in exact and in FP64 distance) from every point of the box than
// that point's centroid: its exact distance exceeds (R + e) (1 + 2^-16)^2
// less e, and the relative gap dwarfs the FP64 rounding.
__device__ inline float prune_threshold_r(float R, float e)
{
    float r = (R + e) * MARGIN_UP * MARGIN_UP;
    return r * r * MARGIN_UP + TAU;
}

// The same with U = an FP32 max-distance from the box to one existing
// centroid (its exact distance from every point is at most dist_hi(U, e)).
__device__ inline float prune_threshold(float U, float e) { return prune_threshold_r(dist_hi(U, e), e); }

// Upper bound (FP32, rounded up) on R + drift for exact-distance bounds R
// and centroid drift bounds (non-negative; +inf stays +inf).
__device__ inline float bound_add(float R, float drift) { return (R + drift) * MARGIN_UP; }

// Inter bound (Eq. (4), (5)): every point within exact distance r of c_j,
// where every other centroid is at exact distance >= cb from c_j, is
// strictly nearer to c_j when 2 r < cb (triangle inequality).  s: an FP32
// squared distance (or box max-distance) bounding r through dist_hi;
// cb_s: the smallest FP32 squared distance from fl32(c_j) to another fl32
// centroid, so dist_lo(cb_s, 2e) <= cb (each centroid is within e of its
// fl32 copy).  The factor 1 + 2^-14 keeps the gap far above the FP32
// rounding of the test and the FP64 rounding of the canonical distances,
// so the kept centroid is also the strict FP64 argmin.
__device__ inline bool inter_keep(float cb_s, float s, float e)
{
    return dist_lo(cb_s, 2.0f * e) > 2.0f * dist_hi(s, e) * (1.0f + 0x1p-14f);
}

template <int D>
__device__ inline float sqdist32(const float *x, const float *c)
{
    float t = x[0] - c[0];
    float s = t * t;
#pragma unroll
    for (int i = 1; i < D; ++i) {
        t = x[i] - c[i];
        s = fmaf(t, t, s);
    }
    return s;
}

// Canonical FP64 squared distance: rounded differences, rounded squares,
// left-to-right sum, no contraction (this library is built with
// -ffp-contract=off, and the pragma pins it here as well).
template <int D>
__device__ inline double sqdist64(const double *x, const double *c)
{
#pragma clang fp contract(off)
    double t = x[0] - c[0];
    double s = t * t;
#pragma unroll
    for (int i = 1; i < D; ++i) {
        t = x[i] - c[i];
        s = s + t * t;
    }
    return s;
}

// Box distances (FP32).  lo/hi: leaf box; c: point.
template <int D>
__device__ inline float box_mind(const float *lo, const float *hi, const float *c)
{
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        float g = fmaxf(fmaxf(lo[i] - c[i], c[i] - hi[i]), 0.0f);
        s = fmaf(g, g, s);
    }
    return s;
}
template <int D>
__device__ inline float box_maxd(const float *lo, const float *hi, const float *c)
{
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        float g = fmaxf(fabsf(c[i] - lo[i]), fabsf(hi[i] - c[i]));
        s = fmaf(g, g, s);
    }
    return s;
}
// Box-to-box: min and max over point pairs.
template <int D>
__device__ inline float bb_mind(const float *alo, const float *ahi, const float *blo, const float *bhi)
{
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        float g = fmaxf(fmaxf(alo[i] - bhi[i], blo[i] - ahi[i]), 0.0f);
        s = fmaf(g, g, s);
    }
    return s;
}
template <int D>
__device__ inline float bb_maxd(const float *alo, const float *ahi, const float *blo, const float *bhi)
{
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        float g = fmaxf(fabsf(bhi[i] - alo[i]), fabsf(ahi[i] - blo[i]));
        s = fmaf(g, g, s);
    }
    return s;
}

// ------------------------------------------------------------------------
// Exact fixed-point coordinates.  Every coordinate v of the data set is an
// integer multiple of 2^-S (S fixed at init), so V = v * 2^S is an integer
// of at most MAX_FIX_BITS bits including the sum over all points.  V is kept
// as hi * 2^32 + lo with lo in [0, 2^32): sums of lo fit int64 for n < 2^31,
// sums of hi fit int64 because the total stays below 2^94.
// ------------------------------------------------------------------------
__device__ inline void fix_split_f32(float v, int S, int64_t &hi, int64_t &lo)
{
    uint32_t b = __float_as_uint(v);
    uint32_t ex = (b >> 23) & 0xffu;
    int64_t m = (int64_t)(b & 0x7fffffu);
    int e2;
    if (ex == 0) {
        e2 = -149;
    } else {
        m |= 0x800000;
        e2 = (int)ex - 150;
    }
    int sh = e2 + S;
    // sh < 0 only for values whose trailing mantissa zeros make the right
    // shift exact (S is chosen from each value's lowest set bit).
    unsigned __int128 mag = sh >= 0 ? ((unsigned __int128)(uint64_t)m << sh)
                                    : (unsigned __int128)(-sh >= 64 ? 0ull : ((uint64_t)m >> (-sh)));
    __int128 V = (b >> 31) ? -(__int128)mag : (__int128)mag;
    hi = (int64_t)(V >> 32);
    lo = (int64_t)(uint32_t)(uint64_t)V;
}

// The same value as one int64 when it has at most FIX64_BITS bits (the
// shift is then in [0, FIX64_BITS - 24] or a right shift of trailing zeros).
__device__ inline int64_t fix_f32(float v, int S)
{
    const uint32_t b = __float_as_uint(v);
    const uint32_t ex = (b >> 23) & 0xffu;
    const uint32_t m = ex ? ((b & 0x7fffffu) | 0x800000u) : (b & 0x7fffffu);
    const int sh = (ex ? (int)ex - 150 : -149) + S;
    const int64_t mag = sh >= 0 ? ((int64_t)m << sh) : (int64_t)(m >> (-sh > 31 ? 31 : -sh));
    return (b >> 31) ? -mag : mag;
}

__device__ inline void fix_split_f64(double v, int S, int64_t &hi, int64_t &lo)
{
    uint64_t b = (uint64_t)__double_as_longlong(v);
    uint32_t ex = (uint32_t)((b >> 52) & 0x7ffu);
    int64_t m = (int64_t)(b & 0xfffffffffffffull);
    int e2;
    if (ex == 0) {
        e2 = -1074;
    } else {
        m |= (int64_t)1 << 52;
        e2 = (int)ex - 1075;
    }
    int sh = e2 + S;
    // sh < 0 only for values whose trailing mantissa zeros make the right
    // shift exact (S is chosen from each value's lowest set bit).
    unsigned __int128 mag = sh >= 0 ? ((unsigned __int128)(uint64_t)m << sh)
                                    : (unsigned __int128)(-sh >= 64 ? 0ull : ((uint64_t)m >> (-sh)));
    __int128 V = (b >> 63) ? -(__int128)mag : (__int128)mag;
    hi = (int64_t)(V >> 32);
    lo = (int64_t)(uint32_t)(uint64_t)V;
}

// Exponents of the lowest and highest set bit of a nonzero value.
__device__ inline void bits_f32(float v, int &elsb, int &emsb)
{
    uint32_t b = __float_as_uint(v);
    uint32_t ex = (b >> 23) & 0xffu;
    uint32_t m = b & 0x7fffffu;
    int e2 = ex == 0 ? -149 : (int)ex - 150;
    if (ex)
        m |= 0x800000u;
    elsb = e2 + __ffs((int)m) - 1;
    emsb = e2 + 31 - __clz((int)m);
}
__device__ inline void bits_f64(double v, int &elsb, int &emsb)
{
    uint64_t b = (uint64_t)__double_as_longlong(v);
    uint32_t ex = (uint32_t)((b >> 52) & 0x7ffu);
    uint64_t m = b & 0xfffffffffffffull;
    int e2 = ex == 0 ? -1074 : (int)ex - 1075;
    if (ex)
        m |= 1ull << 52;
    elsb = e2 + __ffsll((unsigned long long)m) - 1;
    emsb = e2 + 63 - __clzll((long long)m);
}

// Round hi*2^32 + lo (exact integer) times 2^-S to the nearest double, ties to even.
__device__ inline double fix128_to_double(__int128 V, int S)
{
    if (V == 0)
        return 0.0;
    bool neg = V < 0;
    unsigned __int128 M = neg ? (unsigned __int128)(-V) : (unsigned __int128)V;
    uint64_t mh = (uint64_t)(M >> 64), ml = (uint64_t)M;
    int top = mh ? 127 - __clzll((long long)mh) : 63 - __clzll((long long)ml); // index of the highest set bit
    uint64_t mant;
    int ex; // value = mant * 2^ex * 2^-S
    if (top <= 52) {
        mant = ml;
        ex = 0;
    } else {
        int drop = top - 52;
        unsigned __int128 q = M >> drop;
        mant = (uint64_t)q;
        unsigned __int128 rem = M - (q << drop);
        unsigned __int128 half = (unsigned __int128)1 << (drop - 1);
        if (rem > half || (rem == half && (mant & 1u))) {
            ++mant;
            if (mant == ((uint64_t)1 << 53)) {
                mant >>= 1;
                ++drop;
            }
        }
        ex = drop;
    }
    double r = ldexp((double)mant, ex - S); // exact: mant < 2^53, no underflow for S < 1000
    return neg ? -r : r;
}

__device__ inline double fix_to_double(int64_t hi, int64_t lo, int S)
{
    return fix128_to_double(((__int128)hi << 32) + (__int128)lo, S);
}

// ------------------------------------------------------------------------
// Wave helpers
// ------------------------------------------------------------------------
__device__ inline int lane_id() { return (int)__lane_id(); }

// A value every lane of the workgroup holds the same copy of (read from LDS
// after a barrier), made visibly uniform to the compiler.  Loops and
// branches around __syncthreads() must depend only on such values, or the
// compiler may treat them as divergent and split the barrier across lanes.
__device__ inline int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ inline uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

// Wave reductions.  Each row of 16 lanes is scanned with DPP row shifts
// (lane i combines lane i-1, i-2, i-4, i-8 of its row; lanes without a
// source keep their value), so lane 15 of every row holds the row's result;
// the four row results are then read as scalars and combined in a fixed
// order.  Plain VALU work, no LDS round trips.  The whole wave must be
// active; the result is uniform.
constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114, DPP_ROW_SHR8 = 0x118;

template <int CTRL>
__device__ inline int dpp_row(int old, int v)
{
    return __builtin_amdgcn_update_dpp(old, v, CTRL, 0xf, 0xf, false);
}
__device__ inline float rl_f(float v, int t) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), t)); }
__device__ inline int rl_i(int v, int t) { return __builtin_amdgcn_readlane(v, t); }
__device__ inline int64_t rl_i64(int64_t v, int t)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, t);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), t);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ inline double rl_d(double v, int t)
{
    return __longlong_as_double((long long)rl_i64((int64_t)__double_as_longlong(v), t));
}

template <int CTRL>
__device__ inline int dpp_row0(int v) // 0 where the row has no source lane
{
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}
template <int CTRL>
__device__ inline int64_t dpp_row_i64(int64_t v) // 0 where the row has no source lane
{
    const int lo = dpp_row0<CTRL>((int)(uint32_t)v);
    const int hi = dpp_row0<CTRL>((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ inline int64_t wave_sum_i64(int64_t v)
{
    v += dpp_row_i64<DPP_ROW_SHR1>(v);
    v += dpp_row_i64<DPP_ROW_SHR2>(v);
    v += dpp_row_i64<DPP_ROW_SHR4>(v);
    v += dpp_row_i64<DPP_ROW_SHR8>(v);
    return (rl_i64(v, 15) + rl_i64(v, 31)) + (rl_i64(v, 47) + rl_i64(v, 63));
}
__device__ inline int32_t wave_sum_i32(int32_t v)
{
    v += dpp_row0<DPP_ROW_SHR1>(v);
    v += dpp_row0<DPP_ROW_SHR2>(v);
    v += dpp_row0<DPP_ROW_SHR4>(v);
    v += dpp_row0<DPP_ROW_SHR8>(v);
    return (rl_i(v, 15) + rl_i(v, 31)) + (rl_i(v, 47) + rl_i(v, 63));
}
__device__ inline double wave_sum_f64(double v) // fixed order: deterministic
{
    auto step = [](double x, auto ctrl) {
        const int64_t b = dpp_row_i64<decltype(ctrl)::value>((int64_t)__double_as_longlong(x));
        return x + __longlong_as_double((long long)b); // +0.0 where the row has no source lane
    };
    v = step(v, std::integral_constant<int, DPP_ROW_SHR1>());
    v = step(v, std::integral_constant<int, DPP_ROW_SHR2>());
    v = step(v, std::integral_constant<int, DPP_ROW_SHR4>());
    v = step(v, std::integral_constant<int, DPP_ROW_SHR8>());
    auto rl_d = [](double x, int t) { return __longlong_as_double((long long)rl_i64((int64_t)__double_as_longlong(x), t)); };
    return (rl_d(v, 15) + rl_d(v, 31)) + (rl_d(v, 47) + rl_d(v, 63));
}
__device__ inline float wave_min_f32(float v)
{
    v = fminf(v, __int_as_float(dpp_row<DPP_ROW_SHR1>(__float_as_int(v), __float_as_int(v))));
    v = fminf(v, __int_as_float(dpp_row<DPP_ROW_SHR2>(__float_as_int(v), __float_as_int(v))));
    v = fminf(v, __int_as_float(dpp_row<DPP_ROW_SHR4>(__float_as_int(v), __float_as_int(v))));
    v = fminf(v, __int_as_float(dpp_row<DPP_ROW_SHR8>(__float_as_int(v), __float_as_int(v))));
    return fminf(fminf(rl_f(v, 15), rl_f(v, 31)), fminf(rl_f(v, 47), rl_f(v, 63)));
}

// Exact per-cluster accumulation of one wave's points.  Lanes with valid set
// contribute (count 1, fixed-point coordinates) to cluster `a`.  Lanes of
// the same cluster are summed in-wave, then one lane adds the partial sums
// to the global accumulators with integer atomics (order-independent).
//   acc: [k][D][2] int64 (hi, lo); cnt: [k] int32
template <int D>
__device__ inline void wave_accumulate(bool valid, int a, const int64_t (&hi)[D], const int64_t (&lo)[D],
                                       int64_t *acc, int32_t *cnt)
{
    uint64_t active = __ballot(valid);
    while (active) {
        int leader = __ffsll((unsigned long long)active) - 1;
        int c = rl_i(a, leader);
        bool in = valid && a == c && ((active >> lane_id()) & 1ull);
        uint64_t grp = __ballot(in);
        int32_t n = __popcll(grp);
        int64_t sh[D], sl[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            sh[i] = wave_sum_i64(in ? hi[i] : 0);
            sl[i] = wave_sum_i64(in ? lo[i] : 0);
        }
        if (lane_id() == leader) { // the sums are uniform; one lane adds them
            int64_t *ac = acc + (int64_t)c * D * 2;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                atomicAdd((unsigned long long *)&ac[2 * i], (unsigned long long)sh[i]);
                atomicAdd((unsigned long long *)&ac[2 * i + 1], (unsigned long long)sl[i]);
            }
            atomicAdd(&cnt[c], n);
        }
        active &= ~grp;
    }
}

// As wave_accumulate for at most `groups` clusters of the wave; the lanes of
// any further cluster add their own values (per-lane integer atomics, the
// same exact sums).  For points spread over many clusters the wave
// reductions would cost more than the atomics they save.
template <int D>
__device__ inline void wave_accumulate_few(bool valid, int a, const int64_t (&hi)[D], const int64_t (&lo)[D],
                                           int64_t *acc, int32_t *cnt, int groups)
{
    uint64_t active = __ballot(valid);
    for (int g = 0; active && g < groups; ++g) {
        const int leader = __ffsll((unsigned long long)active) - 1;
        const int c = rl_i(a, leader);
        const bool in = valid && a == c && ((active >> lane_id()) & 1ull);
        const uint64_t grp = __ballot(in);
        int64_t sh[D], sl[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            sh[i] = wave_sum_i64(in ? hi[i] : 0);
            sl[i] = wave_sum_i64(in ? lo[i] : 0);
        }
        if (lane_id() == leader) {
            int64_t *ac = acc + (int64_t)c * D * 2;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                atomicAdd((unsigned long long *)&ac[2 * i], (unsigned long long)sh[i]);
                atomicAdd((unsigned long long *)&ac[2 * i + 1], (unsigned long long)sl[i]);
            }
            atomicAdd(&cnt[c], (int32_t)__popcll(grp));
        }
        active &= ~grp;
    }
    if ((active >> lane_id()) & 1ull) {
        int64_t *ac = acc + (int64_t)a * D * 2;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            atomicAdd((unsigned long long *)&ac[2 * i], (unsigned long long)hi[i]);
            atomicAdd((unsigned long long *)&ac[2 * i + 1], (unsigned long long)lo[i]);
        }
        atomicAdd(&cnt[a], 1);
    }
}

// Cloud of point (or sorted position) i: the b with off[b] <= i < off[b + 1]
// (every cloud is non-empty).
__device__ inline int cloud_of(const int64_t *off, int B, int64_t i)
{
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// One wave's share of the inter-bound pair scan (see pair_plan in tree.hip).
struct alignas(16) PairItem {
    int32_t first;  // global id of the chunk's first centroid (one per lane), -1: an idle wave
    int32_t c0, c1; // the chunk's cloud: centroids [c0, c1)
    int32_t sl;     // slice t | (slices s << 8): the wave scans c0 + t, c0 + t + s, ...
};

// Implicit 8-ary centroid tree of one cloud (see tree.hip).
struct TreeArgs {
    float4 *cs;               // [k] fl32 centroids in tree order, w = global centroid id bits
    float4 *node_lo, *node_hi; // [nnodes] level 0 (buckets) first
    int nlev;                 // levels, the last one is the root
    int start;                // lowest level with at most TREE_START_MAX nodes
    int64_t nnodes;
    int64_t k;                // centroids of the cloud
    int64_t c0;               // global id of its first centroid
    int64_t lev_size[TREE_MAX_LEVELS];
    int64_t lev_off[TREE_MAX_LEVELS];
};

// ------------------------------------------------------------------------
// Context
// ------------------------------------------------------------------------
struct Scratch {
    std::vector<void *> ptrs;
    size_t bytes = 0;
};

} // namespace ekm

struct km_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    km_config cfg{};
    int64_t n = 0, k = 0;
    int d = 2;
    int f = 64;          // maximum leaf size
    int G = ekm::GROUP_LEAVES; // leaves per group (sharing one candidate list)
    // clouds: a context holds B independent point sets, cloud b owning points
    // [pt_off[b], pt_off[b+1]) and centroids [c_off[b], c_off[b+1]) of the
    // concatenated arrays; its points keep to their own centroids.  Ids are
    // global inside the context and cloud-local in assign_out.
    int B = 1;
    std::vector<int64_t> h_pt_off, h_c_off; // [B+1] on the host
    int64_t *pt_off = nullptr, *c_off = nullptr; // [B+1] on the device
    ekm::TreeArgs *trees = nullptr;  // [B] device copies of each cloud's tree arguments
    std::vector<ekm::TreeArgs> h_trees;
    ekm::Grid *grids = nullptr;      // [B] Morton grid of each cloud (its bounding box)
    std::vector<ekm::Grid> h_grids;
    int32_t *leaf_cloud = nullptr;   // [L]
    int32_t *group_cloud = nullptr;  // [ngroups]
    // inter-bound pair scan (clouds of at most TREE_SMALL_K centroids): workgroups of the tree
    // launch after its B tree workgroups, PAIR_WAVES wave items each (see pair_plan)
    int64_t npair_blocks = 0;
    ekm::PairItem *pair_items = nullptr;
    int tree_kcap = 64;              // LDS capacity of the small-k tree launch (small_tree_cap)
    int heavy_wgs = 64;              // workgroups of the per-leaf pass (heavy_blocks of the largest cloud)
    int tile = 1024;     // brute-path LDS tile (centroids)
    int S = 0;           // fixed-point scale exponent
    int fix64 = 0;       // every point's fixed-point coordinate fits FIX64_BITS bits
    ekm::Grid grid{};    // Morton grid over the data bounding box
    // A0: Morton-ordered points and leaves
    void *xs = nullptr;           // [d][n] float or double
    int32_t *perm = nullptr;      // [n] Morton position -> caller index
    int32_t *a = nullptr;         // [n] current assignment in Morton order (-1 before the first step)
    int64_t L = 0;                // number of leaves
    int32_t *leaf_start = nullptr;// [L+1]
    float *leaf_box = nullptr;    // [L][2][4] lo xyz pad, hi xyz pad
    int64_t *leaf_sum = nullptr;  // [L][d][2] exact fixed-point sums
    int32_t *leaf_own = nullptr;  // [L] cluster of every point of the leaf, OWN_MIXED or OWN_NONE
    float *leaf_r = nullptr;      // [L] bound on the exact distance from each point of the leaf to its
                                  //     centroid at the last step's positions (+inf before the first)
    int32_t *heavy = nullptr;     // [L] ids of the leaves deferred to the per-leaf pass of this step
    int32_t *heavy_cnt = nullptr; // [1] their number (reset by the finalize kernel)
    // A1: centroid tree
    float4 *c32 = nullptr;        // [k] fl32(c) in caller order
    uint32_t *ckey = nullptr, *ckey2 = nullptr;
    int32_t *cval = nullptr, *cval2 = nullptr;
    ekm::TreeArgs tree{};
    float *cerr = nullptr;        // [1] bits of an FP32 upper bound on max_j ||c_j||
    // inter bound (Eq. (3)): cb_s[j] = bits of the smallest FP32 squared distance from fl32(c_j)
    // to another fl32 centroid; cb_hi[j] >= min_{i != j} ||c_i - c_j|| (large-k path, Eq. (9))
    unsigned *cb_s = nullptr;     // [k]
    float *cb_hi = nullptr;       // [k]
    double *c_prev = nullptr;     // [k][d] centroids of the previous step (drift, Eq. (9))
    unsigned *drift_max = nullptr; // [1] bits of max_j drift (large-k path)
    float *drift = nullptr;       // [k] drift of each centroid (large-k path)
    // groups: runs of at most GROUP_LEAVES consecutive leaves inside one group cell
    int64_t ngroups = 0;
    int32_t *group_leaf = nullptr; // [ngroups+1] first leaf of each group
    int32_t *group_parts = nullptr; // [ngroups] parts the main pass splits each group into (0: whole)
    float4 *group_box = nullptr;  // [ngroups][2]
    // A5: exact sums
    int64_t *acc = nullptr;       // [k][d][2]
    int32_t *cnt = nullptr;       // [k]
    int64_t nblk_stat = 0;
    int64_t *stat_part = nullptr; // [nblk][NSTAT]
    int64_t nblk_sse = 0;
    double *sse_part = nullptr;   // [nblk_sse] objective partials of the SSE pass
    int64_t *fin_part = nullptr;  // [FIN_MAX_STAT_WG][NSTAT + 1] totals of the statistics-folding workgroups
    int32_t *fin_ticket = nullptr; // [1] folding workgroups done (0 between steps)
    int64_t *stat_out = nullptr;  // [NSTAT]
    double *sse_out = nullptr;    // [1]
    int64_t *host_stat = nullptr; // pinned [NSTAT + 1]
    // radix sort scratch
    uint32_t *rs_hist = nullptr;
    int64_t rs_hist_len = 0;
    uint32_t *scan_tmp = nullptr;
    ekm::Scratch mem;
    char *arena = nullptr; // current arena (see ctx_alloc)
    bool groups_in_arena = false; // the current arena holds the model's group part (ctx_alloc_groups)
    size_t arena_size = 0, arena_used = 0;
    int steps_done = 0;
    int32_t *ctl = nullptr;       // [CTL_N] device-side loop control
    int32_t *host_ctl = nullptr;  // pinned [(RUN_AHEAD + 1) * CTL_N]: ctl copies taken after launch groups
    hipEvent_t chunk_ev[ekm::RUN_AHEAD] = {}; // completion of those copies
    int64_t *stat_hist = nullptr; // [hist_cap][NSTAT + 1] per-step statistics of a run
    int64_t hist_cap = 0;
    // kmeans_run's centroids while it runs (the caller's array is copied in
    // and out), and its chunk of RUN_CHUNK steps on them, captured once
    double *c_run = nullptr;      // [k][d]
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t chunk_exec = nullptr;
    const double *chunk_c = nullptr;
    int chunk_failed = 0;
    int small_lists = 0;          // KM_FLAG_SMALL_LISTS: tiny candidate capacities (tests of the fallbacks)
    // KM_FLAG_TIMING: five events per recorded step (phase boundaries)
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::array<hipEvent_t, KM_NPHASE + 1>> ev_steps;
};

namespace ekm {

void set_error(const std::string &msg);
bool hip_ok(hipError_t e, const char *what);

// Device allocation tracked in the context.
// Device memory of a context: buffers are carved, ALLOC_ALIGN-aligned, from
// the current arena (one hipMalloc sized for a phase of the build) while it
// has room, else allocated on their own.  mem.bytes counts what the context
// took from the runtime.
constexpr size_t ALLOC_ALIGN = 256;
inline size_t alloc_size(size_t count, size_t elem)
{
    const size_t b = (count ? count : 1) * elem;
    return (b + ALLOC_ALIGN - 1) / ALLOC_ALIGN * ALLOC_ALIGN;
}

template <class T>
T *ctx_alloc(km_ctx *ctx, size_t count)
{
    const size_t bytes = alloc_size(count, sizeof(T));
    if (ctx->arena && ctx->arena_used + bytes <= ctx->arena_size) {
        void *p = ctx->arena + ctx->arena_used;
        ctx->arena_used += bytes;
        return (T *)p;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess)
        return nullptr;
    ctx->mem.ptrs.push_back(p);
    ctx->mem.bytes += bytes;
    return (T *)p;
}

// A buffer of the workspace model's group part (leaf groups, statistics
// rows): from the arena when the arena was sized with that part, else an
// allocation of its own, so that it never takes the arena space of a later
// buffer of the other parts.
template <class T>
T *ctx_alloc_groups(km_ctx *ctx, size_t count)
{
    if (ctx->groups_in_arena)
        return ctx_alloc<T>(ctx, count);
    char *a = ctx->arena;
    ctx->arena = nullptr;
    T *p = ctx_alloc<T>(ctx, count);
    ctx->arena = a;
    return p;
}

// Starts a new arena of `bytes` (the rest of the previous one is unused).
inline bool ctx_arena(km_ctx *ctx, size_t bytes)
{
    void *p = nullptr;
    if (bytes == 0 || hipMalloc(&p, bytes) != hipSuccess)
        return false;
    ctx->mem.ptrs.push_back(p);
    ctx->mem.bytes += bytes;
    ctx->arena = (char *)p;
    ctx->arena_size = bytes;
    ctx->arena_used = 0;
    return true;
}

// Bytes of the buffers the build allocates once the leaf count L (and, with
// `with_groups`, the group count) is known (api.hip, from the workspace model).
size_t ctx_bytes_after_counts(const km_ctx *ctx, int64_t L, int64_t groups, bool with_groups);

// sort.hip
size_t radix_scratch_words(int64_t n);
hipError_t radix_sort_u32(uint32_t *keys, int32_t *vals, uint32_t *keys_tmp, int32_t *vals_tmp, int64_t n,
                          int bits, uint32_t *hist, uint32_t *scan_tmp, hipStream_t s, bool *result_in_tmp);
hipError_t exclusive_scan_u32(uint32_t *data, int64_t n, uint32_t *tmp, hipStream_t s);
size_t scan_scratch_words(int64_t n);

// leaves.hip
size_t scan_record_bytes(); // input-scan record per cloud (leaves.hip)
km_status build_leaves(km_ctx *ctx, const void *points);

// tree.hip
km_status build_centroid_tree(km_ctx *ctx, const double *c_in, bool resort);
constexpr int TREE_RESORT = 8; // the centroid trees re-sort their centroids every this many steps
bool small_trees(const km_ctx *ctx);
constexpr int TREE_SMALL_K = 4096; // largest cloud whose tree one workgroup builds in LDS
constexpr int PAIR_WAVES = 16;     // waves per pair-scan workgroup (the tree workgroup's size)
int64_t pair_plan(const int64_t *c_off, int B, std::vector<PairItem> *items);
int small_tree_cap(const int64_t *c_off, int B);
hipError_t tree_setup();
void tree_layout(int64_t k, TreeArgs &T);

// assign.hip
km_status run_assign(km_ctx *ctx, const double *c_in, hipEvent_t between);
km_status run_sse(km_ctx *ctx, const double *c_in);
int64_t sse_blocks(int64_t n);

// reduce.hip
km_status run_finalize(km_ctx *ctx, const double *c_in, double *c_out, int32_t *assign_out, bool with_sse);
km_status set_ctl(km_ctx *ctx, int32_t max_iter, int32_t stable, int32_t reset_run);
km_status scatter_assignment(km_ctx *ctx, int32_t *assign_out);

} // namespace ekm
