// Assignment step (Algorithm 1's Assign over the point index, with its kNN
// search over the centroid index), fused with the accumulation half of the
// centroid update.
//
// k_assign_waves: one wave per group of GROUP_LEAVES consecutive leaves;
// see the comment at the kernel.  U, the smallest FP32 max-distance from a
// box to a node or centroid seen so far, bounds the distance from every
// point of the box to some centroid (the paper inherits such bounds from
// parent nodes, Eq. (7)); nodes and centroids whose FP32 min-distance to the
// box exceeds prune_threshold(U) are dropped.
//
// k_assign_brute32 / k_assign_brute64: Lloyd's assignment over all k
// centroids staged through LDS tiles (the GPU baseline; FP64 is the plain
// canonical computation).
#include "ekm_internal.hpp"

namespace ekm {

constexpr int ASSIGN_THREADS = 256;
constexpr int G_WAVES = ASSIGN_THREADS / WAVE; // independent waves per workgroup
// Per-wave LDS capacities: candidate list entries and descent entries per
// level.  A leaf whose list does not fit in the main pass goes to the
// per-leaf pass, whose waves have room for crowded leaves (one workgroup
// per CU there).
constexpr int SW_MAIN = 256, FR_MAIN = 1024;
constexpr int SW_HEAVY = 1024, FR_HEAVY = 4096;
static_assert(GROUP_LEAVES <= WAVE, "one lane holds one leaf of the group");
static_assert(TREE_START_MAX <= FR_MAIN && TREE_START_MAX <= FR_HEAVY, "the first descent level fits");
static_assert(MAX_LEAF <= WAVE, "one lane holds one point of a leaf");

struct AssignArgs {
    const void *xs;     // [d][n] Morton order
    int64_t n, k;
    int32_t *a;         // [n]
    const double *c_in; // [k][d]
    const float4 *c32;  // [k]
    const unsigned *cmax_bits;
    // leaves and groups
    const int32_t *leaf_start;
    int64_t L;
    const float4 *leaf_box;
    const int64_t *leaf_sum;
    int32_t *leaf_prev;
    int32_t *heavy;
    int32_t *heavy_cnt;
    const int32_t *group_leaf;
    const float4 *group_box;
    int64_t ngroups;
    // centroid tree
    TreeArgs T;
    // update
    int S;
    int fix64;
    int64_t *acc;
    int32_t *cnt;
    int64_t *stat_part;
    double *sse_part;
    int want_sse;
    int tile;
};

__device__ inline float err_bound(const unsigned *cmax_bits)
{
    // ||c - fl32(c)|| <= 2^-24 ||c|| (plus an absolute term for FP32 underflow)
    return __uint_as_float(*cmax_bits) * 0x1p-24f * (1.0f + 0x1p-20f) + 0x1p-100f;
}

__device__ inline void f4_to(const float4 v, float *o)
{
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
}

struct BlockStats {
    long long v[NSTAT];
    double sse[G_WAVES];
};

// Per-wave LDS of the indexed kernel.  Only lanes of the owning wave touch
// it; writes by some lanes are read by others only after wave_sync().
template <int SW, int FR>
struct WaveSharedT {
    static constexpr int sw = SW, fr = FR, npar = FR / TREE_BUCKET;
    float4 sc[SW];        // candidate list of the current box: fl32 coordinates, w = centroid id
    int par[2][npar];     // kept nodes of the previous descent level
    float fm[FR];         // min-distances of the current level's entries (lane-private slots)
};
using WaveMain = WaveSharedT<SW_MAIN, FR_MAIN>;
using WaveHeavy = WaveSharedT<SW_HEAVY, FR_HEAVY>;

// Orders this wave's LDS writes before its later LDS reads by other lanes
// (the LDS executes one wave's operations in issue order; the fences keep
// the compiler from moving accesses across).
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


__device__ inline void stats_begin(BlockStats &bs)
{
    if (threadIdx.x < NSTAT)
        bs.v[threadIdx.x] = 0;
    if (threadIdx.x < G_WAVES)
        bs.sse[threadIdx.x] = 0.0;
    __syncthreads();
}

// per-thread counters -> partial row `row` (fixed-order FP64 for the SSE)
__device__ inline void stats_end(BlockStats &bs, const AssignArgs &A, const int64_t (&c)[NSTAT], double sse,
                                 int64_t row)
{
#pragma unroll
    for (int q = 0; q < NSTAT; ++q) {
        int64_t w = wave_sum_i64(c[q]);
        if (lane_id() == 0 && w)
            atomicAdd((unsigned long long *)&bs.v[q], (unsigned long long)w);
    }
    double ws = wave_sum_f64(sse);
    if (lane_id() == 0)
        bs.sse[threadIdx.x / WAVE] = ws;
    __syncthreads();
    if (threadIdx.x < NSTAT)
        A.stat_part[row * NSTAT + threadIdx.x] = bs.v[threadIdx.x];
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < G_WAVES; ++w)
            s += bs.sse[w];
        A.sse_part[row] = s;
    }
}

// Statistics of one workgroup of independent waves: each wave adds its
// (wave-uniform) counters to LDS with atomics and parks its SSE in its own
// slot; the wave that arrives last writes the workgroup's row, summing the
// SSE slots in wave order (deterministic).  Initialised before any wave
// diverges (the kernel's single workgroup barrier).
struct BlockCombine {
    unsigned long long v[NSTAT];
    double sse[G_WAVES];
    int done;
};

__device__ inline void combine_init(BlockCombine &bc)
{
    if (threadIdx.x < NSTAT)
        bc.v[threadIdx.x] = 0;
    if (threadIdx.x < G_WAVES)
        bc.sse[threadIdx.x] = 0.0;
    if (threadIdx.x == 0)
        bc.done = 0;
    __syncthreads();
}

__device__ inline void combine_end(BlockCombine &bc, const AssignArgs &A, const int64_t (&c)[NSTAT], double sse,
                                   int64_t row)
{
    const int lane = lane_id();
    int64_t mine = 0;
#pragma unroll
    for (int q = 0; q < NSTAT; ++q)
        if (lane == q)
            mine = c[q];
    const double ws = A.want_sse ? wave_sum_f64(sse) : 0.0;
    if (lane < NSTAT && mine)
        __hip_atomic_fetch_add(&bc.v[lane], (unsigned long long)mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (lane == 0)
        bc.sse[threadIdx.x / WAVE] = ws;
    int last = 0;
    if (lane == 0)
        last = __hip_atomic_fetch_add(&bc.done, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) == G_WAVES - 1;
    if (!rl_i(last, 0))
        return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (lane < NSTAT)
        A.stat_part[row * NSTAT + lane] =
            (int64_t)__hip_atomic_load(&bc.v[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (lane == 0) {
        double s = 0.0;
        for (int w = 0; w < G_WAVES; ++w)
            s += bc.sse[w];
        A.sse_part[row] = s;
    }
}

// Number of lanes of the wave with `p` set (wave-uniform).
__device__ inline int wave_count(bool p) { return __popcll(__ballot(p)); }

// ------------------------------------------------------------- tree search
// Fills sh.sc with the candidate list of box [lo, hi] and returns its
// length, or -1 if a descent level or the list does not fit.  The whole
// wave calls; the result is uniform.
//
// The descent starts at the lowest tree level with at most TREE_START_MAX
// nodes and evaluates every node there; each later level evaluates the
// children of the nodes kept at the level above (at most FR_CAP entries),
// and the last step the centroids of the kept buckets.  U is the smallest
// box-to-node max-distance seen at any level (a valid bound: every node
// holds a centroid).  Each lane keeps the min-distances of its entries in
// its own LDS slots between the two passes of a level.
template <int D, class WS>
__device__ int wave_search(const float *lo, const float *hi, const AssignArgs &A, float e, WS &sh)
{
    const TreeArgs &T = A.T;
    const int lane = lane_id();
    const uint64_t lt = lanemask_lt();
    wave_sync(); // earlier readers of sh are done
    int level = T.start;
    int np = -1; // kept parents at the level above (-1: the start level is evaluated densely)
    int cur = 0;
    float U = INFINITY;
    while (true) {
        const int64_t off = T.lev_off[level], lsz = T.lev_size[level];
        const int F = np < 0 ? (int)lsz : np * TREE_BUCKET;
        float Ul = INFINITY;
#pragma unroll 4
        for (int i = lane; i < F; i += WAVE) {
            const int64_t node = np < 0 ? i : (int64_t)sh.par[cur][i / TREE_BUCKET] * TREE_BUCKET + i % TREE_BUCKET;
            float m = INFINITY;
            if (node < lsz) {
                float nl[3], nh[3];
                f4_to(T.node_lo[off + node], nl);
                f4_to(T.node_hi[off + node], nh);
                m = bb_mind<D>(lo, hi, nl, nh);
                Ul = fminf(Ul, bb_maxd<D>(lo, hi, nl, nh));
            }
            sh.fm[i] = m; // read back by this lane only
        }
        U = fminf(U, wave_min_f32(Ul));
        const float thr = prune_threshold(U, e);
        const int nxt = cur ^ 1;
        int cnt = 0;
        for (int i0 = 0; i0 < F; i0 += WAVE) {
            const int i = i0 + lane;
            const bool keep = i < F && sh.fm[i] <= thr;
            const uint64_t mk = __ballot(keep);
            const int pos = cnt + __popcll(mk & lt);
            if (keep && pos < WS::npar)
                sh.par[nxt][pos] =
                    np < 0 ? i : sh.par[cur][i / TREE_BUCKET] * TREE_BUCKET + i % TREE_BUCKET;
            cnt += __popcll(mk);
        }
        if (cnt > WS::npar)
            return -1;
        wave_sync();
        np = cnt;
        cur = nxt;
        if (level == 0)
            break;
        --level;
    }
    // centroids of the kept buckets
    const int F = np * TREE_BUCKET;
    float Ul = INFINITY;
#pragma unroll 4
    for (int i = lane; i < F; i += WAVE) {
        const int64_t t = (int64_t)sh.par[cur][i / TREE_BUCKET] * TREE_BUCKET + i % TREE_BUCKET;
        float m = INFINITY;
        if (t < A.k) {
            float cc[3];
            f4_to(T.cs[t], cc);
            m = box_mind<D>(lo, hi, cc);
            Ul = fminf(Ul, box_maxd<D>(lo, hi, cc));
        }
        sh.fm[i] = m;
    }
    U = fminf(U, wave_min_f32(Ul));
    const float thr = prune_threshold(U, e);
    int cnt = 0;
    for (int i0 = 0; i0 < F; i0 += WAVE) {
        const int i = i0 + lane;
        const bool keep = i < F && sh.fm[i] <= thr;
        const uint64_t mk = __ballot(keep);
        const int pos = cnt + __popcll(mk & lt);
        if (keep && pos < WS::sw) // the entry was loaded by this lane a moment ago (cache hit)
            sh.sc[pos] = T.cs[(int64_t)sh.par[cur][i / TREE_BUCKET] * TREE_BUCKET + i % TREE_BUCKET];
        cnt += __popcll(mk);
    }
    wave_sync();
    return cnt > WS::sw ? -1 : cnt;
}

// --------------------------------------------------------------- epilogue
// Record the new assignment, count changes, add each point to its cluster's
// exact fixed-point sum.
template <int D, class TV>
__device__ inline void finish_point(const AssignArgs &A, bool valid, int64_t p, const TV (&x)[D], int best,
                                    int64_t &changed, double &sse)
{
    if (valid) {
        int old = A.a[p];
        if (old != best) {
            A.a[p] = best;
            ++changed;
        }
        if (A.want_sse) {
            double xd[D], cd[D];
            for (int i = 0; i < D; ++i) {
                xd[i] = (double)x[i];
                cd[i] = A.c_in[(int64_t)best * D + i];
            }
            sse += sqdist64<D>(xd, cd);
        }
    }
    int64_t hi[D], lo[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        if (sizeof(TV) == 4)
            fix_split_f32((float)x[i], A.S, hi[i], lo[i]);
        else
            fix_split_f64((double)x[i], A.S, hi[i], lo[i]);
    }
    wave_accumulate<D>(valid, best, hi, lo, A.acc, A.cnt);
}

template <int D>
__device__ inline int brute64_all(const double (&xd)[D], const AssignArgs &A)
{
    double best = INFINITY;
    int bj = 0;
    for (int64_t j = 0; j < A.k; ++j) {
        double Dv = sqdist64<D>(xd, A.c_in + j * D);
        if (Dv < best) {
            best = Dv;
            bj = (int)j;
        }
    }
    return bj;
}

// Exact accumulation of one leaf's points (lane = point, `valid` lanes are
// the whole leaf) into their clusters.  The clusters present are taken one
// at a time; a cluster's coordinate sums are wave sums of the points'
// fixed-point values (one int64 per coordinate when every value fits
// FIX64_BITS bits, else the hi/lo parts), its count a ballot popcount.  The
// last cluster gets the leaf's precomputed exact sum minus what the others
// took.  The values are then split into the (hi, lo) accumulator form and
// lanes 0..2D-1 (sums) and 2D (count) add them with integer atomics.  A
// leaf spread over many clusters (crowded centroids) stops reducing after
// ACC_ROUNDS clusters; its remaining points add their own values.
constexpr int ACC_ROUNDS = 3;
template <int D>
__device__ inline void accumulate_leaf(bool valid, int a, const float (&x)[D], const int64_t *lsum,
                                       const AssignArgs &A)
{
    const int lane = lane_id();
    int64_t v0[D], v1[D]; // fix64: value, 0; else hi, lo
#pragma unroll
    for (int i = 0; i < D; ++i) {
        if (A.fix64) {
            v0[i] = valid ? fix_f32(x[i], A.S) : 0;
            v1[i] = 0;
        } else {
            fix_split_f32(x[i], A.S, v0[i], v1[i]);
            if (!valid)
                v0[i] = v1[i] = 0;
        }
    }
    int64_t took_hi[D], took_lo[D];
#pragma unroll
    for (int i = 0; i < D; ++i)
        took_hi[i] = took_lo[i] = 0;
    uint64_t active = __ballot(valid);
    for (int round = 0; active; ++round) {
        if (round == ACC_ROUNDS) {
            if ((active >> lane) & 1ull) {
                int64_t *ac = A.acc + (int64_t)a * D * 2;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    int64_t h = v0[i], l = v1[i];
                    if (A.fix64) {
                        h = v0[i] >> 32;
                        l = v0[i] - (h << 32);
                    }
                    atomicAdd((unsigned long long *)&ac[2 * i], (unsigned long long)h);
                    atomicAdd((unsigned long long *)&ac[2 * i + 1], (unsigned long long)l);
                }
                atomicAdd(&A.cnt[a], 1);
            }
            break;
        }
        const int c = rl_i(a, __ffsll((unsigned long long)active) - 1);
        const bool in = valid && a == c;
        const uint64_t grp = __ballot(in);
        active &= ~grp;
        int64_t sh[D], sl[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            if (active == 0) {
                sh[i] = lsum[2 * i] - took_hi[i];
                sl[i] = lsum[2 * i + 1] - took_lo[i];
            } else if (A.fix64) {
                const int64_t t = wave_sum_i64(in ? v0[i] : 0);
                sh[i] = t >> 32; // floor, so that sl is in [0, 2^32)
                sl[i] = t - (sh[i] << 32);
            } else {
                sh[i] = wave_sum_i64(in ? v0[i] : 0);
                sl[i] = wave_sum_i64(in ? v1[i] : 0);
            }
            took_hi[i] += sh[i];
            took_lo[i] += sl[i];
        }
        int64_t mine = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            if (lane == 2 * i)
                mine = sh[i];
            if (lane == 2 * i + 1)
                mine = sl[i];
        }
        if (lane < 2 * D)
            atomicAdd((unsigned long long *)&A.acc[(int64_t)c * D * 2 + lane], (unsigned long long)mine);
        else if (lane == 2 * D)
            atomicAdd(&A.cnt[c], __popcll(grp));
    }
}

// ------------------------------------------------------------- leaves
// The wave's list is read in chunks of 64 entries, lane j holding entry
// 64c + j in registers; a candidate is then broadcast to all lanes with
// readlane (scalar operands, no LDS round trip per candidate).
template <class WS>
__device__ inline float4 list_entry(const WS &sh, int j, int sn)
{
    return j < sn ? sh.sc[j] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Candidate filter of one leaf box against the wave's list (sn entries):
// returns the candidate count m, the id of the first candidate (the only
// one when m == 1) and the threshold for the later mask passes.
template <int D, class WS>
__device__ inline int leaf_filter(const float *blo, const float *bhi, int sn, float e, const WS &sh,
                                  float &thr, int &j1)
{
    const int lane = lane_id();
    const int nch = (sn + WAVE - 1) / WAVE;
    float U = INFINITY;
    for (int c = 0; c < nch; ++c) {
        const int j = c * WAVE + lane;
        const float4 c4 = list_entry(sh, j, sn);
        float cc[3];
        f4_to(c4, cc);
        if (j < sn)
            U = fminf(U, box_maxd<D>(blo, bhi, cc));
    }
    thr = prune_threshold(wave_min_f32(U), e);
    int m = 0;
    j1 = -1;
    for (int c = 0; c < nch; ++c) {
        const int j = c * WAVE + lane;
        const float4 c4 = list_entry(sh, j, sn);
        float cc[3];
        f4_to(c4, cc);
        const bool keep = j < sn && box_mind<D>(blo, bhi, cc) <= thr;
        const uint64_t mk = __ballot(keep);
        if (mk && j1 < 0)
            j1 = rl_i(__float_as_int(c4.w), __ffsll((unsigned long long)mk) - 1);
        m += __popcll(mk);
    }
    return m;
}

// Running (best, second-best, best id) of an FP32 scan.  The best is kept
// as one 64-bit key (value bits << 32 | id): squared distances are >= 0, so
// their bit patterns order like the values, and one unsigned compare gives
// the (value, id) order with the lowest id first among equal values.
struct Best2 {
    uint64_t key;
    float s2;
};
__device__ inline Best2 best2_init() { return Best2{~0ull, INFINITY}; }
__device__ inline float best2_s1(const Best2 &b) { return __uint_as_float((uint32_t)(b.key >> 32)); }
__device__ inline int best2_id(const Best2 &b) { return (int)(uint32_t)b.key; }
__device__ inline void best2_add(Best2 &b, float sv, int cid)
{
    const uint64_t k = ((uint64_t)__float_as_uint(sv) << 32) | (uint32_t)cid;
    const bool better = k < b.key;
    b.s2 = fminf(b.s2, better ? best2_s1(b) : sv); // the loser of the two
    b.key = better ? k : b.key;
}
// Merge of two scans over disjoint candidate sets.
__device__ inline Best2 best2_merge(const Best2 &a, const Best2 &b)
{
    const bool af = a.key < b.key;
    Best2 r;
    r.key = af ? a.key : b.key;
    r.s2 = fminf(best2_s1(af ? b : a), fminf(a.s2, b.s2));
    return r;
}
constexpr int SCAN_ILP = 4; // independent scans interleaved over the candidates

// FP32 scan of one point (one lane) against the leaf's candidates: the list
// entries within `thr` of the leaf box, in chunks, each candidate broadcast
// from the lane that holds it.  Lanes whose best-vs-second margin is below
// the error bound are decided again with canonical FP64 distances over the
// candidates that can still be nearest: those whose FP32 lower bound does
// not exceed the best one's upper bound (any other is strictly farther in
// exact and in FP64 arithmetic).  Returns the centroid id.
template <int D, class WS>
__device__ inline int assign_point(const float (&x)[D], bool valid, const float *blo, const float *bhi, float thr,
                                   int sn, float e, const AssignArgs &A, const WS &sh,
                                   int64_t (&st)[NSTAT])
{
    const int lane = lane_id();
    const int nch = (sn + WAVE - 1) / WAVE;
    Best2 bs[SCAN_ILP];
#pragma unroll
    for (int u = 0; u < SCAN_ILP; ++u)
        bs[u] = best2_init();
    for (int c = 0; c < nch; ++c) {
        const int jl = c * WAVE + lane;
        const float4 c4 = list_entry(sh, jl, sn);
        float cl[3];
        f4_to(c4, cl);
        uint64_t mk = __ballot(jl < sn && box_mind<D>(blo, bhi, cl) <= thr);
        while (mk) {
            // up to SCAN_ILP candidates per round, one per independent scan
#pragma unroll
            for (int u = 0; u < SCAN_ILP; ++u) {
                if (mk) {
                    const int b = __ffsll((unsigned long long)mk) - 1;
                    mk &= mk - 1;
                    float cc[3] = {rl_f(c4.x, b), rl_f(c4.y, b), D == 3 ? rl_f(c4.z, b) : 0.0f};
                    best2_add(bs[u], sqdist32<D>(x, cc), rl_i(__float_as_int(c4.w), b));
                }
            }
        }
    }
#pragma unroll
    for (int u = 1; u < SCAN_ILP; ++u)
        bs[0] = best2_merge(bs[0], bs[u]);
    const float s1 = best2_s1(bs[0]), s2 = bs[0].s2;
    const int id1 = best2_id(bs[0]);
    const bool re = valid && !margin_safe(s1, s2, e);
    const int nre = wave_count(re);
    if (nre == 0)
        return id1;
    st[ST_RECHECK] += nre;
    double xd[D];
    for (int i = 0; i < D; ++i)
        xd[i] = (double)x[i];
    const float s_cap = lo_inverse(dist_hi(s1, e), e); // dist_lo(s) <= dist_hi(s1) implies s <= s_cap
    double bd = INFINITY;
    int bj = 0x7fffffff;
    for (int c = 0; c < nch; ++c) {
        const int jl = c * WAVE + lane;
        const float4 c4 = list_entry(sh, jl, sn);
        float cl[3];
        f4_to(c4, cl);
        const bool kc = jl < sn && box_mind<D>(blo, bhi, cl) <= thr;
        double cdl[3] = {0.0, 0.0, 0.0}; // this lane's FP64 centroid, broadcast below
        if (kc)
            for (int i = 0; i < D; ++i)
                cdl[i] = A.c_in[(int64_t)__float_as_int(c4.w) * D + i];
        uint64_t mk = __ballot(kc);
        while (mk) {
            const int b = __ffsll((unsigned long long)mk) - 1;
            mk &= mk - 1;
            float cc[3] = {rl_f(c4.x, b), rl_f(c4.y, b), D == 3 ? rl_f(c4.z, b) : 0.0f};
            const int cid = rl_i(__float_as_int(c4.w), b);
            double cd[D];
            for (int i = 0; i < D; ++i)
                cd[i] = rl_d(cdl[i], b);
            if (re && sqdist32<D>(x, cc) <= s_cap) {
                const double Dv = sqdist64<D>(xd, cd);
                if (Dv < bd || (Dv == bd && cid < bj)) {
                    bd = Dv;
                    bj = cid;
                }
            }
        }
    }
    return re ? bj : id1;
}

// Epilogue of a leaf assigned point by point: record changed assignments
// (aold: the previous assignments, loaded by the caller), SSE terms, exact
// cluster sums.
template <int D>
__device__ inline void leaf_finish(const AssignArgs &A, int64_t l, bool valid, int64_t p, const float (&x)[D],
                                   int best, int aold, int64_t (&st)[NSTAT], double &sse)
{
    const bool ch = valid && aold != best;
    if (ch)
        A.a[p] = best;
    st[ST_CHANGED] += wave_count(ch);
    if (A.want_sse && valid) {
        double xd[D], cd[D];
        for (int i = 0; i < D; ++i) {
            xd[i] = (double)x[i];
            cd[i] = A.c_in[(int64_t)best * D + i];
        }
        sse += sqdist64<D>(xd, cd);
    }
    accumulate_leaf<D>(valid, best, x, A.leaf_sum + l * D * 2, A);
}

// Fallback for a leaf whose candidate list does not fit: scan all k
// centroids in FP32 (fl32 copies from global memory), same margin rule.
template <int D>
__device__ void process_leaf_all(int64_t l, int s, int size, int prev, const AssignArgs &A, float e,
                                 int64_t (&st)[NSTAT], double &sse)
{
    const int lane = lane_id();
    const float *xs = (const float *)A.xs;
    const bool valid = lane < size;
    const int64_t p = (int64_t)s + lane;
    if (lane == 0 && prev != -1)
        A.leaf_prev[l] = -1;
    float x[D];
    for (int i = 0; i < D; ++i)
        x[i] = valid ? xs[(int64_t)i * A.n + p] : 0.0f;
    // all k centroids, 64 at a time in registers (the next chunk loading
    // while this one is scanned), ascending j: strict < keeps the lowest index
    Best2 bs[SCAN_ILP];
#pragma unroll
    for (int u = 0; u < SCAN_ILP; ++u)
        bs[u] = best2_init();
    float4 cur = lane < A.k ? A.c32[lane] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int64_t j0 = 0; j0 < A.k; j0 += WAVE) {
        const int64_t jn = j0 + WAVE + lane;
        const float4 nxt = jn < A.k ? A.c32[jn] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const int cn = (int)(A.k - j0 < WAVE ? A.k - j0 : WAVE);
        for (int b0 = 0; b0 < cn; b0 += SCAN_ILP) {
#pragma unroll
            for (int u = 0; u < SCAN_ILP; ++u) {
                const int b = b0 + u;
                if (b < cn) {
                    float cc[3] = {rl_f(cur.x, b), rl_f(cur.y, b), D == 3 ? rl_f(cur.z, b) : 0.0f};
                    best2_add(bs[u], sqdist32<D>(x, cc), (int)(j0 + b));
                }
            }
        }
        cur = nxt;
    }
#pragma unroll
    for (int u = 1; u < SCAN_ILP; ++u)
        bs[0] = best2_merge(bs[0], bs[u]);
    const float s1 = best2_s1(bs[0]), s2 = bs[0].s2;
    int best = best2_id(bs[0]);
    const bool re = valid && !margin_safe(s1, s2, e);
    if (re) {
        double xd[D];
        for (int i = 0; i < D; ++i)
            xd[i] = (double)x[i];
        best = brute64_all<D>(xd, A);
    }
    const int nv = wave_count(valid);
    st[ST_RECHECK] += wave_count(re);
    st[ST_EVALS] += (int64_t)nv * A.k;
    st[ST_FALLBACK_PTS] += nv;
    leaf_finish<D>(A, l, valid, p, x, best, valid ? A.a[p] : -1, st, sse);
}

// Per-leaf data held by lane t of the wave for leaf l0 + t of its group.
struct LeafRegs {
    float lo[3], hi[3];
    int start, size, prev;
};

template <int D>
__device__ inline void leaf_of(const LeafRegs &r, int t, float *blo, float *bhi)
{
#pragma unroll
    for (int i = 0; i < D; ++i) {
        blo[i] = rl_f(r.lo[i], t);
        bhi[i] = rl_f(r.hi[i], t);
    }
}

// One leaf against the wave's list (the per-leaf path: no prefetch).
template <int D, class WS>
__device__ void process_leaf(int64_t l, int s, int size, int prev, const float *blo, const float *bhi, int sn,
                             const AssignArgs &A, float e, const WS &sh, int64_t (&st)[NSTAT], double &sse)
{
    const int lane = lane_id();
    const float *xs = (const float *)A.xs;
    float thr;
    int j1;
    const int m = leaf_filter<D>(blo, bhi, sn, e, sh, thr, j1);
    if (m == 0) {
        process_leaf_all<D>(l, s, size, prev, A, e, st, sse);
        return;
    }
    const bool valid = lane < size;
    const int64_t p = (int64_t)s + lane;
    st[ST_CANDS] += m;
    st[ST_EVALS] += (int64_t)m * size;
    if (lane == 0 && prev != -1)
        A.leaf_prev[l] = -1;
    float x[D];
    for (int i = 0; i < D; ++i)
        x[i] = valid ? xs[(int64_t)i * A.n + p] : 0.0f;
    const int aold = valid ? A.a[p] : -1;
    const int best = assign_point<D>(x, valid, blo, bhi, thr, sn, e, A, sh, st);
    leaf_finish<D>(A, l, valid, p, x, best, aold, st, sse);
}

// Points and previous assignments of leaf t, as far as its filter result
// needs them (a single-candidate leaf that keeps its cluster needs neither).
template <int D>
__device__ inline void load_leaf(const LeafRegs &r, int t, int m, int j1, const AssignArgs &A, float (&xv)[D],
                                 int &av)
{
    const int lane = lane_id();
    const float *xs = (const float *)A.xs;
    const int s = rl_i(r.start, t), size = rl_i(r.size, t), prev = rl_i(r.prev, t);
    const int64_t p = (int64_t)s + lane;
    const bool valid = lane < size;
    const bool need_x = m <= HEAVY_M && (m != 1 || A.want_sse);
    const bool need_a = m <= HEAVY_M && (m != 1 || prev != j1);
    av = -1;
    for (int i = 0; i < D; ++i)
        xv[i] = 0.0f;
    if (valid && need_x)
        for (int i = 0; i < D; ++i)
            xv[i] = xs[(int64_t)i * A.n + p];
    if (valid && need_a)
        av = A.a[p];
}

// k_assign_waves: one wave per group (at most GROUP_LEAVES consecutive
// leaves inside one compact Morton cell, see leaves.hip); the waves of a
// workgroup are independent and the kernel has no workgroup barrier.
//
//  1. Group search: the centroid-tree descent for the group's bounding box
//     gives the group list S (kNN-style pruning with the upper bound U, the
//     node pruning of Eq. (8), made conservative for rounding).
//  2. Leaf filter: for a leaf box b inside the group box, the same rule
//     applied to S alone gives exactly the leaf's candidates over all k
//     centroids: a centroid outside S has min-distance to b at least its
//     min-distance to the group box, above prune_threshold(U_group) >=
//     prune_threshold(U_b), and the centroid that realised U_group is in S.
//     Lanes test S in chunks of 64; ballots give the candidate set.
//  3. A leaf with one candidate is assigned to it without any distance
//     evaluation (Eq. (6)'s batch assignment) and adds its precomputed exact
//     sum to that cluster.  Otherwise each lane (one point) scans the
//     candidates in FP32; a point whose best-vs-second margin is below the
//     error bound is decided again with canonical FP64 distances.
//
// If S does not fit, the wave searches leaf by leaf, and a leaf whose own
// list does not fit scans all k centroids; results are the same.
template <int D>
__device__ void group_work(int64_t g, const AssignArgs &A, WaveMain &sh, int64_t (&st)[NSTAT], double &sse);

template <int D>
__global__ void __launch_bounds__(ASSIGN_THREADS) k_assign_waves(AssignArgs A)
{
    __shared__ WaveMain wsh[G_WAVES];
    __shared__ BlockCombine bc;
    combine_init(bc);
    const int64_t g = (int64_t)blockIdx.x * G_WAVES + threadIdx.x / WAVE;
    int64_t st[NSTAT] = {0, 0, 0, 0, 0, 0, 0, 0};
    double sse = 0.0;
    if (g < A.ngroups) // whole wave; nothing in group_work synchronises across waves
        group_work<D>(g, A, wsh[threadIdx.x / WAVE], st, sse);
    combine_end(bc, A, st, sse, blockIdx.x);
}

template <int D>
__device__ void group_work(int64_t g, const AssignArgs &A, WaveMain &sh, int64_t (&st)[NSTAT], double &sse)
{
    const int lane = lane_id();
    const float e = err_bound(A.cmax_bits);
    const int64_t l0 = A.group_leaf[g];
    const int nl = A.group_leaf[g + 1] - (int)l0; // 1..GROUP_LEAVES
    LeafRegs r;
    for (int i = 0; i < 3; ++i)
        r.lo[i] = r.hi[i] = 0.0f;
    r.start = r.size = 0;
    r.prev = -1;
    if (lane < nl) {
        const float4 bl = A.leaf_box[2 * (l0 + lane)], bh = A.leaf_box[2 * (l0 + lane) + 1];
        f4_to(bl, r.lo);
        f4_to(bh, r.hi);
        r.start = A.leaf_start[l0 + lane];
        r.size = A.leaf_start[l0 + lane + 1] - r.start;
        r.prev = A.leaf_prev[l0 + lane];
    }
    float glo[3], ghi[3];
    f4_to(A.group_box[2 * g], glo);
    f4_to(A.group_box[2 * g + 1], ghi);
    const int sn = wave_search<D>(glo, ghi, A, e, sh);
    if (sn < 0) {
        // the group's list does not fit: search leaf by leaf
        for (int t = 0; t < nl; ++t) {
            float blo[3], bhi[3];
            leaf_of<D>(r, t, blo, bhi);
            const int ln = wave_search<D>(blo, bhi, A, e, sh);
            if (ln >= 0) {
                process_leaf<D>(l0 + t, rl_i(r.start, t), rl_i(r.size, t), rl_i(r.prev, t), blo, bhi, ln, A, e, sh,
                                st, sse);
            } else if (lane == 0) { // the per-leaf pass has room for it
                A.heavy[l0 + t] = 1;
                atomicAdd(A.heavy_cnt, 1);
            }
        }
        return;
    }
    // filter every leaf first; lane t keeps leaf t's results
    float r_thr = 0.0f;
    int r_m = 0, r_j = -1;
    for (int t = 0; t < nl; ++t) {
        float blo[3], bhi[3];
        leaf_of<D>(r, t, blo, bhi);
        float thr;
        int j1;
        const int m = leaf_filter<D>(blo, bhi, sn, e, sh, thr, j1);
        if (m != 1)
            j1 = -1;
        if (lane == t) {
            r_thr = thr;
            r_m = m;
            r_j = j1;
        }
    }
    float xn[D];
    int an;
    load_leaf<D>(r, 0, rl_i(r_m, 0), rl_i(r_j, 0), A, xn, an);
    for (int t = 0; t < nl; ++t) {
        float x[D];
        for (int i = 0; i < D; ++i)
            x[i] = xn[i];
        const int aold = an;
        const int m = rl_i(r_m, t), j1 = rl_i(r_j, t);
        const float thr = rl_f(r_thr, t);
        if (t + 1 < nl)
            load_leaf<D>(r, t + 1, rl_i(r_m, t + 1), rl_i(r_j, t + 1), A, xn, an);
        const int64_t l = l0 + t;
        const int s = rl_i(r.start, t), size = rl_i(r.size, t), prev = rl_i(r.prev, t);
        const int64_t p = (int64_t)s + lane;
        const bool valid = lane < size;
        if (m > HEAVY_M) { // a wave of its own in the per-leaf pass
            if (lane == 0) {
                A.heavy[l] = 1;
                atomicAdd(A.heavy_cnt, 1);
            }
            continue;
        }
        st[ST_CANDS] += m;
        if (m == 1) {
            const int j = j1;
            if (prev != j) {
                const bool ch = valid && aold != j;
                if (ch)
                    A.a[p] = j;
                st[ST_CHANGED] += wave_count(ch);
                if (lane == 0)
                    A.leaf_prev[l] = j;
            }
            // the leaf's exact sum and count: one atomic per lane
            if (lane < 2 * D) {
                int64_t *ac = A.acc + (int64_t)j * D * 2;
                atomicAdd((unsigned long long *)&ac[lane], (unsigned long long)A.leaf_sum[l * D * 2 + lane]);
            } else if (lane == 2 * D) {
                atomicAdd(&A.cnt[j], size);
            }
            st[ST_SINGLE] += size;
            if (A.want_sse && valid) {
                double xd[D], cd[D];
                for (int i = 0; i < D; ++i) {
                    xd[i] = (double)x[i];
                    cd[i] = A.c_in[(int64_t)j * D + i];
                }
                sse += sqdist64<D>(xd, cd);
            }
            continue;
        }
        if (m == 0) { // cannot happen for a well-formed tree; stay correct regardless
            process_leaf_all<D>(l, s, size, prev, A, e, st, sse);
            continue;
        }
        if (lane == 0 && prev != -1)
            A.leaf_prev[l] = -1;
        float blo[3], bhi[3];
        leaf_of<D>(r, t, blo, bhi);
        const int best = assign_point<D>(x, valid, blo, bhi, thr, sn, e, A, sh, st);
        st[ST_EVALS] += (int64_t)m * size;
        leaf_finish<D>(A, l, valid, p, x, best, aold, st, sse);
    }
}

// k_assign_heavy: the leaves k_assign_waves flagged as deferred (more than
// HEAVY_M candidates), each with its own tree search for the leaf box, then
// the point-by-point scan.  Such leaves sit where many centroids crowd
// near a large sparse cell; spreading them over waves keeps one group from
// serialising several of them.  Wave w takes leaves w, w + nw, w + 2nw, ...
// in increasing order, so which wave sums which leaf (and the FP64 SSE
// rounding) does not depend on timing; it clears the flags it consumed.
template <int D>
__global__ void __launch_bounds__(ASSIGN_THREADS) k_assign_heavy(AssignArgs A)
{
    __shared__ WaveHeavy wsh[G_WAVES];
    __shared__ BlockCombine bc;
    combine_init(bc);
    WaveHeavy &sh = wsh[threadIdx.x / WAVE];
    const int64_t w = (int64_t)blockIdx.x * G_WAVES + threadIdx.x / WAVE;
    const int64_t nw = (int64_t)gridDim.x * G_WAVES;
    const float e = err_bound(A.cmax_bits);
    int64_t st[NSTAT] = {0, 0, 0, 0, 0, 0, 0, 0};
    double sse = 0.0;
    if (uniform_int(*A.heavy_cnt) > 0) {
        for (int64_t base = w; base < A.L; base += nw * WAVE) {
            const int64_t lf = base + (int64_t)lane_id() * nw;
            uint64_t mk = __ballot(lf < A.L && A.heavy[lf] != 0);
            while (mk) {
                const int b = __ffsll((unsigned long long)mk) - 1;
                mk &= mk - 1;
                const int64_t l = base + (int64_t)b * nw;
                const int s = A.leaf_start[l], size = A.leaf_start[l + 1] - s, prev = A.leaf_prev[l];
                float blo[3], bhi[3];
                f4_to(A.leaf_box[2 * l], blo);
                f4_to(A.leaf_box[2 * l + 1], bhi);
                const int ln = wave_search<D>(blo, bhi, A, e, sh);
                if (ln >= 0)
                    process_leaf<D>(l, s, size, prev, blo, bhi, ln, A, e, sh, st, sse);
                else
                    process_leaf_all<D>(l, s, size, prev, A, e, st, sse);
                if (lane_id() == 0)
                    A.heavy[l] = 0;
            }
        }
    }
    combine_end(bc, A, st, sse, (A.ngroups + G_WAVES - 1) / G_WAVES + blockIdx.x);
}

// ------------------------------------------------------------- brute force
template <int D>
__global__ void __launch_bounds__(ASSIGN_THREADS) k_assign_brute32(AssignArgs A)
{
    __shared__ BlockStats bs;
    extern __shared__ float4 tile[];
    stats_begin(bs);
    int64_t st[NSTAT] = {0, 0, 0, 0, 0, 0, 0, 0};
    double sse = 0.0;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = p < A.n;
    const float *xs = (const float *)A.xs;
    float x[D];
    for (int i = 0; i < D; ++i)
        x[i] = valid ? xs[(int64_t)i * A.n + p] : 0.0f;
    const float e = err_bound(A.cmax_bits);
    float s1 = INFINITY, s2 = INFINITY;
    int id1 = 0;
    for (int64_t t0 = 0; t0 < A.k; t0 += A.tile) {
        int tn = (int)((A.k - t0) < A.tile ? (A.k - t0) : A.tile);
        __syncthreads();
        for (int t = threadIdx.x; t < tn; t += blockDim.x)
            tile[t] = A.c32[t0 + t];
        __syncthreads();
        for (int t = 0; t < tn; ++t) {
            float4 c4 = tile[t];
            float c[3] = {c4.x, c4.y, c4.z};
            float sv = sqdist32<D>(x, c);
            if (sv < s1) { // ascending j: the first of equal values is kept
                s2 = s1;
                s1 = sv;
                id1 = (int)(t0 + t);
            } else {
                s2 = fminf(s2, sv);
            }
        }
    }
    int best = id1;
    bool re = valid && !margin_safe(s1, s2, e);
    if (re) {
        double xd[D];
        for (int i = 0; i < D; ++i)
            xd[i] = (double)x[i];
        best = brute64_all<D>(xd, A);
    }
    st[ST_RECHECK] += re ? 1 : 0;
    st[ST_EVALS] += valid ? A.k : 0;
    int64_t ch = 0;
    finish_point<D, float>(A, valid, p, x, best, ch, sse);
    st[ST_CHANGED] += ch;
    stats_end(bs, A, st, sse, blockIdx.x);
}

template <int D>
__global__ void __launch_bounds__(ASSIGN_THREADS) k_assign_brute64(AssignArgs A)
{
    __shared__ BlockStats bs;
    extern __shared__ double dtile[];
    stats_begin(bs);
    int64_t st[NSTAT] = {0, 0, 0, 0, 0, 0, 0, 0};
    double sse = 0.0;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = p < A.n;
    const double *xs = (const double *)A.xs;
    double x[D];
    for (int i = 0; i < D; ++i)
        x[i] = valid ? xs[(int64_t)i * A.n + p] : 0.0;
    double best = INFINITY;
    int bj = 0;
    for (int64_t t0 = 0; t0 < A.k; t0 += A.tile) {
        int tn = (int)((A.k - t0) < A.tile ? (A.k - t0) : A.tile);
        __syncthreads();
        for (int t = threadIdx.x; t < tn * D; t += blockDim.x)
            dtile[t] = A.c_in[t0 * D + t];
        __syncthreads();
        for (int t = 0; t < tn; ++t) {
            double Dv = sqdist64<D>(x, dtile + t * D);
            if (Dv < best) {
                best = Dv;
                bj = (int)(t0 + t);
            }
        }
    }
    st[ST_EVALS] += valid ? A.k : 0;
    int64_t ch = 0;
    finish_point<D, double>(A, valid, p, x, bj, ch, sse);
    st[ST_CHANGED] += ch;
    stats_end(bs, A, st, sse, blockIdx.x);
}

// ------------------------------------------------------------- driver
static AssignArgs make_args(km_ctx *ctx, const double *c_in, bool want_sse)
{
    AssignArgs A;
    A.xs = ctx->xs;
    A.n = ctx->n;
    A.k = ctx->k;
    A.a = ctx->a;
    A.c_in = c_in;
    A.c32 = ctx->c32;
    A.cmax_bits = (const unsigned *)ctx->cerr;
    A.leaf_start = ctx->leaf_start;
    A.L = ctx->L;
    A.leaf_box = (const float4 *)ctx->leaf_box;
    A.leaf_sum = ctx->leaf_sum;
    A.leaf_prev = ctx->leaf_prev;
    A.heavy = ctx->heavy;
    A.heavy_cnt = ctx->heavy_cnt;
    A.group_leaf = ctx->group_leaf;
    A.group_box = ctx->group_box;
    A.ngroups = ctx->ngroups;
    A.T = ctx->tree;
    A.S = ctx->S;
    A.fix64 = ctx->fix64;
    A.acc = ctx->acc;
    A.cnt = ctx->cnt;
    A.stat_part = ctx->stat_part;
    A.sse_part = ctx->sse_part;
    A.want_sse = want_sse ? 1 : 0;
    A.tile = ctx->tile;
    return A;
}

// Rows of per-block (brute) or per-wave-group (indexed) statistics partials.
int64_t assign_blocks(const km_ctx *ctx)
{
    if (ctx->cfg.algo == KM_INDEXED)
        return (ctx->ngroups + G_WAVES - 1) / G_WAVES + heavy_waves(ctx->L) / G_WAVES;
    return (ctx->n + ASSIGN_THREADS - 1) / ASSIGN_THREADS;
}

km_status run_assign(km_ctx *ctx, const double *c_in, bool want_sse)
{
    hipStream_t st = ctx->stream;
    AssignArgs A = make_args(ctx, c_in, want_sse);
    unsigned nb = (unsigned)assign_blocks(ctx);
    const unsigned nwg = (unsigned)((ctx->ngroups + G_WAVES - 1) / G_WAVES);
    const int D = ctx->d;
    if (ctx->cfg.algo == KM_INDEXED) {
        const unsigned nhw = (unsigned)(heavy_waves(ctx->L) / G_WAVES);
        if (D == 2) {
            hipLaunchKernelGGL(k_assign_waves<2>, dim3(nwg), dim3(ASSIGN_THREADS), 0, st, A);
            hipLaunchKernelGGL(k_assign_heavy<2>, dim3(nhw), dim3(ASSIGN_THREADS), 0, st, A);
        } else {
            hipLaunchKernelGGL(k_assign_waves<3>, dim3(nwg), dim3(ASSIGN_THREADS), 0, st, A);
            hipLaunchKernelGGL(k_assign_heavy<3>, dim3(nhw), dim3(ASSIGN_THREADS), 0, st, A);
        }
    } else if (ctx->cfg.point_dtype == KM_F32) {
        size_t lds = (size_t)ctx->tile * sizeof(float4);
        if (D == 2)
            hipLaunchKernelGGL(k_assign_brute32<2>, dim3(nb), dim3(ASSIGN_THREADS), lds, st, A);
        else
            hipLaunchKernelGGL(k_assign_brute32<3>, dim3(nb), dim3(ASSIGN_THREADS), lds, st, A);
    } else {
        size_t lds = (size_t)ctx->tile * D * sizeof(double);
        if (D == 2)
            hipLaunchKernelGGL(k_assign_brute64<2>, dim3(nb), dim3(ASSIGN_THREADS), lds, st, A);
        else
            hipLaunchKernelGGL(k_assign_brute64<3>, dim3(nb), dim3(ASSIGN_THREADS), lds, st, A);
    }
    if (!hip_ok(hipGetLastError(), "assign launch"))
        return KM_ERR_HIP;
    return KM_OK;
}

} // namespace ekm
