// Assignment step (Algorithm 1's Assign over the point index, with its kNN
// search over the centroid index), fused with the update of the exact
// cluster sums.
//
// k_assign_waves: one wave per group of up to GROUP_LEAVES consecutive
// leaves; see the comment at the kernel.  Leaves that still lie within half
// the inter bound of their cluster's centroid keep it without any search
// (Eq. (5)); for the others, U, the smallest FP32 max-distance from a box to
// a node or centroid seen so far, bounds the distance from every point of
// the box to some centroid (the paper inherits such bounds from parent
// nodes, Eq. (7)); nodes and centroids whose FP32 min-distance to the box
// exceeds prune_threshold(U) are dropped.
//
// The cluster sums are exact integers (fixed point) that persist from step
// to step: a point or leaf whose cluster changes moves its exact value from
// the old cluster to the new one (the paper's running sum vectors, Alg. 1's
// cluster update on a move), which gives the same integers as summing every
// cluster afresh, in any order.
//
// k_assign_brute32 / k_assign_brute64: Lloyd's assignment over all k
// centroids staged through LDS tiles (the GPU baseline; FP64 is the plain
// canonical computation); they sum every cluster afresh each step.
#include "ekm_internal.hpp"

namespace ekm {

constexpr int ASSIGN_THREADS = 256;
constexpr int G_WAVES = ASSIGN_THREADS / WAVE; // waves per workgroup of the per-leaf pass
// Per-wave LDS capacities: candidate list entries and descent entries per
// level.  A leaf whose list does not fit in the main pass goes to the
// per-leaf pass, whose waves have room for crowded leaves (one workgroup
// per CU there).
constexpr int SW_MAIN = 256, FR_MAIN = 1024;
static_assert(HEAVY_M >= SW_MAIN, "no leaf is deferred for its candidate count alone (see HEAVY_M)");
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
    const float *cb_s;  // [k] smallest FP32 squared distance from fl32(c_j) to another fl32 centroid
    // leaves and groups
    const int32_t *leaf_start;
    int64_t L;
    const float4 *leaf_box;
    const int64_t *leaf_sum;
    int32_t *leaf_own;
    float *leaf_r;                // [L] per-leaf distance bounds (see km_ctx::leaf_r)
    const unsigned *drift_max;    // bound on the largest centroid drift since the previous step (float bits)
    int32_t *heavy;
    int32_t *heavy_cnt; // their number (reset by the finalize kernel)
    int64_t assign_wg;  // workgroups of the main pass
    const int32_t *group_leaf;
    const float4 *group_box;
    int64_t ngroups;
    // centroid trees (one per cloud) and the cloud of each group and leaf
    const TreeArgs *trees;
    const int32_t *group_cloud, *leaf_cloud;
    // exact sums
    int S;
    int fix64;
    int64_t *acc;
    int32_t *cnt;
    int64_t *stat_part;
    int tile;
    // candidate capacities in use (at most the LDS capacities)
    int sw_main, fr_main, sw_heavy, fr_heavy, heavy_m;
    int32_t *group_parts; // [ngroups] parts each group is split into (0 or 1: whole), set from the last step
    int split_sn;         // a group whose list reaches this length is split at the next step
    const int32_t *ctl; // device loop control: every kernel returns at once when ctl[CTL_STOP]
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
    __syncthreads();
}

// per-thread counters -> partial row `row`
__device__ inline void stats_end(BlockStats &bs, const AssignArgs &A, const int64_t (&c)[NSTAT], int64_t row)
{
#pragma unroll
    for (int q = 0; q < NSTAT; ++q) {
        int64_t w = wave_sum_i64(c[q]);
        if (lane_id() == 0 && w)
            atomicAdd((unsigned long long *)&bs.v[q], (unsigned long long)w);
    }
    __syncthreads();
    if (threadIdx.x < NSTAT)
        A.stat_part[row * NSTAT + threadIdx.x] = bs.v[threadIdx.x];
}

// Statistics of one workgroup of independent waves: each wave adds its
// (wave-uniform) counters to LDS with atomics; the wave that arrives last
// writes the workgroup's row.  Initialised before any wave diverges (the
// kernel's single workgroup barrier).
struct BlockCombine {
    unsigned long long v[NSTAT];
    int done;
};

// Units of work of a main-pass workgroup (2D): (group, part, parts) entries
// that its waves claim one after the other.
constexpr int MAX_PARTS = 4;  // a group's leaves are split over at most this many waves
constexpr int SPLIT_SN = 48;  // list length from which a group is split at the next step
struct UnitList {
    int32_t unit[MAIN_WAVES<2> * MAX_PARTS]; // group slot | part << 8 | parts << 16
    int n, next;
};

__device__ inline void combine_init(BlockCombine &bc)
{
    if (threadIdx.x < NSTAT)
        bc.v[threadIdx.x] = 0;
    if (threadIdx.x == 0)
        bc.done = 0;
    __syncthreads();
}

// Adds one wave's counters to the workgroup's totals.
template <class T>
__device__ inline void combine_add(BlockCombine &bc, const T (&c)[NSTAT])
{
    const int lane = lane_id();
    int64_t mine = 0;
#pragma unroll
    for (int q = 0; q < NSTAT; ++q)
        if (lane == q)
            mine = c[q];
    if (lane < NSTAT && mine)
        __hip_atomic_fetch_add(&bc.v[lane], (unsigned long long)mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Adds one wave's counters (if any) and, in the last wave of the workgroup to
// get here, writes the workgroup's row.
template <class T>
__device__ inline void combine_end(BlockCombine &bc, const AssignArgs &A, const T (&c)[NSTAT], int64_t row)
{
    const int lane = lane_id();
    combine_add(bc, c);
    int last = 0;
    if (lane == 0)
        last = __hip_atomic_fetch_add(&bc.done, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) ==
               (int)(blockDim.x / WAVE) - 1;
    if (!rl_i(last, 0))
        return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (lane < NSTAT)
        A.stat_part[row * NSTAT + lane] =
            (int64_t)__hip_atomic_load(&bc.v[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Number of lanes of the wave with `p` set (wave-uniform).
__device__ inline int wave_count(bool p) { return __popcll(__ballot(p)); }

// ------------------------------------------------------------- tree search
// Fills sh.sc with the candidate list of box [lo, hi] and returns its
// length, or -1 if a descent level (more than fr / TREE_BUCKET kept nodes)
// or the list (more than sw entries) does not fit; fr and sw are at most the
// LDS capacities of WS.  The whole wave calls; the result is uniform.
//
// The descent starts at the lowest tree level with at most TREE_START_MAX
// nodes and evaluates every node there; each later level evaluates the
// children of the nodes kept at the level above (at most FR_CAP entries),
// and the last step the centroids of the kept buckets.  U is the smallest
// box-to-node max-distance seen at any level (a valid bound: every node
// holds a centroid).  Each lane keeps the min-distances of its entries in
// its own LDS slots between the two passes of a level.  thr_cap caps the
// pruning threshold: prune_threshold_r of a bound on the exact distance from
// every point of the box to its previous centroid, carried over from the
// previous step with the centroids' drift (Eq. (9)'s use of drift), or
// +inf.  A centroid beyond it is farther than every point's previous
// centroid, so it is nobody's nearest.
template <int D, class WS>
__device__ int wave_search(const float *lo, const float *hi, const TreeArgs *Tp, float e, WS &sh, int sw, int fr,
                           float thr_cap)
{
    const int npar = fr / TREE_BUCKET;
    const TreeArgs &T = *Tp; // the cloud's tree (read through the pointer: no register copy)
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
        const float thr = fminf(prune_threshold(U, e), thr_cap);
        const int nxt = cur ^ 1;
        int cnt = 0;
        for (int i0 = 0; i0 < F; i0 += WAVE) {
            const int i = i0 + lane;
            const bool keep = i < F && sh.fm[i] <= thr;
            const uint64_t mk = __ballot(keep);
            const int pos = cnt + __popcll(mk & lt);
            if (keep && pos < npar)
                sh.par[nxt][pos] =
                    np < 0 ? i : sh.par[cur][i / TREE_BUCKET] * TREE_BUCKET + i % TREE_BUCKET;
            cnt += __popcll(mk);
        }
        if (cnt > npar)
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
        if (t < T.k) {
            float cc[3];
            f4_to(T.cs[t], cc);
            m = box_mind<D>(lo, hi, cc);
            Ul = fminf(Ul, box_maxd<D>(lo, hi, cc));
        }
        sh.fm[i] = m;
    }
    U = fminf(U, wave_min_f32(Ul));
    const float thr = fminf(prune_threshold(U, e), thr_cap);
    int cnt = 0;
    for (int i0 = 0; i0 < F; i0 += WAVE) {
        const int i = i0 + lane;
        const bool keep = i < F && sh.fm[i] <= thr;
        const uint64_t mk = __ballot(keep);
        const int pos = cnt + __popcll(mk & lt);
        if (keep && pos < sw) // the entry was loaded by this lane a moment ago (cache hit)
            sh.sc[pos] = T.cs[(int64_t)sh.par[cur][i / TREE_BUCKET] * TREE_BUCKET + i % TREE_BUCKET];
        cnt += __popcll(mk);
    }
    wave_sync();
    return cnt > sw ? -1 : cnt;
}

// --------------------------------------------------------------- exact sums
// Fixed-point coordinates of a lane's point: (value, 0) when every value
// fits FIX64_BITS bits, else the (hi, lo) split; zero for lanes without one.
template <int D>
__device__ inline void fix_point(const float (&x)[D], bool on, const AssignArgs &A, int64_t (&v0)[D],
                                 int64_t (&v1)[D])
{
#pragma unroll
    for (int i = 0; i < D; ++i) {
        int64_t h = 0, l = 0; // one assignment per element: the array stays in registers
        if (A.fix64)
            h = fix_f32(x[i], A.S);
        else
            fix_split_f32(x[i], A.S, h, l);
        v0[i] = on ? h : 0;
        v1[i] = on ? l : 0;
    }
}

// Accumulator limbs of an exact value: V = hi * 2^32 + lo with lo in [0, 2^32).
__device__ inline void limbs(__int128 V, int64_t &hi, int64_t &lo)
{
    hi = (int64_t)(V >> 32);
    lo = (int64_t)(V & (__int128)0xffffffff);
}

// Adds sign * x (exact) and sign * 1 to cluster `key` for every lane with
// `in`.  Lanes of one cluster are summed in the wave (DPP), then lanes
// 0..2D-1 add the limbs and lane 2D the count with integer atomics; after
// ACC_ROUNDS clusters the remaining lanes add their own values.  Integer
// addition makes the result independent of the order of all such updates.
constexpr int ACC_ROUNDS = 3;
template <int D>
__device__ inline void wave_scatter(bool in, int key, int sign, const int64_t (&v0)[D], const int64_t (&v1)[D],
                                    const AssignArgs &A)
{
    const int lane = lane_id();
    uint64_t active = __ballot(in);
    for (int round = 0; active; ++round) {
        if (round == ACC_ROUNDS) {
            if ((active >> lane) & 1ull) {
                int64_t *ac = A.acc + (int64_t)key * D * 2;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    __int128 V = A.fix64 ? (__int128)v0[i] : (((__int128)v0[i] << 32) + (__int128)v1[i]);
                    int64_t h, l;
                    limbs(sign < 0 ? -V : V, h, l);
                    atomicAdd((unsigned long long *)&ac[2 * i], (unsigned long long)h);
                    atomicAdd((unsigned long long *)&ac[2 * i + 1], (unsigned long long)l);
                }
                atomicAdd(&A.cnt[key], sign);
            }
            break;
        }
        const int c = rl_i(key, __ffsll((unsigned long long)active) - 1);
        const bool inr = in && key == c;
        const uint64_t grp = __ballot(inr);
        active &= ~grp;
        int64_t mine = 0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            __int128 V;
            if (A.fix64)
                V = (__int128)wave_sum_i64(inr ? v0[i] : 0);
            else
                V = ((__int128)wave_sum_i64(inr ? v0[i] : 0) << 32) + (__int128)wave_sum_i64(inr ? v1[i] : 0);
            int64_t h, l;
            limbs(sign < 0 ? -V : V, h, l);
            if (lane == 2 * i)
                mine = h;
            if (lane == 2 * i + 1)
                mine = l;
        }
        if (lane < 2 * D)
            atomicAdd((unsigned long long *)&A.acc[(int64_t)c * D * 2 + lane], (unsigned long long)mine);
        else if (lane == 2 * D)
            atomicAdd(&A.cnt[c], sign * __popcll(grp));
    }
}

// Adds sign * (the leaf's precomputed exact sum) and sign * size to cluster
// `key` (a whole leaf moving between clusters, without reading its points).
template <int D>
__device__ inline void leaf_sum_add(const AssignArgs &A, int64_t l, int key, int sign, int size)
{
    const int lane = lane_id();
    if (lane < 2 * D) {
        const int64_t *ls = A.leaf_sum + (l * D + (lane >> 1)) * 2;
        __int128 V = ((__int128)ls[0] << 32) + (__int128)ls[1];
        int64_t h, lo;
        limbs(sign < 0 ? -V : V, h, lo);
        atomicAdd((unsigned long long *)&A.acc[(int64_t)key * D * 2 + lane], (unsigned long long)((lane & 1) ? lo : h));
    } else if (lane == 2 * D) {
        atomicAdd(&A.cnt[key], sign * size);
    }
}

// Canonical FP64 argmin over centroids [j0, j1) (lowest index on ties).
template <int D>
__device__ inline int brute64_all(const double (&xd)[D], const AssignArgs &A, int64_t j0, int64_t j1)
{
    double best = INFINITY;
    int bj = (int)j0;
    for (int64_t j = j0; j < j1; ++j) {
        double Dv = sqdist64<D>(xd, A.c_in + j * D);
        if (Dv < best) {
            best = Dv;
            bj = (int)j;
        }
    }
    return bj;
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
// one when m == 1), the threshold for the later mask passes (capped by
// thr_cap, as in wave_search) and U, the smallest FP32 box max-distance to
// a list entry (every point of the box is within exact distance
// dist_hi(U, e) of that entry, hence of its own nearest centroid).
template <int D, class WS>
__device__ inline int leaf_filter(const float *blo, const float *bhi, int sn, float e, const WS &sh,
                                  float thr_cap, float &thr, int &j1, float &Uout)
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
    Uout = wave_min_f32(U);
    thr = fminf(prune_threshold(Uout, e), thr_cap);
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
// entries within `thr` of the leaf box, in chunks of 64 (chunks c0,
// c0 + cstep, ...), each candidate broadcast from the lane that holds it.
template <int D, class WS>
__device__ inline Best2 scan_list(const float (&x)[D], const float *blo, const float *bhi, float thr, int sn,
                                  const WS &sh, int c0, int cstep)
{
    const int lane = lane_id();
    const int nch = (sn + WAVE - 1) / WAVE;
    Best2 bs[SCAN_ILP];
#pragma unroll
    for (int u = 0; u < SCAN_ILP; ++u)
        bs[u] = best2_init();
    for (int c = c0; c < nch; c += cstep) {
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
    return bs[0];
}

// Decision of one point from its FP32 scan result b over the leaf's
// candidates.  Lanes with `need` whose best-vs-second margin is below the
// error bound are decided again with canonical FP64 distances over the
// candidates that can still be nearest: those whose FP32 lower bound does
// not exceed the best one's upper bound (any other is strictly farther in
// exact and in FP64 arithmetic).  Returns the centroid id (meaningful for
// lanes with `need`).
template <int D, class WS>
__device__ inline int recheck_points(const float (&x)[D], bool re, float s1, int id1,
                                                        const float *blo, const float *bhi, float thr, int sn,
                                                        float e, const AssignArgs &A, const WS &sh)
{
    const int lane = lane_id();
    const int nch = (sn + WAVE - 1) / WAVE;
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
            const int bl = __ffsll((unsigned long long)mk) - 1;
            mk &= mk - 1;
            float cc[3] = {rl_f(c4.x, bl), rl_f(c4.y, bl), D == 3 ? rl_f(c4.z, bl) : 0.0f};
            const int cid = rl_i(__float_as_int(c4.w), bl);
            double cd[D];
            for (int i = 0; i < D; ++i)
                cd[i] = rl_d(cdl[i], bl);
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

template <int D, class WS>
__device__ inline int finish_point(const float (&x)[D], bool need, const Best2 &b, const float *blo,
                                   const float *bhi, float thr, int sn, float e, const AssignArgs &A, const WS &sh,
                                   int32_t (&st)[NSTAT], float &s1out)
{
    const float s1 = best2_s1(b), s2 = b.s2;
    s1out = s1;
    const int id1 = best2_id(b);
    const bool re = need && !margin_safe(s1, s2, e);
    const int nre = wave_count(re);
    if (nre == 0)
        return id1;
    st[ST_RECHECK] += nre;
    return recheck_points<D>(x, re, s1, id1, blo, bhi, thr, sn, e, A, sh);
}

template <int D, class WS>
__device__ inline int assign_point(const float (&x)[D], bool need, const float *blo, const float *bhi, float thr,
                                   int sn, float e, const AssignArgs &A, const WS &sh, int32_t (&st)[NSTAT],
                                   float &s1)
{
    const Best2 b = scan_list<D>(x, blo, bhi, thr, sn, sh, 0, 1);
    return finish_point<D>(x, need, b, blo, bhi, thr, sn, e, A, sh, st, s1);
}

// FP32 scan of all k centroids (fl32 copies, 64 at a time in registers, the
// next chunk loading while this one is scanned; ascending j), same margin
// rule, canonical FP64 brute force for the lanes that need it.  For leaves
// whose candidate list does not fit anywhere.
template <int D>
__device__ inline int scan_all(const float (&x)[D], bool need, float e, const AssignArgs &A, const TreeArgs *Tp,
                               int32_t (&st)[NSTAT], float &s1out)
{
    const int lane = lane_id();
    const int64_t c0 = Tp->c0, c1 = Tp->c0 + Tp->k; // the cloud's centroids
    Best2 bs[SCAN_ILP];
#pragma unroll
    for (int u = 0; u < SCAN_ILP; ++u)
        bs[u] = best2_init();
    float4 cur = c0 + lane < c1 ? A.c32[c0 + lane] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int64_t j0 = c0; j0 < c1; j0 += WAVE) {
        const int64_t jn = j0 + WAVE + lane;
        const float4 nxt = jn < c1 ? A.c32[jn] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const int cn = (int)(c1 - j0 < WAVE ? c1 - j0 : WAVE);
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
    s1out = s1;
    int best = best2_id(bs[0]);
    const bool re = need && !margin_safe(s1, s2, e);
    st[ST_RECHECK] += wave_count(re);
    st[ST_FALLBACK_PTS] += wave_count(need);
    if (re) {
        double xd[D];
        for (int i = 0; i < D; ++i)
            xd[i] = (double)x[i];
        best = brute64_all<D>(xd, A, c0, c1);
    }
    return best;
}

// A leaf as the wave sees it (uniform values).
// oc / ocb: fl32 of the centroid of cluster `own` and its inter bound cb_s
// (when own >= 0).
// R: bound on the exact distance from each of its points to its previous
// centroid at this step's positions (+inf if unknown).
struct LeafJob {
    int64_t l;
    int s, size, own;
    float lo[3], hi[3];
    float oc[3], ocb;
    float R;
};

// Per-leaf data held by lane t of the wave for leaf l0 + t of its group.
struct LeafRegs {
    float lo[3], hi[3];
    float oc[3], ocb;
    float R;
    int start, size, own;
};

template <int D>
__device__ inline LeafJob job_of(const LeafRegs &r, int t, int64_t l0)
{
    LeafJob J;
    J.l = l0 + t;
    J.s = rl_i(r.start, t);
    J.size = rl_i(r.size, t);
    J.own = rl_i(r.own, t);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        J.lo[i] = i < D ? rl_f(r.lo[i], t) : 0.0f;
        J.hi[i] = i < D ? rl_f(r.hi[i], t) : 0.0f;
        J.oc[i] = i < D ? rl_f(r.oc[i], t) : 0.0f;
    }
    J.ocb = rl_f(r.ocb, t);
    J.R = rl_f(r.R, t);
    return J;
}

template <int D>
__device__ inline LeafJob job_load(const AssignArgs &A, int64_t l)
{
    LeafJob J;
    J.l = l;
    J.s = A.leaf_start[l];
    J.size = A.leaf_start[l + 1] - J.s;
    J.own = A.leaf_own[l];
    f4_to(A.leaf_box[2 * l], J.lo);
    f4_to(A.leaf_box[2 * l + 1], J.hi);
    J.oc[0] = J.oc[1] = J.oc[2] = J.ocb = 0.0f;
    if (J.own >= 0) {
        f4_to(A.c32[J.own], J.oc);
        J.ocb = A.cb_s[J.own];
    }
    J.R = bound_add(A.leaf_r[l], __uint_as_float(*A.drift_max));
    return J;
}

// A lane's point of a leaf and its previous assignment (-1 past the leaf's
// end or before the first step).
template <int D>
struct LeafPts {
    float x[D];
    int a;
};

template <int D>
__device__ inline LeafPts<D> load_pts(const AssignArgs &A, const LeafJob &J)
{
    const int lane = lane_id();
    const bool valid = lane < J.size;
    const int64_t p = (int64_t)J.s + lane;
    const float *xs = (const float *)A.xs;
    LeafPts<D> P;
    for (int i = 0; i < D; ++i)
        P.x[i] = valid ? xs[(int64_t)i * A.n + p] : 0.0f;
    P.a = valid ? A.a[p] : -1;
    return P;
}

// A leaf with a single candidate j (Eq. (6): the whole leaf is assigned to
// it without any distance evaluation) that was wholly in one cluster (or in
// none yet): its precomputed exact sum moves, its points are not read.
// R: the leaf's new distance bound.
template <int D>
__device__ void single_leaf(const AssignArgs &A, const LeafJob &J, int j, float R, int32_t (&st)[NSTAT])
{
    st[ST_SINGLE] += J.size;
    const int lane = lane_id();
    if (lane == 0)
        A.leaf_r[J.l] = R;
    if (J.own == j)
        return; // already wholly in j
    if (lane < J.size)
        A.a[(int64_t)J.s + lane] = j;
    st[ST_CHANGED] += J.size;
    if (J.own >= 0)
        leaf_sum_add<D>(A, J.l, J.own, -1, J.size);
    leaf_sum_add<D>(A, J.l, j, +1, J.size);
    if (lane == 0)
        A.leaf_own[J.l] = j;
}

// Point-by-point decision of a leaf (lane = point, P loaded by the caller).
// In a leaf wholly in cluster j, a point still within half the inter bound
// of c_j keeps it (Eq. (4); c_j and cb_j are the same for the whole wave);
// the other points are decided by `scan` (a single candidate of a leaf of
// mixed clusters: every point goes to it).  Changed points move their exact
// values between clusters (one inlined copy of the scatter, run for the
// old and then the new cluster); the leaf's common cluster and its distance
// bound (each point's exact distance to its centroid is at most dist_hi of
// its FP32 distance to the centroid kept, or to the FP32 best, which is no
// nearer than the chosen one) are recorded for the next step.  `scan`
// returns the decision and the FP32 best distance.
template <int D, class ScanFn>
__device__ void decide_points(const AssignArgs &A, const LeafJob &J, const LeafPts<D> &P, float e,
                              int64_t evals_per_point, ScanFn scan, int32_t (&st)[NSTAT])
{
    const int lane = lane_id();
    const bool valid = lane < J.size;
    const int64_t p = (int64_t)J.s + lane;
    bool pk = false;
    float s = 0.0f; // FP32 distance to the centroid kept or found
    if (J.own >= 0) {
        s = sqdist32<D>(P.x, J.oc);
        pk = valid && inter_keep(J.ocb, s, e);
        st[ST_KEEP_PTS] += wave_count(pk);
    }
    const bool need = valid && !pk;
    const int nneed = wave_count(need);
    int best = P.a;
    if (nneed) {
        st[ST_EVALS] += evals_per_point * nneed;
        float s1;
        const int b = scan(P.x, need, s1);
        if (need) {
            best = b;
            s = s1;
        }
    }
    const float R = -wave_min_f32(valid ? -dist_hi(s, e) : 0.0f);
    if (lane == 0)
        A.leaf_r[J.l] = R;
    if (nneed == 0)
        return; // every point keeps its cluster: nothing changes
    const bool ch = valid && best != P.a;
    const int nch = wave_count(ch);
    if (nch) {
        st[ST_CHANGED] += nch;
        int64_t v0[D], v1[D];
        fix_point<D>(P.x, ch, A, v0, v1);
#pragma unroll 1
        for (int pass = 0; pass < 2; ++pass)
            wave_scatter<D>(pass ? ch : ch && P.a >= 0, pass ? best : P.a, pass ? +1 : -1, v0, v1, A);
        if (ch)
            A.a[p] = best;
    }
    const int b0 = rl_i(best, 0); // lane 0 always holds a point
    const int own = wave_count(valid && best != b0) == 0 ? b0 : OWN_MIXED;
    if (own != J.own && lane == 0)
        A.leaf_own[J.l] = own;
}

// A leaf whose candidate list does not fit: every point scans all k.
template <int D>
__device__ void leaf_all(const AssignArgs &A, const LeafJob &J, float e, const TreeArgs *Tp, int32_t (&st)[NSTAT])
{
    const LeafPts<D> P = load_pts<D>(A, J);
    decide_points<D>(A, J, P, e, Tp->k,
                     [&](const float (&x)[D], bool need, float &s1) { return scan_all<D>(x, need, e, A, Tp, st, s1); },
                     st);
}

// A leaf against the wave's list (sn entries), after its filter found m >= 1
// candidates (m == 0 cannot happen for a well-formed tree; callers send such
// a leaf to the scan of all k regardless) and U (see leaf_filter); P: its
// points (loaded by the caller; not read for a single candidate of a leaf
// wholly in one cluster).
template <int D, class WS>
__device__ void leaf_listed(const AssignArgs &A, const LeafJob &J, int m, int j1, float thr, float U, int sn,
                            float e, const WS &sh, const LeafPts<D> &P, int32_t (&st)[NSTAT])
{
    st[ST_CANDS] += m;
    if (m == 1 && J.own != OWN_MIXED) {
        single_leaf<D>(A, J, j1, dist_hi(U, e), st);
        return;
    }
    if (m == 1)
        st[ST_SINGLE] += J.size;
    decide_points<D>(A, J, P, e, m == 1 ? 0 : m,
                     [&](const float (&x)[D], bool need, float &s1) {
                         if (m == 1) {
                             s1 = U; // the box max-distance bounds every point's distance
                             return j1;
                         }
                         return assign_point<D>(x, need, J.lo, J.hi, thr, sn, e, A, sh, st, s1);
                     },
                     st);
}

__device__ inline void defer_leaf(const AssignArgs &A, int64_t l, int32_t (&st)[NSTAT])
{
    st[ST_DEFERRED] += 1;
    if (lane_id() == 0)
        A.heavy[atomicAdd(A.heavy_cnt, 1)] = (int32_t)l;
}

// k_assign_waves: one wave per group (at most GROUP_LEAVES consecutive
// leaves inside one compact Morton cell, see leaves.hip); the waves of a
// workgroup are independent and the kernel has no workgroup barrier.  The
// points form a three-level hierarchy, region (the group's cell) -> leaf ->
// point, and the region's candidate list and bounds pass down to its leaves
// (Eq. (7)).
//
//  1. Inter bound (Eq. (5)): a leaf wholly in cluster j whose box lies
//     within half of cb_j (the distance from c_j to its nearest other
//     centroid) of c_j stays in j; nothing about it changes.  A group whose
//     leaves all stay skips the rest.
//  2. Group search: the centroid-tree descent for the bounding box of the
//     remaining leaves gives the list S (kNN-style pruning with the upper
//     bound U, the node pruning of Eq. (8), made conservative for rounding).
//  3. Leaf filter: for a leaf box b inside that box, the same rule applied
//     to S alone gives exactly the leaf's candidates over all k centroids:
//     a centroid outside S has min-distance to b at least its min-distance
//     to the searched box, above prune_threshold(U_box) >=
//     prune_threshold(U_b), and the centroid that realised U_box is in S.
//  4. A region whose list holds one centroid is assigned to it whole, and a
//     leaf with one candidate is assigned to it, without any distance
//     evaluation (Eq. (6)'s batch assignment).  Otherwise each lane (one
//     point) keeps its cluster by the inter bound (Eq. (4)) or scans the
//     candidates in FP32; a point whose best-vs-second margin is below the
//     error bound is decided again with canonical FP64 distances.
//
// If S does not fit, the wave searches leaf by leaf; a leaf whose own list
// does not fit, or that has more than heavy_m candidates, goes to the
// per-leaf pass.  Results are the same on every path.
template <int D>
__device__ void group_work(int64_t g, int part, int parts, const AssignArgs &A, WaveMain &sh,
                           int32_t (&st)[NSTAT])
{
    const int lane = lane_id();
    const bool inpart = (lane & (parts - 1)) == part; // this unit's leaves: t = part, part + parts, ...
    const float e = err_bound(A.cmax_bits);
    const TreeArgs *Tp = A.trees + A.group_cloud[g];
    const int64_t l0 = A.group_leaf[g];
    const int nl = A.group_leaf[g + 1] - (int)l0; // 1..GROUP_LEAVES
    const float drift = __uint_as_float(*A.drift_max);
    LeafRegs r;
    for (int i = 0; i < 3; ++i)
        r.lo[i] = r.hi[i] = 0.0f;
    r.start = r.size = 0;
    r.own = OWN_NONE;
    r.R = 0.0f;
    if (lane < nl) {
        const float4 bl = A.leaf_box[2 * (l0 + lane)], bh = A.leaf_box[2 * (l0 + lane) + 1];
        f4_to(bl, r.lo);
        f4_to(bh, r.hi);
        r.start = A.leaf_start[l0 + lane];
        r.size = A.leaf_start[l0 + lane + 1] - r.start;
        r.own = A.leaf_own[l0 + lane];
        r.R = bound_add(A.leaf_r[l0 + lane], drift); // the last step's bound, moved with the centroids
    }
    bool keep = false;
    r.oc[0] = r.oc[1] = r.oc[2] = r.ocb = 0.0f;
    if (lane < nl && r.own >= 0) {
        f4_to(A.c32[r.own], r.oc);
        r.ocb = A.cb_s[r.own];
        const float s = box_maxd<D>(r.lo, r.hi, r.oc);
        keep = inter_keep(r.ocb, s, e);
        if (keep && inpart)
            A.leaf_r[l0 + lane] = dist_hi(s, e); // every point is within this of c_own
    }
    const uint64_t kept = __ballot(keep);
    const uint64_t todo_all = __ballot(lane < nl) & ~kept;
    uint64_t todo = todo_all & __ballot(inpart);
    if (kept)
        st[ST_KEEP_LEAF_PTS] += wave_sum_i32(keep && inpart ? r.size : 0);
    // the unit holding the group's first leaf to decide sets the group's
    // parts for the next step (from its first list)
    const bool lead = todo_all ? (((todo_all & (~todo_all + 1ull)) & todo) != 0) : part == 0;
    if (!todo) {
        if (!todo_all && part == 0) {
            st[ST_GROUP_SKIP] += 1;
            if (lane == 0 && parts > 1)
                A.group_parts[g] = 1;
        }
        return;
    }
    // The points of every leaf still to decide, loaded at once: one round
    // trip for the group, overlapping the search below (slot t holds this
    // lane's point of leaf l0 + t).  The leaf loop then issues no loads after
    // its stores and atomics, so it never waits for those to complete.
    float gx[GROUP_LEAVES][D];
    int ga[GROUP_LEAVES];
#pragma unroll
    for (int t = 0; t < GROUP_LEAVES; ++t) {
        const int64_t p = (int64_t)rl_i(r.start, t) + lane;
        const bool v = ((todo >> t) & 1ull) && lane < rl_i(r.size, t);
#pragma unroll
        for (int i = 0; i < D; ++i)
            gx[t][i] = v ? ((const float *)A.xs)[(int64_t)i * A.n + p] : 0.0f;
        ga[t] = v ? A.a[p] : -1;
    }
    // Searches: one for the bounding box of every remaining leaf; if its
    // list does not fit, one per leaf (a leaf whose own list still does not
    // fit goes to the per-leaf pass).  One inlined copy of the search, the
    // filters and the leaf decisions serves both.
    bool per_leaf = false;
    while (todo) {
        const uint64_t unit = per_leaf ? (todo & (~todo + 1ull)) : todo; // leaves of this search
        const bool mine = (unit >> lane) & 1ull;
        float ulo[3] = {0.0f, 0.0f, 0.0f}, uhi[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int i = 0; i < D; ++i) {
            ulo[i] = wave_min_f32(mine ? r.lo[i] : INFINITY);
            uhi[i] = -wave_min_f32(mine ? -r.hi[i] : INFINITY);
        }
        const float Ru = -wave_min_f32(mine ? -r.R : 0.0f); // every point of the unit is within Ru of a centroid
        const int sn = wave_search<D>(ulo, uhi, Tp, e, sh, A.sw_main, A.fr_main, prune_threshold_r(Ru, e));
        if (D == 2 && lead && !per_leaf && lane == 0) {
            // a long list: the next step splits the group's leaves over 2 or 4
            // waves (at most one per leaf to decide)
            // (a part's list is shorter than the whole group's: a split group
            // stays split down to a quarter of the threshold)
            const int nd = __popcll(todo_all);
            const int lim = parts > 1 ? (A.split_sn + 3) / 4 : A.split_sn;
            const int want = sn < 0 || sn >= lim ? (nd >= 4 ? 4 : (nd >= 2 ? 2 : 1)) : 1;
            if (want != (parts > 1 ? parts : 1))
                A.group_parts[g] = want;
        }
        if (sn < 0) {
            if (!per_leaf) {
                st[ST_GROUP_OVF] += 1;
                per_leaf = true;
            } else {
                defer_leaf(A, l0 + __ffsll((unsigned long long)unit) - 1, st);
                todo &= ~unit;
            }
            continue;
        }
        todo &= ~unit;
        // filter every leaf of the unit first; lane t keeps leaf t's results
        float r_thr = 0.0f, r_u = 0.0f;
        int r_m = 0, r_j = -1;
        if (sn == 1 && !per_leaf) {
            // a region (the group's cell) whose list holds one centroid: it is
            // every point's nearest, and the region is assigned to it as a unit
            float cc[3];
            const float4 c4 = sh.sc[0];
            f4_to(c4, cc);
            if (mine) {
                r_m = 1;
                r_j = __float_as_int(c4.w);
                r_u = box_maxd<D>(r.lo, r.hi, cc); // the leaf filter's U
            }
            st[ST_REGION_PTS] += wave_sum_i32(mine ? r.size : 0);
        }
        for (uint64_t q = (sn == 1 && !per_leaf) ? 0ull : unit; q; q &= q - 1) {
            const int t = __ffsll((unsigned long long)q) - 1;
            float blo[3], bhi[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                blo[i] = i < D ? rl_f(r.lo[i], t) : 0.0f;
                bhi[i] = i < D ? rl_f(r.hi[i], t) : 0.0f;
            }
            float thr, U;
            int j1;
            const int m = leaf_filter<D>(blo, bhi, sn, e, sh, prune_threshold_r(rl_f(r.R, t), e), thr, j1, U);
            if (lane == t) {
                r_thr = thr;
                r_m = m;
                r_j = j1;
                r_u = U;
            }
        }
        for (uint64_t q = unit; q; q &= q - 1) {
            const int t = __ffsll((unsigned long long)q) - 1;
            const LeafJob J = job_of<D>(r, t, l0);
            const int m = rl_i(r_m, t);
            LeafPts<D> P; // slot t (selected with a uniform index: the slots stay in registers)
#pragma unroll
            for (int u = 0; u < GROUP_LEAVES; ++u)
                if (u == t) {
#pragma unroll
                    for (int i = 0; i < D; ++i)
                        P.x[i] = gx[u][i];
                    P.a = ga[u];
                }
            if (m == 0 || m > A.heavy_m) { // a wave of its own in the per-leaf pass
                defer_leaf(A, J.l, st);
                continue;
            }
            leaf_listed<D>(A, J, m, rl_i(r_j, t), rl_f(r_thr, t), rl_f(r_u, t), sn, e, sh, P, st);
        }
    }
}

template <int D>
__global__ void __launch_bounds__(MAIN_WAVES<D> * WAVE) k_assign_waves(AssignArgs A)
{
    constexpr int NW = MAIN_WAVES<D>;
    if (A.ctl[CTL_STOP])
        return; // the run is over (the whole workgroup returns)
    __shared__ WaveMain wsh[NW];
    __shared__ BlockCombine bc;
    if (D == 3) {
        // one group per wave: the loop below costs the 3D kernel registers
        // (3 waves per SIMD instead of 4), and 3D lists stay short
        combine_init(bc);
        const int wv = uniform_int(threadIdx.x / WAVE);
        const int64_t g = (int64_t)blockIdx.x * NW + wv;
        int32_t st[NSTAT] = {};
        if (g < A.ngroups)
            group_work<D>(g, 0, 1, A, wsh[wv], st);
        combine_end(bc, A, st, blockIdx.x);
        return;
    }
    __shared__ UnitList ul;
    if (threadIdx.x == 0) {
        // the workgroup's groups as units of work: a group split at this step
        // (a long list at the last one) gives one unit per part
        int n = 0;
        for (int u = 0; u < NW; ++u) {
            const int64_t g = (int64_t)blockIdx.x * NW + u;
            if (g >= A.ngroups)
                break;
            const int gp = A.group_parts[g];
            const int parts = gp >= 4 ? 4 : (gp >= 2 ? 2 : 1); // a power of two
            for (int p = 0; p < parts; ++p)
                ul.unit[n++] = u | (p << 8) | (parts << 16);
        }
        ul.n = n;
        ul.next = 0;
    }
    combine_init(bc); // (its barrier also publishes the unit list)
    const int wv = uniform_int(threadIdx.x / WAVE); // the compiler then keeps group values in scalar registers
    // every wave claims units until none is left (a bounded loop: no wave
    // waits for another, and nothing in group_work synchronises across waves);
    // a unit's counters go to the workgroup's totals at once, so that none
    // stays live from one unit to the next
    while (true) {
        int i = 0;
        if (lane_id() == 0)
            i = __hip_atomic_fetch_add(&ul.next, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        i = uniform_int(rl_i(i, 0));
        if (i >= ul.n)
            break;
        const int un = uniform_int(ul.unit[i]);
        const int64_t g = (int64_t)blockIdx.x * NW + (un & 0xff);
        int32_t st[NSTAT] = {}; // one group's counts fit 32 bits (at most 512 points x 256 candidates)
        group_work<D>(g, (un >> 8) & 0xff, un >> 16, A, wsh[wv], st);
        combine_add(bc, st);
    }
    const int32_t none[NSTAT] = {};
    combine_end(bc, A, none, blockIdx.x);
}

// k_assign_heavy: the leaves k_assign_waves deferred (a list of
// heavy_cnt leaf ids), one workgroup per leaf: wave 0 searches the tree for
// the leaf box (larger LDS capacities) into the workgroup's LDS, every wave
// holds the leaf's points and scans a quarter of the candidate chunks, the
// four partial (best, second) results meet in LDS and wave 0 finishes the
// decision (recheck, moves of the exact sums).  A leaf whose list still
// does not fit scans all k.  Such leaves sit where many centroids crowd near
// a large sparse cell.  The barriers sit in a loop whose trip count is the
// same for every wave of the workgroup.
struct HeavyShared {
    WaveHeavy ws;
    uint64_t key[G_WAVES][WAVE]; // FP32 (value, id) keys; FP64 distance bits in the recheck
    float s2[G_WAVES][WAVE];
    int32_t id64[G_WAVES][WAVE];
    int sn;
};

// FP32 best and second best of a point over centroids [j0, j1) of c32,
// 64 at a time (the next chunk loaded while this one is scanned).
template <int D>
__device__ inline Best2 scan_range(const float (&x)[D], const AssignArgs &A, int64_t j0, int64_t j1)
{
    const int lane = lane_id();
    Best2 bs[SCAN_ILP];
#pragma unroll
    for (int u = 0; u < SCAN_ILP; ++u)
        bs[u] = best2_init();
    float4 cur = j0 + lane < j1 ? A.c32[j0 + lane] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int64_t c = j0; c < j1; c += WAVE) {
        const int64_t jn = c + WAVE + lane;
        const float4 nxt = jn < j1 ? A.c32[jn] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const int cn = (int)(j1 - c < WAVE ? j1 - c : WAVE);
        for (int b0 = 0; b0 < cn; b0 += SCAN_ILP) {
#pragma unroll
            for (int u = 0; u < SCAN_ILP; ++u) {
                const int b = b0 + u;
                if (b < cn) {
                    float cc[3] = {rl_f(cur.x, b), rl_f(cur.y, b), D == 3 ? rl_f(cur.z, b) : 0.0f};
                    best2_add(bs[u], sqdist32<D>(x, cc), (int)(c + b));
                }
            }
        }
        cur = nxt;
    }
#pragma unroll
    for (int u = 1; u < SCAN_ILP; ++u)
        bs[0] = best2_merge(bs[0], bs[u]);
    return bs[0];
}

// The FP64 recheck over centroids [j0, j1): the canonical FP64 argmin
// (value, lowest id) among the centroids whose FP32 distance is at most T
// (every other one is strictly farther than the FP32 best, see lo_inverse),
// for lanes with `re`.
template <int D>
__device__ inline void recheck_range(const float (&x)[D], bool re, float T, const AssignArgs &A, int64_t j0,
                                     int64_t j1, double &bd, int &bj)
{
    const int lane = lane_id();
    double xd[D];
    for (int i = 0; i < D; ++i)
        xd[i] = (double)x[i];
    bd = INFINITY;
    bj = 0x7fffffff;
    for (int64_t c = j0; c < j1; c += WAVE) {
        const float4 cur = c + lane < j1 ? A.c32[c + lane] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const int cn = (int)(j1 - c < WAVE ? j1 - c : WAVE);
        for (int b = 0; b < cn; ++b) {
            float cc[3] = {rl_f(cur.x, b), rl_f(cur.y, b), D == 3 ? rl_f(cur.z, b) : 0.0f};
            if (re && sqdist32<D>(x, cc) <= T) {
                const double Dv = sqdist64<D>(xd, A.c_in + (c + b) * D);
                if (Dv < bd) { // ids increase: the lowest one wins a tie
                    bd = Dv;
                    bj = (int)(c + b);
                }
            }
        }
    }
}

template <int D>
__global__ void __launch_bounds__(ASSIGN_THREADS) k_assign_heavy(AssignArgs A)
{
    if (A.ctl[CTL_STOP] || *A.heavy_cnt == 0)
        return; // the run is over, or no leaf was deferred (the finalize kernel then skips these rows)
    __shared__ HeavyShared hs;
    __shared__ BlockCombine bc;
    combine_init(bc);
    const int w = uniform_int(threadIdx.x / WAVE), lane = lane_id();
    const float e = err_bound(A.cmax_bits);
    int64_t tot[NSTAT] = {}; // the workgroup's leaves; st: one leaf's counts (at most 64 points x 2^20 centroids)
    const int cnt = uniform_int(*A.heavy_cnt);
    for (int i = blockIdx.x; i < cnt; i += gridDim.x) {
        int32_t st[NSTAT] = {};
        const LeafJob J = job_load<D>(A, A.heavy[i]);
        const TreeArgs *Tp = A.trees + A.leaf_cloud[J.l];
        if (w == 0) {
            const int sn =
                wave_search<D>(J.lo, J.hi, Tp, e, hs.ws, A.sw_heavy, A.fr_heavy, prune_threshold_r(J.R, e));
            if (lane == 0)
                hs.sn = sn;
        }
        __syncthreads();
        const int sn = uniform_int(hs.sn);
        float thr = 0.0f, U = 0.0f;
        int j1 = -1, m = 0;
        if (sn >= 0) // every wave: the same m
            m = leaf_filter<D>(J.lo, J.hi, sn, e, hs.ws, prune_threshold_r(J.R, e), thr, j1, U);
        if (m >= 2) {
            const LeafPts<D> P = load_pts<D>(A, J);
            const Best2 b = scan_list<D>(P.x, J.lo, J.hi, thr, sn, hs.ws, w, G_WAVES);
            hs.key[w][lane] = b.key;
            hs.s2[w][lane] = b.s2;
            __syncthreads();
            if (w == 0) {
                Best2 t = b;
                for (int u = 1; u < G_WAVES; ++u)
                    t = best2_merge(t, Best2{hs.key[u][lane], hs.s2[u][lane]});
                st[ST_CANDS] += m;
                decide_points<D>(A, J, P, e, m,
                                 [&](const float (&x)[D], bool need, float &s1) {
                                     return finish_point<D>(x, need, t, J.lo, J.hi, thr, sn, e, A, hs.ws, st, s1);
                                 },
                                 st);
            }
        } else if (sn < 0 || m == 0) {
            // no list: every point scans all of its cloud's centroids, each
            // wave a quarter, FP32 first, then the FP64 recheck where the
            // merged margin asks for it
            const LeafPts<D> P = load_pts<D>(A, J);
            const int64_t c0 = Tp->c0, kk = Tp->k;
            const int64_t q0 = c0 + kk * w / G_WAVES, q1 = c0 + kk * (w + 1) / G_WAVES;
            const Best2 b = scan_range<D>(P.x, A, q0, q1);
            hs.key[w][lane] = b.key;
            hs.s2[w][lane] = b.s2;
            __syncthreads();
            Best2 t = Best2{hs.key[0][lane], hs.s2[0][lane]};
            for (int u = 1; u < G_WAVES; ++u)
                t = best2_merge(t, Best2{hs.key[u][lane], hs.s2[u][lane]});
            const float s1 = best2_s1(t);
            const bool re = lane < J.size && !margin_safe(s1, t.s2, e);
            __syncthreads(); // every wave has read the keys
            int best64 = -1;
            if (uniform_int(wave_count(re)) > 0) { // the same points in every wave
                double bd;
                int bj;
                recheck_range<D>(P.x, re, lo_inverse(dist_hi(s1, e), e), A, q0, q1, bd, bj);
                hs.key[w][lane] = (uint64_t)__double_as_longlong(bd); // non-negative: bits order like values
                hs.id64[w][lane] = bj;
                __syncthreads();
                uint64_t kb = hs.key[0][lane];
                int jb = hs.id64[0][lane];
                for (int u = 1; u < G_WAVES; ++u) {
                    const uint64_t ku = hs.key[u][lane];
                    const int ju = hs.id64[u][lane];
                    if (ku < kb || (ku == kb && ju < jb)) {
                        kb = ku;
                        jb = ju;
                    }
                }
                best64 = jb;
            }
            if (w == 0)
                decide_points<D>(A, J, P, e, kk,
                                 [&](const float (&x)[D], bool need, float &s1o) {
                                     s1o = s1;
                                     st[ST_RECHECK] += wave_count(need && re);
                                     st[ST_FALLBACK_PTS] += wave_count(need);
                                     return re ? best64 : best2_id(t);
                                 },
                                 st);
        } else if (w == 0) {
            const LeafPts<D> P = load_pts<D>(A, J);
            leaf_listed<D>(A, J, m, j1, thr, U, sn, e, hs.ws, P, st);
        }
#pragma unroll
        for (int q = 0; q < NSTAT; ++q)
            tot[q] += st[q];
        __syncthreads(); // the workgroup's LDS is free for the next leaf
    }
    combine_end(bc, A, tot, A.assign_wg + blockIdx.x);
}

// ------------------------------------------------------------- brute force
// Record the new assignment, count changes, add the point to its cluster's
// exact fixed-point sum (the brute path sums every cluster afresh).
template <int D, class TV>
__device__ inline void finish_point(const AssignArgs &A, bool valid, int64_t p, const TV (&x)[D], int best,
                                    int64_t &changed)
{
    if (valid) {
        int old = A.a[p];
        if (old != best) {
            A.a[p] = best;
            ++changed;
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
__global__ void __launch_bounds__(ASSIGN_THREADS) k_assign_brute32(AssignArgs A)
{
    if (A.ctl[CTL_STOP])
        return; // the run is over (the whole workgroup returns)
    __shared__ BlockStats bs;
    extern __shared__ float4 tile[];
    stats_begin(bs);
    int64_t st[NSTAT] = {};
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
        best = brute64_all<D>(xd, A, 0, A.k);
    }
    st[ST_RECHECK] += re ? 1 : 0;
    st[ST_EVALS] += valid ? A.k : 0;
    int64_t ch = 0;
    finish_point<D, float>(A, valid, p, x, best, ch);
    st[ST_CHANGED] += ch;
    stats_end(bs, A, st, blockIdx.x);
}

template <int D>
__global__ void __launch_bounds__(ASSIGN_THREADS) k_assign_brute64(AssignArgs A)
{
    if (A.ctl[CTL_STOP])
        return; // the run is over (the whole workgroup returns)
    __shared__ BlockStats bs;
    extern __shared__ double dtile[];
    stats_begin(bs);
    int64_t st[NSTAT] = {};
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
    finish_point<D, double>(A, valid, p, x, bj, ch);
    st[ST_CHANGED] += ch;
    stats_end(bs, A, st, blockIdx.x);
}

// ------------------------------------------------------------- objective
// SSE of the step (Eq. (1)'s objective against the centroids assigned to):
// block b sums the canonical D64 of points [b * SSE_CHUNK, (b + 1) *
// SSE_CHUNK) in a fixed order, so the value does not depend on scheduling.
constexpr int SSE_THREADS = 256;
constexpr int SSE_CHUNK = SSE_THREADS * 16;

int64_t sse_blocks(int64_t n) { return (n + SSE_CHUNK - 1) / SSE_CHUNK; }

template <class T, int D>
__global__ void __launch_bounds__(SSE_THREADS) k_sse(const T *xs, const int32_t *a, const double *c, int64_t n,
                                                     double *part, const int32_t *ctl)
{
    if (ctl[CTL_STOP])
        return;
    __shared__ double red[SSE_THREADS];
    const int64_t p0 = (int64_t)blockIdx.x * SSE_CHUNK;
    double s = 0.0;
    for (int q = 0; q < SSE_CHUNK / SSE_THREADS; ++q) {
        const int64_t p = p0 + (int64_t)q * SSE_THREADS + threadIdx.x;
        if (p < n) {
            double xd[D], cd[D];
            const int j = a[p];
            for (int i = 0; i < D; ++i) {
                xd[i] = (double)xs[(int64_t)i * n + p];
                cd[i] = c[(int64_t)j * D + i];
            }
            s += sqdist64<D>(xd, cd);
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = SSE_THREADS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        part[blockIdx.x] = red[0];
}

km_status run_sse(km_ctx *ctx, const double *c_in)
{
    const unsigned nb = (unsigned)sse_blocks(ctx->n);
    hipStream_t st = ctx->stream;
    const bool f32 = ctx->cfg.point_dtype == KM_F32;
    if (ctx->d == 2) {
        if (f32)
            hipLaunchKernelGGL((k_sse<float, 2>), dim3(nb), dim3(SSE_THREADS), 0, st, (const float *)ctx->xs, ctx->a,
                               c_in, ctx->n, ctx->sse_part, ctx->ctl);
        else
            hipLaunchKernelGGL((k_sse<double, 2>), dim3(nb), dim3(SSE_THREADS), 0, st, (const double *)ctx->xs,
                               ctx->a, c_in, ctx->n, ctx->sse_part, ctx->ctl);
    } else {
        if (f32)
            hipLaunchKernelGGL((k_sse<float, 3>), dim3(nb), dim3(SSE_THREADS), 0, st, (const float *)ctx->xs, ctx->a,
                               c_in, ctx->n, ctx->sse_part, ctx->ctl);
        else
            hipLaunchKernelGGL((k_sse<double, 3>), dim3(nb), dim3(SSE_THREADS), 0, st, (const double *)ctx->xs,
                               ctx->a, c_in, ctx->n, ctx->sse_part, ctx->ctl);
    }
    return hip_ok(hipGetLastError(), "objective launch") ? KM_OK : KM_ERR_HIP;
}

// ------------------------------------------------------------- driver
int64_t assign_grid(km_ctx *ctx);

static AssignArgs make_args(km_ctx *ctx, const double *c_in)
{
    AssignArgs A;
    A.xs = ctx->xs;
    A.n = ctx->n;
    A.k = ctx->k;
    A.a = ctx->a;
    A.c_in = c_in;
    A.c32 = ctx->c32;
    A.cmax_bits = (const unsigned *)ctx->cerr;
    A.cb_s = (const float *)ctx->cb_s;
    A.leaf_start = ctx->leaf_start;
    A.L = ctx->L;
    A.leaf_box = (const float4 *)ctx->leaf_box;
    A.leaf_sum = ctx->leaf_sum;
    A.leaf_own = ctx->leaf_own;
    A.leaf_r = ctx->leaf_r;
    A.drift_max = ctx->drift_max;
    A.heavy = ctx->heavy;
    A.heavy_cnt = ctx->heavy_cnt;
    A.assign_wg = assign_grid(ctx);
    A.group_leaf = ctx->group_leaf;
    A.group_box = ctx->group_box;
    A.ngroups = ctx->ngroups;
    A.trees = ctx->trees;
    A.group_cloud = ctx->group_cloud;
    A.leaf_cloud = ctx->leaf_cloud;
    A.S = ctx->S;
    A.fix64 = ctx->fix64;
    A.acc = ctx->acc;
    A.cnt = ctx->cnt;
    A.stat_part = ctx->stat_part;
    A.tile = ctx->tile;
    A.ctl = ctx->ctl;
    if (ctx->small_lists) { // tiny capacities: every fallback path runs (tests)
        A.sw_main = 16;
        A.fr_main = 64;
        A.sw_heavy = 32;
        A.fr_heavy = 128;
        A.heavy_m = 2;
        A.split_sn = 1; // every group with two leaves to decide is split from its second step
    } else {
        A.sw_main = SW_MAIN;
        A.fr_main = FR_MAIN;
        A.sw_heavy = SW_HEAVY;
        A.fr_heavy = FR_HEAVY;
        A.heavy_m = HEAVY_M;
        A.split_sn = SPLIT_SN;
    }
    A.group_parts = ctx->group_parts;
    return A;
}

// Workgroups of the indexed main pass (one wave per group).
int64_t assign_grid(km_ctx *ctx)
{
    const int w = main_waves(ctx->d);
    return (ctx->ngroups + w - 1) / w;
}

// Rows of per-block (brute) or per-workgroup (indexed) statistics partials.
int64_t assign_blocks(km_ctx *ctx)
{
    if (ctx->cfg.algo == KM_INDEXED)
        return assign_grid(ctx) + ctx->heavy_wgs;
    return (ctx->n + ASSIGN_THREADS - 1) / ASSIGN_THREADS;
}

// Launches the assignment passes; `between` (may be null) is recorded between
// the main pass and the per-leaf pass.
km_status run_assign(km_ctx *ctx, const double *c_in, hipEvent_t between)
{
    hipStream_t st = ctx->stream;
    AssignArgs A = make_args(ctx, c_in);
    unsigned nb = (unsigned)assign_blocks(ctx);
    const unsigned nwg = ctx->cfg.algo == KM_INDEXED ? (unsigned)assign_grid(ctx) : 0u;
    const int D = ctx->d;
    if (ctx->cfg.algo == KM_INDEXED) {
        const unsigned nhw = (unsigned)ctx->heavy_wgs;
        if (D == 2)
            hipLaunchKernelGGL(k_assign_waves<2>, dim3(nwg), dim3(MAIN_WAVES<2> * WAVE), 0, st, A);
        else
            hipLaunchKernelGGL(k_assign_waves<3>, dim3(nwg), dim3(MAIN_WAVES<3> * WAVE), 0, st, A);
        if (between)
            hipEventRecord(between, st);
        if (D == 2)
            hipLaunchKernelGGL(k_assign_heavy<2>, dim3(nhw), dim3(ASSIGN_THREADS), 0, st, A);
        else
            hipLaunchKernelGGL(k_assign_heavy<3>, dim3(nhw), dim3(ASSIGN_THREADS), 0, st, A);
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
    if (ctx->cfg.algo != KM_INDEXED && between)
        hipEventRecord(between, st);
    if (!hip_ok(hipGetLastError(), "assign launch"))
        return KM_ERR_HIP;
    return KM_OK;
}

} // namespace ekm
