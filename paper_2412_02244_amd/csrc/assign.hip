// Assignment step (Algorithm 1's Assign over the point index, with its kNN
// search over the centroid index), fused with the accumulation half of the
// centroid update.
//
// k_assign_groups: one workgroup per group of GROUP_LEAVES consecutive
// leaves (Morton order keeps them spatially close).
//
//  1. Group search.  For the group's bounding box B the workgroup descends
//     the 8-ary centroid tree level by level.  U is the smallest FP32
//     max-distance from B to a node or centroid seen so far: every node box
//     contains a centroid, so U bounds the distance from every point of B to
//     some centroid (the paper inherits such upper bounds from parent nodes,
//     Eq. (7)).  Nodes and centroids whose FP32 min-distance to B exceeds
//     prune_threshold(U) are dropped (the node pruning of Eq. (8), made
//     conservative for rounding).  The survivors form the group list S.
//  2. Leaf filter.  For a leaf box b inside B, the same rule applied to S
//     alone gives exactly the leaf's candidates over all k centroids: any
//     centroid outside S has min-distance to b at least its min-distance to
//     B, above prune_threshold(U_B) >= prune_threshold(U_b), while the
//     centroid that realised U_B is in S and bounds U_b.  One wave handles a
//     leaf; lanes test S in chunks of 64 and ballots give the candidate set.
//  3. A leaf with one candidate is assigned to it without a single distance
//     evaluation (Eq. (6)'s batch assignment) and adds its precomputed exact
//     sum to that cluster.  Otherwise each lane (one point) scans the
//     candidates in FP32; a point whose best-vs-second margin is below the
//     error bound is decided again with canonical FP64 distances.
//
// If S (or the descent frontier) does not fit in LDS, the group repeats the
// search leaf by leaf, and a leaf that still does not fit scans all k
// centroids; results are the same, only slower.
//
// k_assign_brute32 / k_assign_brute64: Lloyd's assignment over all k
// centroids staged through LDS tiles (the GPU baseline; FP64 is the plain
// canonical computation).
#include "ekm_internal.hpp"

namespace ekm {

constexpr int ASSIGN_THREADS = 256;
constexpr int G_WAVES = ASSIGN_THREADS / WAVE;
constexpr int LPW = GROUP_LEAVES / G_WAVES; // leaves per wave
constexpr int S_CAP = 1024;                 // group candidate list in LDS
constexpr int F_CAP = 1024;                 // descent frontier in LDS

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
    const float4 *group_box;
    int64_t ngroups;
    // centroid tree
    TreeArgs T;
    // update
    int S;
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

struct GroupShared {
    float4 sc[S_CAP];          // group candidate list: fl32 coordinates, w = centroid id
    int front[2][F_CAP];       // descent frontier (node indices within a level)
    float fmind[F_CAP];        // min-distance of each evaluated entry
    // the group's leaves, loaded once per group (published by the search's barriers)
    float4 lbox[GROUP_LEAVES][2];
    int lstart[GROUP_LEAVES + 1];
    int lprev[GROUP_LEAVES];
    float red[G_WAVES];
    int count[2];
    int overflow;
    int gid;
    BlockStats bs;
};

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

// Block-wide minimum (all threads call; result returned to all).
__device__ inline float block_min(float v, float *red)
{
    v = wave_min_f32(v);
    __syncthreads(); // red may still be read by the previous call
    if (lane_id() == 0)
        red[threadIdx.x / WAVE] = v;
    __syncthreads();
    float m = red[0];
    for (int w = 1; w < G_WAVES; ++w)
        m = fminf(m, red[w]);
    return m;
}

// ------------------------------------------------------------- group search
// Fills sh.sc with the candidate list of box [lo, hi]; returns its length,
// or -1 if the frontier or the list would not fit.  All threads call.
template <int D>
__device__ int block_search(const float *lo, const float *hi, const AssignArgs &A, float e, GroupShared &sh)
{
    const TreeArgs &T = A.T;
    const int tid = threadIdx.x;
    float U = INFINITY;
    int level = T.start;
    int cur = 0;
    int F = (int)T.lev_size[level];
    __syncthreads(); // the previous search's readers are done with sh
    for (int i = tid; i < F; i += ASSIGN_THREADS)
        sh.front[cur][i] = i;
    if (tid == 0)
        sh.overflow = 0;
    __syncthreads();
    // internal levels and the bucket level
    while (true) {
        const int64_t off = T.lev_off[level];
        float Ul = INFINITY;
        for (int i = tid; i < F; i += ASSIGN_THREADS) {
            int64_t node = off + sh.front[cur][i];
            float nl[3], nh[3];
            f4_to(T.node_lo[node], nl);
            f4_to(T.node_hi[node], nh);
            sh.fmind[i] = bb_mind<D>(lo, hi, nl, nh);
            Ul = fminf(Ul, bb_maxd<D>(lo, hi, nl, nh));
        }
        U = fminf(U, block_min(Ul, sh.red));
        const float thr = prune_threshold(U, e);
        const int nxt = cur ^ 1;
        if (tid == 0)
            sh.count[nxt] = 0;
        __syncthreads();
        if (level > 0) {
            const int64_t csz = T.lev_size[level - 1];
            for (int i = tid; i < F; i += ASSIGN_THREADS) {
                if (sh.fmind[i] <= thr) {
                    int64_t first = 8 * (int64_t)sh.front[cur][i];
                    int nch = (int)((csz - first) < 8 ? (csz - first) : 8);
                    int pos = atomicAdd(&sh.count[nxt], nch);
                    if (pos + nch <= F_CAP) {
                        for (int c = 0; c < nch; ++c)
                            sh.front[nxt][pos + c] = (int)(first + c);
                    } else {
                        sh.overflow = 1;
                    }
                }
            }
        } else {
            // surviving buckets, kept as bucket indices
            for (int i = tid; i < F; i += ASSIGN_THREADS)
                if (sh.fmind[i] <= thr) {
                    int pos = atomicAdd(&sh.count[nxt], 1);
                    sh.front[nxt][pos] = sh.front[cur][i]; // pos < F <= F_CAP
                }
        }
        __syncthreads();
        if (uniform_int(sh.overflow))
            return -1;
        cur = nxt;
        F = uniform_int(sh.count[cur]);
        if (level == 0)
            break;
        --level;
    }
    // centroids of the surviving buckets
    const int nent = F * TREE_BUCKET;
    if (nent > F_CAP)
        return -1;
    float Ul = INFINITY;
    for (int i = tid; i < nent; i += ASSIGN_THREADS) {
        int64_t t = (int64_t)sh.front[cur][i / TREE_BUCKET] * TREE_BUCKET + (i % TREE_BUCKET);
        float m = INFINITY;
        if (t < A.k) {
            float c[3];
            f4_to(T.cs[t], c);
            m = box_mind<D>(lo, hi, c);
            Ul = fminf(Ul, box_maxd<D>(lo, hi, c));
        }
        sh.fmind[i] = m;
    }
    U = fminf(U, block_min(Ul, sh.red));
    const float thr = prune_threshold(U, e);
    if (tid == 0)
        sh.count[0] = 0;
    __syncthreads();
    for (int i = tid; i < nent; i += ASSIGN_THREADS) {
        if (sh.fmind[i] <= thr) {
            int64_t t = (int64_t)sh.front[cur][i / TREE_BUCKET] * TREE_BUCKET + (i % TREE_BUCKET);
            int pos = atomicAdd(&sh.count[0], 1);
            if (pos < S_CAP)
                sh.sc[pos] = T.cs[t];
            else
                sh.overflow = 1;
        }
    }
    __syncthreads();
    return uniform_int(sh.overflow) ? -1 : uniform_int(sh.count[0]);
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

template <int D>
__device__ void process_leaf_all(int64_t l, const AssignArgs &A, float e, int64_t (&st)[NSTAT], double &sse);

// ------------------------------------------------------------- leaves
// Candidate filter of one leaf against the group list (one wave): returns
// the candidate count and the first candidate's list index; the threshold
// is returned for the mask pass.
template <int D>
__device__ inline int leaf_filter(const float *blo, const float *bhi, int sn, float e, const GroupShared &sh,
                                  float &thr, int &first)
{
    const int lane = lane_id();
    const int nch = (sn + WAVE - 1) / WAVE;
    float U = INFINITY;
    for (int c = 0; c < nch; ++c) {
        int j = c * WAVE + lane;
        if (j < sn) {
            float cc[3];
            f4_to(sh.sc[j], cc);
            U = fminf(U, box_maxd<D>(blo, bhi, cc));
        }
    }
    thr = prune_threshold(wave_min_f32(U), e);
    int m = 0;
    first = -1;
    for (int c = 0; c < nch; ++c) {
        int j = c * WAVE + lane;
        bool keep = false;
        if (j < sn) {
            float cc[3];
            f4_to(sh.sc[j], cc);
            keep = box_mind<D>(blo, bhi, cc) <= thr;
        }
        unsigned long long mk = __ballot(keep);
        if (mk && first < 0)
            first = c * WAVE + __ffsll(mk) - 1;
        m += __popcll(mk);
    }
    return m;
}

// FP32 scan of one point (one lane) against the leaf's candidates: the list
// entries of the group list within `thr` of the leaf box.  The candidate
// masks are rebuilt chunk by chunk with ballots, so every lane holds them
// in registers (lanes never hand data to each other through LDS).  A point
// whose best-vs-second margin is below the error bound is decided again
// with canonical FP64 distances.  Returns the centroid id.
template <int D>
__device__ inline int assign_point(const float (&x)[D], bool valid, const float *blo, const float *bhi, float thr,
                                   int sn, float e, const AssignArgs &A, const GroupShared &sh,
                                   int64_t (&st)[NSTAT])
{
    const int lane = lane_id();
    const int nch = (sn + WAVE - 1) / WAVE;
    float s1 = INFINITY, s2 = INFINITY;
    int id1 = 0x7fffffff;
    for (int c = 0; c < nch; ++c) {
        const int jl = c * WAVE + lane;
        bool keep = false;
        if (jl < sn) {
            float cc[3];
            f4_to(sh.sc[jl], cc);
            keep = box_mind<D>(blo, bhi, cc) <= thr;
        }
        unsigned long long mk = __ballot(keep);
        while (mk) {
            int b = __ffsll(mk) - 1;
            mk &= mk - 1;
            float4 c4 = sh.sc[c * WAVE + b];
            float cc[3];
            f4_to(c4, cc);
            int cid = __float_as_int(c4.w);
            float sv = sqdist32<D>(x, cc);
            if (sv < s1 || (sv == s1 && cid < id1)) {
                s2 = s1;
                s1 = sv;
                id1 = cid;
            } else {
                s2 = fminf(s2, sv);
            }
        }
    }
    if (valid && !margin_safe(s1, s2, e)) {
        double xd[D];
        for (int i = 0; i < D; ++i)
            xd[i] = (double)x[i];
        double bd = INFINITY;
        int bj = 0x7fffffff;
        for (int j = 0; j < sn; ++j) {
            float4 c4 = sh.sc[j];
            float cc[3];
            f4_to(c4, cc);
            if (!(box_mind<D>(blo, bhi, cc) <= thr))
                continue;
            int cid = __float_as_int(c4.w);
            double Dv = sqdist64<D>(xd, A.c_in + (int64_t)cid * D);
            if (Dv < bd || (Dv == bd && cid < bj)) {
                bd = Dv;
                bj = cid;
            }
        }
        ++st[ST_RECHECK];
        return bj;
    }
    return id1;
}

// One wave: its LPW consecutive leaves of the group (leaf indices l0 + t).
// The candidate filters of all its leaves run first (LDS only); then the
// leaves are processed in order while the next leaf's points and previous
// assignments are already being loaded.
template <int D>
__device__ inline void load_leaf(int t, int m, int j1, const AssignArgs &A, const GroupShared &sh, float (&xv)[D],
                                 int &av)
{
    const int lane = lane_id();
    const float *xs = (const float *)A.xs;
    const int s = sh.lstart[t], size = sh.lstart[t + 1] - s;
    const int64_t p = (int64_t)s + lane;
    const bool valid = lane < size;
    const bool need_x = m != 1 || A.want_sse;
    const bool need_a = m != 1 || sh.lprev[t] != j1;
    av = -1;
    for (int i = 0; i < D; ++i)
        xv[i] = 0.0f;
    if (valid && need_x)
        for (int i = 0; i < D; ++i)
            xv[i] = xs[(int64_t)i * A.n + p];
    if (valid && need_a)
        av = A.a[p];
}

template <int D>
__device__ void process_wave_leaves(int64_t l0, int nl, int sn, const AssignArgs &A, float e, GroupShared &sh,
                                    int64_t (&st)[NSTAT], double &sse)
{
    const int lane = lane_id();
    const int tb = (threadIdx.x / WAVE) * LPW;
    const int te = (tb + LPW < nl) ? tb + LPW : nl;
    // filter every leaf first; lane r keeps leaf tb + r's results
    float r_thr = 0.0f;
    int r_m = 0, r_j = -1;
    for (int t = tb; t < te; ++t) {
        float blo[3], bhi[3];
        f4_to(sh.lbox[t][0], blo);
        f4_to(sh.lbox[t][1], bhi);
        float thr;
        int first;
        const int m = leaf_filter<D>(blo, bhi, sn, e, sh, thr, first);
        const int j1 = m == 1 ? __float_as_int(sh.sc[first].w) : -1;
        if (lane == t - tb) {
            r_thr = thr;
            r_m = m;
            r_j = j1;
        }
    }
    if (tb >= te)
        return;
    float xn[D];
    int an;
    load_leaf<D>(tb, __shfl(r_m, 0), __shfl(r_j, 0), A, sh, xn, an);
    for (int t = tb; t < te; ++t) {
        float x[D];
        for (int i = 0; i < D; ++i)
            x[i] = xn[i];
        const int aold = an;
        const int m = __shfl(r_m, t - tb), j1 = __shfl(r_j, t - tb);
        const float thr = __shfl(r_thr, t - tb);
        if (t + 1 < te)
            load_leaf<D>(t + 1, __shfl(r_m, t + 1 - tb), __shfl(r_j, t + 1 - tb), A, sh, xn, an);
        const int64_t l = l0 + t;
        const int s = sh.lstart[t], size = sh.lstart[t + 1] - s;
        const int64_t p = (int64_t)s + lane;
        const bool valid = lane < size;
        if (lane == 0)
            st[ST_CANDS] += m;
        if (m == 1) {
            const int j = j1;
            if (sh.lprev[t] != j) {
                if (valid && aold != j) {
                    A.a[p] = j;
                    ++st[ST_CHANGED];
                }
                if (lane == 0)
                    A.leaf_prev[l] = j;
            }
            if (lane == 0) {
                int64_t *ac = A.acc + (int64_t)j * D * 2;
                for (int i = 0; i < 2 * D; ++i)
                    atomicAdd((unsigned long long *)&ac[i], (unsigned long long)A.leaf_sum[l * D * 2 + i]);
                atomicAdd(&A.cnt[j], size);
                st[ST_SINGLE] += size;
            }
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
        if (m == 0) { // cannot happen for a well-formed tree; stay in bounds regardless
            process_leaf_all<D>(l, A, e, st, sse);
            continue;
        }
        if (lane == 0 && sh.lprev[t] != -1)
            A.leaf_prev[l] = -1;
        float blo[3], bhi[3];
        f4_to(sh.lbox[t][0], blo);
        f4_to(sh.lbox[t][1], bhi);
        const int best = assign_point<D>(x, valid, blo, bhi, thr, sn, e, A, sh, st);
        if (lane == 0)
            st[ST_EVALS] += (int64_t)m * size;
        if (valid && aold != best) {
            A.a[p] = best;
            ++st[ST_CHANGED];
        }
        if (A.want_sse && valid) {
            double xd[D], cd[D];
            for (int i = 0; i < D; ++i) {
                xd[i] = (double)x[i];
                cd[i] = A.c_in[(int64_t)best * D + i];
            }
            sse += sqdist64<D>(xd, cd);
        }
        int64_t hi[D], lo[D];
#pragma unroll
        for (int i = 0; i < D; ++i)
            fix_split_f32(x[i], A.S, hi[i], lo[i]);
        wave_accumulate<D>(valid, best, hi, lo, A.acc, A.cnt);
    }
}

// One wave, one leaf (the per-leaf fallback when the group list overflows).
template <int D>
__device__ void process_leaf(int64_t l, int sn, const AssignArgs &A, float e, GroupShared &sh,
                             int64_t (&st)[NSTAT], double &sse)
{
    const int lane = lane_id();
    const float *xs = (const float *)A.xs;
    const int32_t s = A.leaf_start[l], size = A.leaf_start[l + 1] - s;
    const bool valid = lane < size;
    const int64_t p = (int64_t)s + lane;
    float blo[3], bhi[3];
    f4_to(A.leaf_box[2 * l], blo);
    f4_to(A.leaf_box[2 * l + 1], bhi);
    float thr;
    int first;
    const int m = leaf_filter<D>(blo, bhi, sn, e, sh, thr, first);
    if (m == 0) {
        process_leaf_all<D>(l, A, e, st, sse);
        return;
    }
    if (lane == 0) {
        st[ST_CANDS] += m;
        st[ST_EVALS] += (int64_t)m * size;
        A.leaf_prev[l] = -1;
    }
    float x[D];
    for (int i = 0; i < D; ++i)
        x[i] = valid ? xs[(int64_t)i * A.n + p] : 0.0f;
    const int best = assign_point<D>(x, valid, blo, bhi, thr, sn, e, A, sh, st);
    int64_t ch = 0;
    finish_point<D, float>(A, valid, p, x, best, ch, sse);
    st[ST_CHANGED] += ch;
}

// Fallback for a leaf whose candidate list does not fit: scan all k
// centroids in FP32 (fl32 copies from global memory), same margin rule.
template <int D>
__device__ void process_leaf_all(int64_t l, const AssignArgs &A, float e, int64_t (&st)[NSTAT], double &sse)
{
    const int lane = lane_id();
    const float *xs = (const float *)A.xs;
    const int32_t s = A.leaf_start[l], size = A.leaf_start[l + 1] - s;
    const bool valid = lane < size;
    const int64_t p = (int64_t)s + lane;
    if (lane == 0 && A.leaf_prev[l] != -1)
        A.leaf_prev[l] = -1;
    float x[D];
    for (int i = 0; i < D; ++i)
        x[i] = valid ? xs[(int64_t)i * A.n + p] : 0.0f;
    float s1 = INFINITY, s2 = INFINITY;
    int id1 = 0;
    for (int64_t j = 0; j < A.k; ++j) {
        float cc[3];
        f4_to(A.c32[j], cc);
        float sv = sqdist32<D>(x, cc);
        if (sv < s1) {
            s2 = s1;
            s1 = sv;
            id1 = (int)j;
        } else {
            s2 = fminf(s2, sv);
        }
    }
    int best = id1;
    const bool re = valid && !margin_safe(s1, s2, e);
    if (re) {
        double xd[D];
        for (int i = 0; i < D; ++i)
            xd[i] = (double)x[i];
        best = brute64_all<D>(xd, A);
        ++st[ST_RECHECK];
    }
    if (valid) {
        st[ST_EVALS] += A.k;
        ++st[ST_FALLBACK_PTS];
    }
    int64_t ch = 0;
    finish_point<D, float>(A, valid, p, x, best, ch, sse);
    st[ST_CHANGED] += ch;
}

template <int D>
__global__ void __launch_bounds__(ASSIGN_THREADS, 4) k_assign_groups(AssignArgs A)
{
    __shared__ GroupShared sh;
    const int tid = threadIdx.x, wid = tid / WAVE;
    const float e = err_bound(A.cmax_bits);
    const int64_t g = blockIdx.x; // one group of leaves per workgroup
    if (tid < NSTAT)
        sh.bs.v[tid] = 0;
    if (tid < G_WAVES)
        sh.bs.sse[tid] = 0.0;
    int64_t st[NSTAT] = {0, 0, 0, 0, 0, 0, 0, 0};
    double sse = 0.0;
    const int64_t l0 = g * GROUP_LEAVES;
    const int nl = (int)((l0 + GROUP_LEAVES < A.L) ? GROUP_LEAVES : A.L - l0);
    if (tid < nl) {
        sh.lbox[tid][0] = A.leaf_box[2 * (l0 + tid)];
        sh.lbox[tid][1] = A.leaf_box[2 * (l0 + tid) + 1];
        sh.lprev[tid] = A.leaf_prev[l0 + tid];
    }
    if (tid <= nl)
        sh.lstart[tid] = A.leaf_start[l0 + tid];
    float glo[3], ghi[3];
    f4_to(A.group_box[2 * g], glo);
    f4_to(A.group_box[2 * g + 1], ghi);
    const int sn = block_search<D>(glo, ghi, A, e, sh); // its barriers publish the leaf data
    if (sn >= 0) {
        process_wave_leaves<D>(l0, nl, sn, A, e, sh, st, sse);
    } else {
        // the group's list does not fit: search leaf by leaf (uniform loop)
        for (int t = 0; t < nl; ++t) {
            const int64_t l = l0 + t;
            float blo[3], bhi[3];
            f4_to(A.leaf_box[2 * l], blo);
            f4_to(A.leaf_box[2 * l + 1], bhi);
            const int ln = block_search<D>(blo, bhi, A, e, sh);
            if (wid == 0) {
                if (ln >= 0)
                    process_leaf<D>(l, ln, A, e, sh, st, sse);
                else
                    process_leaf_all<D>(l, A, e, st, sse);
            }
        }
    }
    stats_end(sh.bs, A, st, sse, g);
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
    A.group_box = ctx->group_box;
    A.ngroups = ctx->ngroups;
    A.T = ctx->tree;
    A.S = ctx->S;
    A.acc = ctx->acc;
    A.cnt = ctx->cnt;
    A.stat_part = ctx->stat_part;
    A.sse_part = ctx->sse_part;
    A.want_sse = want_sse ? 1 : 0;
    A.tile = ctx->tile;
    return A;
}

// Rows of per-block (brute) or per-group (indexed) statistics partials.
int64_t assign_blocks(const km_ctx *ctx)
{
    if (ctx->cfg.algo == KM_INDEXED)
        return ctx->ngroups;
    return (ctx->n + ASSIGN_THREADS - 1) / ASSIGN_THREADS;
}

km_status run_assign(km_ctx *ctx, const double *c_in, bool want_sse)
{
    hipStream_t st = ctx->stream;
    AssignArgs A = make_args(ctx, c_in, want_sse);
    unsigned nb = (unsigned)assign_blocks(ctx);
    const int D = ctx->d;
    if (ctx->cfg.algo == KM_INDEXED) {
        if (D == 2)
            hipLaunchKernelGGL(k_assign_groups<2>, dim3(nb), dim3(ASSIGN_THREADS), 0, st, A);
        else
            hipLaunchKernelGGL(k_assign_groups<3>, dim3(nb), dim3(ASSIGN_THREADS), 0, st, A);
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
