// Assignment step (Algorithm 1's Assign over the point index, with the kNN
// search over the centroid index), fused with the accumulation half of the
// centroid update.
//
//  k_leaf_candidates  one thread per leaf: walk the centroid tree twice.
//     Pass 1 finds U, the smallest FP32 max-distance from the leaf box to a
//     centroid (nodes are skipped when their min-distance cannot beat the
//     current U; node max-distances tighten U early, as the paper inherits
//     upper bounds from parent nodes, Eq. (7)).  Pass 2 lists every centroid
//     whose min-distance to the box is within prune_threshold(U): all others
//     are strictly farther than the U-centroid from every point of the leaf
//     (the node pruning of Eq. (8), made conservative for rounding).
//  k_assign_indexed   one wave per leaf.  One candidate: the whole leaf goes
//     to it without a distance evaluation (Eq. (6)'s batch assignment), and
//     the leaf's precomputed exact sum goes to that cluster.  Otherwise each
//     lane scans the candidates in FP32; a point whose best-vs-second margin
//     is below the error bound is decided again with canonical FP64
//     distances.  Leaves with more than CAND_CAP candidates fall back to a
//     per-point tree search (the paper's per-point kNN with k = 1).
//  k_assign_brute32 / k_assign_brute64   Lloyd's assignment over all k
//     centroids staged through LDS tiles (the GPU baseline; FP64 is the
//     plain canonical computation).
#include "ekm_internal.hpp"

namespace ekm {

constexpr int ASSIGN_THREADS = 256;
constexpr int STACK_DEPTH = 20; // >= tree height + 2 for k <= 2^20
constexpr int PT_CAP = 8;       // per-point candidate list in the overflow path

struct AssignArgs {
    const void *xs;          // [d][n] Morton order
    int64_t n, k;
    int32_t *a;              // [n]
    const double *c_in;      // [k][d]
    const float4 *c32;       // [k]
    const unsigned *cmax_bits;
    // leaves
    const int32_t *leaf_start;
    int64_t L;
    const float4 *leaf_box;
    const int64_t *leaf_sum;
    int32_t *leaf_prev;
    int32_t *cand;
    int32_t *ncand;
    // centroid tree
    const float4 *cs;
    const float4 *node_lo, *node_hi;
    int tree_h;
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

// Depth-first walk of the implicit centroid tree for the box [lo, hi].
// COLLECT = false: tighten U (returns the number of centroids examined).
// COLLECT = true:  list centroids with min-distance <= T (returns the count,
// stores at most cap ids).  stack: this thread's LDS stack, stride apart.
template <int D, bool COLLECT>
__device__ int tree_walk(const float *lo, const float *hi, const AssignArgs &A, float &U, float T, int *out, int cap,
                         int *stack, int stride)
{
    const int64_t nleaf = (int64_t)1 << A.tree_h;
    int sp = 0;
    stack[0] = 1;
    sp = 1;
    int found = 0;
    if (!COLLECT) {
        float nl[3], nh[3];
        f4_to(A.node_lo[1], nl);
        f4_to(A.node_hi[1], nh);
        U = fminf(U, bb_maxd<D>(lo, hi, nl, nh));
    }
    while (sp > 0) {
        int v = stack[(--sp) * stride];
        if (v >= nleaf) {
            int64_t b = v - nleaf;
            int64_t t0 = b * TREE_BUCKET, t1 = t0 + TREE_BUCKET;
            if (t1 > A.k)
                t1 = A.k;
            for (int64_t t = t0; t < t1; ++t) {
                float4 c4 = A.cs[t];
                float c[3];
                f4_to(c4, c);
                if (!COLLECT) {
                    U = fminf(U, box_maxd<D>(lo, hi, c));
                    ++found;
                } else if (box_mind<D>(lo, hi, c) <= T) {
                    if (found < cap)
                        out[found] = __float_as_int(c4.w);
                    ++found;
                }
            }
            continue;
        }
        float l0[3], h0[3], l1[3], h1[3];
        f4_to(A.node_lo[2 * v], l0);
        f4_to(A.node_hi[2 * v], h0);
        f4_to(A.node_lo[2 * v + 1], l1);
        f4_to(A.node_hi[2 * v + 1], h1);
        float m0 = bb_mind<D>(lo, hi, l0, h0), m1 = bb_mind<D>(lo, hi, l1, h1);
        bool k0, k1;
        if (!COLLECT) {
            U = fminf(U, fminf(bb_maxd<D>(lo, hi, l0, h0), bb_maxd<D>(lo, hi, l1, h1)));
            k0 = m0 < U;
            k1 = m1 < U;
        } else {
            k0 = m0 <= T;
            k1 = m1 <= T;
        }
        // push the farther child first so the nearer one is visited next
        int nearc = m0 <= m1 ? 2 * v : 2 * v + 1, farc = nearc ^ 1;
        bool knear = m0 <= m1 ? k0 : k1, kfar = m0 <= m1 ? k1 : k0;
        if (kfar)
            stack[(sp++) * stride] = farc;
        if (knear)
            stack[(sp++) * stride] = nearc;
    }
    return found;
}

// One thread per leaf.
template <int D>
__global__ void __launch_bounds__(ASSIGN_THREADS) k_leaf_candidates(AssignArgs A)
{
    __shared__ int stack_mem[STACK_DEPTH * ASSIGN_THREADS];
    int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= A.L)
        return;
    float lo[3], hi[3];
    f4_to(A.leaf_box[2 * l], lo);
    f4_to(A.leaf_box[2 * l + 1], hi);
    float e = err_bound(A.cmax_bits);
    float U = INFINITY;
    int *stack = stack_mem + threadIdx.x;
    tree_walk<D, false>(lo, hi, A, U, 0.0f, nullptr, 0, stack, ASSIGN_THREADS);
    float T = prune_threshold(U, e);
    int m = tree_walk<D, true>(lo, hi, A, U, T, A.cand + l * CAND_CAP, CAND_CAP, stack, ASSIGN_THREADS);
    A.ncand[l] = m;
}

// --------------------------------------------------------------- epilogue
// Shared tail of every assignment kernel: record the new assignment, count
// changes, and add each point to its cluster's exact fixed-point sum.
template <int D, class T>
__device__ inline void finish_point(const AssignArgs &A, bool valid, int64_t p, const T (&x)[D], int best,
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
        if (sizeof(T) == 4)
            fix_split_f32((float)x[i], A.S, hi[i], lo[i]);
        else
            fix_split_f64((double)x[i], A.S, hi[i], lo[i]);
    }
    wave_accumulate<D>(valid, best, hi, lo, A.acc, A.cnt);
}

struct BlockStats {
    long long v[NSTAT];
    double sse[ASSIGN_THREADS / WAVE];
};

__device__ inline void stats_begin(BlockStats &bs)
{
    if (threadIdx.x < NSTAT)
        bs.v[threadIdx.x] = 0;
    if (threadIdx.x < ASSIGN_THREADS / WAVE)
        bs.sse[threadIdx.x] = 0.0;
    __syncthreads();
}
// per-thread counters -> block partial row (fixed-order FP64 for the SSE)
__device__ inline void stats_end(BlockStats &bs, const AssignArgs &A, const int64_t (&c)[NSTAT], double sse)
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
        A.stat_part[(int64_t)blockIdx.x * NSTAT + threadIdx.x] = bs.v[threadIdx.x];
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < ASSIGN_THREADS / WAVE; ++w)
            s += bs.sse[w];
        A.sse_part[blockIdx.x] = s;
    }
}

// ------------------------------------------------------------- indexed
// Canonical FP64 argmin (lowest index on ties) over a list of centroid ids.
template <int D>
__device__ inline int brute64_all(const double (&xd)[D], const AssignArgs &A);

template <int D>
__device__ inline int recheck64(const double (&xd)[D], const AssignArgs &A, const int32_t *ids, int m)
{
    if (m <= 0) // cannot happen for a well-formed tree; never return an invalid id
        return brute64_all<D>(xd, A);
    double best = INFINITY;
    int bj = 0x7fffffff;
    for (int t = 0; t < m; ++t) {
        int j = ids[t];
        double Dv = sqdist64<D>(xd, A.c_in + (int64_t)j * D);
        if (Dv < best || (Dv == best && j < bj)) {
            best = Dv;
            bj = j;
        }
    }
    return bj;
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
__global__ void __launch_bounds__(ASSIGN_THREADS) k_assign_indexed(AssignArgs A)
{
    __shared__ BlockStats bs;
    __shared__ int stack_mem[STACK_DEPTH * ASSIGN_THREADS];
    __shared__ int ptc_mem[PT_CAP * ASSIGN_THREADS];
    stats_begin(bs);
    int64_t st[NSTAT] = {0, 0, 0, 0, 0, 0, 0, 0};
    double sse = 0.0;
    const int lane = lane_id();
    const int64_t l = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const float *xs = (const float *)A.xs;
    if (l < A.L) { // uniform per wave
        const int32_t s = A.leaf_start[l], size = A.leaf_start[l + 1] - s;
        const int m = A.ncand[l];
        const bool valid = lane < size;
        const int64_t p = (int64_t)s + lane;
        const float e = err_bound(A.cmax_bits);
        if (m == 1) {
            const int j = A.cand[l * CAND_CAP];
            const int prev = A.leaf_prev[l];
            if (prev != j) {
                if (valid) {
                    if (A.a[p] != j) {
                        A.a[p] = j;
                        ++st[ST_CHANGED];
                    }
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
                st[ST_CANDS] += 1;
            }
            if (A.want_sse && valid) {
                double xd[D], cd[D];
                for (int i = 0; i < D; ++i) {
                    xd[i] = (double)xs[(int64_t)i * A.n + p];
                    cd[i] = A.c_in[(int64_t)j * D + i];
                }
                sse += sqdist64<D>(xd, cd);
            }
        } else {
            if (lane == 0 && A.leaf_prev[l] != -1)
                A.leaf_prev[l] = -1;
            float x[D];
            for (int i = 0; i < D; ++i)
                x[i] = valid ? xs[(int64_t)i * A.n + p] : 0.0f;
            int best = 0;
            if (m >= 1 && m <= CAND_CAP) {
                // lane t holds candidate t; each lane scans all m in FP32
                int myid = lane < m ? A.cand[l * CAND_CAP + lane] : 0;
                float4 myc = A.c32[myid];
                float s1 = INFINITY, s2 = INFINITY;
                int id1 = 0x7fffffff;
                for (int t = 0; t < m; ++t) {
                    int cid = __builtin_amdgcn_readlane(myid, t);
                    float c[3];
                    c[0] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(myc.x), t));
                    c[1] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(myc.y), t));
                    c[2] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(myc.z), t));
                    float sv = sqdist32<D>(x, c);
                    if (sv < s1 || (sv == s1 && cid < id1)) {
                        s2 = s1;
                        s1 = sv;
                        id1 = cid;
                    } else {
                        s2 = fminf(s2, sv);
                    }
                }
                best = id1;
                bool re = valid && !margin_safe(s1, s2, e);
                if (re) {
                    double xd[D];
                    for (int i = 0; i < D; ++i)
                        xd[i] = (double)x[i];
                    best = recheck64<D>(xd, A, A.cand + l * CAND_CAP, m);
                }
                if (lane == 0) {
                    st[ST_EVALS] += (int64_t)m * size;
                    st[ST_CANDS] += m;
                }
                st[ST_RECHECK] += re ? 1 : 0;
            } else {
                // too many candidates for the leaf box: search per point
                int *stack = stack_mem + threadIdx.x;
                int *ids = ptc_mem + threadIdx.x * PT_CAP;
                if (valid) {
                    float U = INFINITY;
                    int seen = tree_walk<D, false>(x, x, A, U, 0.0f, nullptr, 0, stack, ASSIGN_THREADS);
                    float T = prune_threshold(U, e);
                    int cnt = tree_walk<D, true>(x, x, A, U, T, ids, PT_CAP, stack, ASSIGN_THREADS);
                    st[ST_EVALS] += seen;
                    if (cnt == 1) {
                        best = ids[0];
                    } else {
                        double xd[D];
                        for (int i = 0; i < D; ++i)
                            xd[i] = (double)x[i];
                        best = cnt <= PT_CAP ? recheck64<D>(xd, A, ids, cnt) : brute64_all<D>(xd, A);
                        ++st[ST_RECHECK];
                    }
                    ++st[ST_OVERFLOW_PTS];
                }
                if (lane == 0)
                    st[ST_CANDS] += m;
            }
            int64_t ch = 0;
            finish_point<D, float>(A, valid, p, x, best, ch, sse);
            st[ST_CHANGED] += ch;
        }
    }
    stats_end(bs, A, st, sse);
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
    stats_end(bs, A, st, sse);
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
    stats_end(bs, A, st, sse);
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
    A.cand = ctx->cand;
    A.ncand = ctx->ncand;
    A.cs = ctx->cs;
    A.node_lo = ctx->node_lo;
    A.node_hi = ctx->node_hi;
    A.tree_h = ctx->tree_h;
    A.S = ctx->S;
    A.acc = ctx->acc;
    A.cnt = ctx->cnt;
    A.stat_part = ctx->stat_part;
    A.sse_part = ctx->sse_part;
    A.want_sse = want_sse ? 1 : 0;
    A.tile = ctx->tile;
    return A;
}

int64_t assign_blocks(const km_ctx *ctx)
{
    if (ctx->cfg.algo == KM_INDEXED)
        return (ctx->L * WAVE + ASSIGN_THREADS - 1) / ASSIGN_THREADS;
    return (ctx->n + ASSIGN_THREADS - 1) / ASSIGN_THREADS;
}

km_status run_assign(km_ctx *ctx, const double *c_in, bool want_sse)
{
    hipStream_t st = ctx->stream;
    AssignArgs A = make_args(ctx, c_in, want_sse);
    unsigned nb = (unsigned)assign_blocks(ctx);
    const int D = ctx->d;
    if (ctx->cfg.algo == KM_INDEXED) {
        unsigned gl = (unsigned)((ctx->L + ASSIGN_THREADS - 1) / ASSIGN_THREADS);
        if (D == 2) {
            hipLaunchKernelGGL(k_leaf_candidates<2>, dim3(gl), dim3(ASSIGN_THREADS), 0, st, A);
            hipLaunchKernelGGL(k_assign_indexed<2>, dim3(nb), dim3(ASSIGN_THREADS), 0, st, A);
        } else {
            hipLaunchKernelGGL(k_leaf_candidates<3>, dim3(gl), dim3(ASSIGN_THREADS), 0, st, A);
            hipLaunchKernelGGL(k_assign_indexed<3>, dim3(nb), dim3(ASSIGN_THREADS), 0, st, A);
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
