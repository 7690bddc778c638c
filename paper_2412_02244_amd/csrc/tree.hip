// Centroid index, rebuilt from the current centroids every iteration
// (Algorithm 1 rebuilds its centroid tree at the top of each pass of the
// loop; node layout in the subsection on indexes over spatial vectors and
// centroids).
//
// GPU realisation: centroids are rounded to FP32, sorted along the Morton
// curve of the data grid (ties by index, stable radix sort), grouped into
// buckets of TREE_BUCKET consecutive centroids, and covered by an implicit
// 8-ary tree: level 0 holds the buckets, node i of level l covers nodes
// 8i..8i+7 of level l-1, and the top level is a single root.  Each node
// stores the exact FP32 bounding box of its centroids.  Cutting a
// Morton-sorted run into equal consecutive pieces splits space along the
// interleaved coordinates, i.e. kd-style splits, three levels at a time.
// A wide tree keeps the descent short: three levels cover k = 4096.
#include "ekm_internal.hpp"

namespace ekm {

constexpr int SMALL_K = 4096;
constexpr int TREE_THREADS = 1024;
constexpr int TREE_WAVES = TREE_THREADS / WAVE;

__device__ inline void box_empty(float4 &lo, float4 &hi)
{
    lo = make_float4(INFINITY, INFINITY, INFINITY, 0.0f);
    hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.0f);
}
__device__ inline void box_add(float4 &lo, float4 &hi, float4 p)
{
    lo.x = fminf(lo.x, p.x);
    lo.y = fminf(lo.y, p.y);
    lo.z = fminf(lo.z, p.z);
    hi.x = fmaxf(hi.x, p.x);
    hi.y = fmaxf(hi.y, p.y);
    hi.z = fmaxf(hi.z, p.z);
}
__device__ inline void box_union(float4 &lo, float4 &hi, float4 blo, float4 bhi)
{
    lo.x = fminf(lo.x, blo.x);
    lo.y = fminf(lo.y, blo.y);
    lo.z = fminf(lo.z, blo.z);
    hi.x = fmaxf(hi.x, bhi.x);
    hi.y = fmaxf(hi.y, bhi.y);
    hi.z = fmaxf(hi.z, bhi.z);
}

// fl32(c), its Morton key, and the norm bound used for ||c - fl32(c)|| <=
// 2^-24 ||c||.  The norm is rounded up to FP32.
template <int D>
__device__ inline float centroid_prep_one(const double *c, int64_t j, const Grid &g, float4 &q4, uint32_t &key)
{
    float q[3] = {0.0f, 0.0f, 0.0f};
    double s = 0.0;
    for (int i = 0; i < D; ++i) {
        double v = c[j * D + i];
        q[i] = (float)v;
        s += v * v;
    }
    q4 = make_float4(q[0], q[1], q[2], 0.0f);
    key = morton_key<D>(q, g);
    double nrm = sqrt(s) * (1.0 + 0x1p-40);
    float nb = (float)nrm;
    if ((double)nb < nrm)
        nb = nextafterf(nb, INFINITY);
    return nb;
}

// ------------------------------------------------------------------ small k
// Everything in one workgroup, LDS-resident after one read of the centroids:
// prep, stable LSD radix sort (8-bit digits) of the top 16 key bits, the
// tree-ordered copy and every node box; global memory is only written.
template <int D>
__global__ void __launch_bounds__(TREE_THREADS) k_tree_small(const double *c, int64_t k, Grid g, TreeArgs T,
                                                             float4 *c32, unsigned *cmax_bits)
{
    extern __shared__ unsigned char smem[];
    float4 *cq = (float4 *)smem;              // [SMALL_K] fl32 centroids, caller order
    uint32_t *key = (uint32_t *)(cq + SMALL_K); // [SMALL_K]
    uint32_t *id = key + SMALL_K;             // [SMALL_K]
    uint32_t *key2 = id + SMALL_K;            // [SMALL_K]
    uint32_t *id2 = key2 + SMALL_K;           // [SMALL_K]
    uint32_t *wcnt = id2 + SMALL_K;           // [TREE_WAVES][256]
    uint32_t *base = wcnt + TREE_WAVES * 256; // [256]
    __shared__ float red[TREE_WAVES];
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / WAVE;
    const int kk = (int)k;
    const int shift = key_bits(D) - 16; // sort on the top 16 bits
    float nb = 0.0f;
    for (int j = tid; j < kk; j += TREE_THREADS) {
        float4 q4;
        uint32_t kb;
        nb = fmaxf(nb, centroid_prep_one<D>(c, j, g, q4, kb));
        cq[j] = q4;
        c32[j] = q4;
        key[j] = kb >> shift;
        id[j] = (uint32_t)j;
    }
    nb = -wave_min_f32(-nb);
    if (lane == 0)
        red[wid] = nb;
    __syncthreads();
    if (tid == 0) {
        float m = 0.0f;
        for (int w = 0; w < TREE_WAVES; ++w)
            m = fmaxf(m, red[w]);
        *cmax_bits = __float_as_uint(m);
    }
    // two stable passes over 8-bit digits
    for (int pass = 0; pass < 2; ++pass) {
        const int sh = 8 * pass;
        uint32_t *kin = pass ? key2 : key, *vin = pass ? id2 : id;
        uint32_t *kout = pass ? key : key2, *vout = pass ? id : id2;
        if (tid < 256)
            base[tid] = 0;
        __syncthreads();
        for (int j = tid; j < kk; j += TREE_THREADS)
            atomicAdd(&base[(kin[j] >> sh) & 0xffu], 1u);
        __syncthreads();
        // exclusive scan of the 256 digit counts: 4 waves scan 64 each
        if (tid < 256) {
            uint32_t v = base[tid], x = v;
#pragma unroll
            for (int o = 1; o < WAVE; o <<= 1) {
                uint32_t y = __shfl_up(x, o);
                if (lane >= o)
                    x += y;
            }
            if (lane == WAVE - 1)
                wcnt[wid] = x; // wave totals (wcnt is free here)
            base[tid] = x - v;
        }
        __syncthreads();
        if (tid < 256) {
            uint32_t add = 0;
            for (int w = 0; w < wid; ++w)
                add += wcnt[w];
            base[tid] += add;
        }
        __syncthreads();
        for (int r0 = 0; r0 < kk; r0 += TREE_THREADS) {
            if (tid < 256)
                for (int w = 0; w < TREE_WAVES; ++w)
                    wcnt[w * 256 + tid] = 0;
            __syncthreads();
            int j = r0 + tid;
            bool valid = j < kk;
            uint32_t kv = valid ? kin[j] : 0u, vv = valid ? vin[j] : 0u;
            uint32_t dig = (kv >> sh) & 0xffu;
            uint64_t m = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                uint64_t bal = __ballot((dig >> b) & 1u);
                m &= ((dig >> b) & 1u) ? bal : ~bal;
            }
            int rank = __popcll(m & lanemask_lt());
            if (valid && rank == 0)
                wcnt[wid * 256 + dig] = (uint32_t)__popcll(m);
            __syncthreads();
            uint32_t pos = base[dig] + (uint32_t)rank;
            for (int w = 0; w < wid; ++w)
                pos += wcnt[w * 256 + dig];
            __syncthreads();
            if (tid < 256) {
                uint32_t add = 0;
                for (int w = 0; w < TREE_WAVES; ++w)
                    add += wcnt[w * 256 + tid];
                base[tid] += add;
            }
            if (valid) {
                kout[pos] = kv;
                vout[pos] = vv;
            }
            __syncthreads();
        }
    }
    // sorted ids are back in `id`; node boxes go to LDS (over key2/id2,
    // free now: at most 2 * SMALL_K / TREE_BUCKET float4 pairs) and out
    float4 *nlo = (float4 *)key2, *nhi = nlo + T.nnodes;
    for (int t = tid; t < kk; t += TREE_THREADS) {
        int cid = (int)id[t];
        float4 p = cq[cid];
        p.w = __int_as_float(cid);
        T.cs[t] = p;
    }
    const int nb0 = (int)T.lev_size[0];
    for (int b = tid; b < nb0; b += TREE_THREADS) {
        float4 lo, hi;
        box_empty(lo, hi);
        const int te = (b + 1) * TREE_BUCKET < kk ? (b + 1) * TREE_BUCKET : kk;
        for (int t = b * TREE_BUCKET; t < te; ++t)
            box_add(lo, hi, cq[id[t]]);
        nlo[b] = lo;
        nhi[b] = hi;
        T.node_lo[b] = lo;
        T.node_hi[b] = hi;
    }
    __syncthreads();
    for (int l = 1; l < T.nlev; ++l) {
        const int off = (int)T.lev_off[l], poff = (int)T.lev_off[l - 1], psz = (int)T.lev_size[l - 1];
        for (int i = tid; i < (int)T.lev_size[l]; i += TREE_THREADS) {
            float4 lo, hi;
            box_empty(lo, hi);
            const int ce = 8 * i + 8 < psz ? 8 * i + 8 : psz;
            for (int ch = 8 * i; ch < ce; ++ch)
                box_union(lo, hi, nlo[poff + ch], nhi[poff + ch]);
            nlo[off + i] = lo;
            nhi[off + i] = hi;
            T.node_lo[off + i] = lo;
            T.node_hi[off + i] = hi;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ large k
template <int D>
__global__ void __launch_bounds__(256) k_centroid_prep(const double *c, int64_t k, Grid g, float4 *c32,
                                                       uint32_t *keys, int32_t *vals, unsigned *cmax_bits)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float nb = 0.0f;
    if (j < k) {
        float4 q4;
        uint32_t kb;
        nb = centroid_prep_one<D>(c, j, g, q4, kb);
        c32[j] = q4;
        keys[j] = kb;
        vals[j] = (int32_t)j;
    }
    // non-negative floats order like their bit patterns
    float m = -wave_min_f32(-nb);
    if (lane_id() == 0)
        atomicMax(cmax_bits, __float_as_uint(m));
}

__global__ void __launch_bounds__(256) k_tree_buckets(const float4 *c32, const int32_t *sorted_id, int64_t k,
                                                      TreeArgs T)
{
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= T.lev_size[0])
        return;
    float4 lo, hi;
    box_empty(lo, hi);
    for (int64_t t = b * TREE_BUCKET; t < k && t < (b + 1) * TREE_BUCKET; ++t) {
        int id = sorted_id[t];
        float4 p = c32[id];
        box_add(lo, hi, p);
        p.w = __int_as_float(id);
        T.cs[t] = p;
    }
    T.node_lo[b] = lo;
    T.node_hi[b] = hi;
}

__global__ void __launch_bounds__(256) k_tree_level(TreeArgs T, int l)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= T.lev_size[l])
        return;
    const int64_t off = T.lev_off[l], poff = T.lev_off[l - 1], psz = T.lev_size[l - 1];
    float4 lo, hi;
    box_empty(lo, hi);
    for (int64_t ch = 8 * i; ch < 8 * i + 8 && ch < psz; ++ch)
        box_union(lo, hi, T.node_lo[poff + ch], T.node_hi[poff + ch]);
    T.node_lo[off + i] = lo;
    T.node_hi[off + i] = hi;
}

static size_t small_tree_lds()
{
    return (size_t)SMALL_K * 16 + (size_t)SMALL_K * 16 + (size_t)TREE_WAVES * 256 * 4 + 256 * 4;
}
// The node boxes of a k <= SMALL_K tree fit in the key2/id2 region.
static_assert(2 * (SMALL_K / TREE_BUCKET + SMALL_K / TREE_BUCKET / 7 + 8) * 16 <= SMALL_K * 8,
              "node boxes of the small tree fit in LDS");

km_status build_centroid_tree(km_ctx *ctx, const double *c_in)
{
    hipStream_t st = ctx->stream;
    const int64_t k = ctx->k;
    unsigned *cmax = (unsigned *)ctx->cerr;
    if (ctx->cfg.algo == KM_INDEXED && k <= SMALL_K) {
        if (ctx->d == 2)
            hipLaunchKernelGGL(k_tree_small<2>, dim3(1), dim3(TREE_THREADS), small_tree_lds(), st, c_in, k, ctx->grid,
                               ctx->tree, ctx->c32, cmax);
        else
            hipLaunchKernelGGL(k_tree_small<3>, dim3(1), dim3(TREE_THREADS), small_tree_lds(), st, c_in, k, ctx->grid,
                               ctx->tree, ctx->c32, cmax);
        return hip_ok(hipGetLastError(), "centroid tree launch") ? KM_OK : KM_ERR_HIP;
    }
    unsigned g = (unsigned)((k + 255) / 256);
    if (ctx->d == 2)
        hipLaunchKernelGGL(k_centroid_prep<2>, dim3(g), dim3(256), 0, st, c_in, k, ctx->grid, ctx->c32, ctx->ckey,
                           ctx->cval, cmax);
    else
        hipLaunchKernelGGL(k_centroid_prep<3>, dim3(g), dim3(256), 0, st, c_in, k, ctx->grid, ctx->c32, ctx->ckey,
                           ctx->cval, cmax);
    if (ctx->cfg.algo != KM_INDEXED) // the brute path needs only fl32(c) and the norm bound
        return hip_ok(hipGetLastError(), "centroid prep launch") ? KM_OK : KM_ERR_HIP;
    bool in_tmp = false;
    if (!hip_ok(radix_sort_u32(ctx->ckey, ctx->cval, ctx->ckey2, ctx->cval2, k, key_bits(ctx->d), ctx->rs_hist,
                               ctx->scan_tmp, st, &in_tmp),
                "centroid radix sort"))
        return KM_ERR_HIP;
    const int32_t *sid = in_tmp ? ctx->cval2 : ctx->cval;
    const TreeArgs &T = ctx->tree;
    hipLaunchKernelGGL(k_tree_buckets, dim3((unsigned)((T.lev_size[0] + 255) / 256)), dim3(256), 0, st, ctx->c32,
                       sid, k, T);
    for (int l = 1; l < T.nlev; ++l)
        hipLaunchKernelGGL(k_tree_level, dim3((unsigned)((T.lev_size[l] + 255) / 256)), dim3(256), 0, st, T, l);
    return hip_ok(hipGetLastError(), "centroid tree launch") ? KM_OK : KM_ERR_HIP;
}

// Allow the single-workgroup tree kernel its LDS budget.
hipError_t tree_setup()
{
    int need = (int)small_tree_lds();
    (void)hipFuncSetAttribute((const void *)k_tree_small<2>, hipFuncAttributeMaxDynamicSharedMemorySize, need);
    (void)hipFuncSetAttribute((const void *)k_tree_small<3>, hipFuncAttributeMaxDynamicSharedMemorySize, need);
    (void)hipGetLastError(); // a refusal shows up as a launch error of the tree kernel instead
    return hipSuccess;
}

// Level sizes of the 8-ary tree over ceil(k / TREE_BUCKET) buckets.
void tree_layout(int64_t k, TreeArgs &T)
{
    int64_t sz = (k + TREE_BUCKET - 1) / TREE_BUCKET, off = 0;
    T.nlev = 0;
    while (true) {
        T.lev_size[T.nlev] = sz;
        T.lev_off[T.nlev] = off;
        off += sz;
        ++T.nlev;
        if (sz == 1)
            break;
        sz = (sz + 7) / 8;
    }
    T.nnodes = off;
    // a descent starts at the lowest level small enough to evaluate every node
    T.start = T.nlev - 1;
    while (T.start > 0 && T.lev_size[T.start - 1] <= TREE_START_MAX)
        --T.start;
}

} // namespace ekm
