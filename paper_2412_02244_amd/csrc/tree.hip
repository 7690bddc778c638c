// Centroid index, rebuilt from the current centroids every iteration
// (Algorithm 1 rebuilds its centroid tree at the top of each pass of the
// loop; node layout in the subsection on indexes over spatial vectors and
// centroids).
//
// GPU realisation: centroids are rounded to FP32, sorted along the Morton
// curve of the data grid (ties by index), grouped into buckets of
// TREE_BUCKET consecutive centroids, and covered by an implicit balanced
// binary tree in heap order (node 1 = root, children 2i and 2i+1, bucket b =
// node 2^h + b).  Each node stores the exact FP32 bounding box of its
// centroids.  Splitting a Morton-sorted run at its middle halves the set
// along the interleaved coordinates, i.e. a kd-style split.  Padding nodes
// past the last bucket hold an empty (inverted) box, which every distance
// test prunes.
#include "ekm_internal.hpp"

namespace ekm {

constexpr int SMALL_K = 8192;
constexpr int TREE_THREADS = 1024;

// fl32 copy, Morton key, and a bound on max_j ||c_j|| for the rounding error
// bound ||c - fl32(c)|| <= 2^-24 ||c||.
template <int D>
__global__ void __launch_bounds__(256) k_centroid_prep(const double *c, int64_t k, Grid g, float4 *c32,
                                                       uint32_t *keys, int32_t *vals, unsigned *cmax_bits)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float nb = 0.0f;
    if (j < k) {
        float q[3] = {0.0f, 0.0f, 0.0f};
        double s = 0.0;
        for (int i = 0; i < D; ++i) {
            double v = c[j * D + i];
            q[i] = (float)v;
            s += v * v;
        }
        c32[j] = make_float4(q[0], q[1], q[2], 0.0f);
        keys[j] = morton_key<D>(q, g);
        vals[j] = (int32_t)j;
        double nrm = sqrt(s) * (1.0 + 0x1p-40);
        nb = (float)nrm;
        if ((double)nb < nrm)
            nb = nextafterf(nb, INFINITY);
    }
    // non-negative floats order like their bit patterns
    float m = -wave_min_f32(-nb);
    if (lane_id() == 0)
        atomicMax(cmax_bits, __float_as_uint(m));
}

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

// Whole tree in one workgroup for k <= SMALL_K: bitonic sort of
// (key << 32 | id) in LDS, then buckets and internal boxes level by level.
__global__ void __launch_bounds__(TREE_THREADS) k_tree_small(const float4 *c32, const uint32_t *keys, int64_t k,
                                                             int h, float4 *cs, float4 *node_lo, float4 *node_hi)
{
    extern __shared__ unsigned long long sk[]; // [P] then boxes
    int P = 1;
    while (P < k)
        P <<= 1;
    for (int i = threadIdx.x; i < P; i += blockDim.x)
        sk[i] = i < k ? (((unsigned long long)keys[i] << 32) | (unsigned)i) : ~0ull;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < P / 2; t += blockDim.x) {
                int lo = 2 * t - (t & (stride - 1));
                int hi = lo + stride;
                bool up = (lo & size) == 0;
                unsigned long long a = sk[lo], b = sk[hi];
                if ((a > b) == up) {
                    sk[lo] = b;
                    sk[hi] = a;
                }
            }
            __syncthreads();
        }
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        int id = (int)(sk[i] & 0xffffffffu);
        float4 p = c32[id];
        p.w = __int_as_float(id);
        cs[i] = p;
    }
    // boxes: LDS after the keys
    float4 *blo = (float4 *)(sk + P);
    int nleaf = 1 << h;
    float4 *bhi = blo + 2 * nleaf;
    int64_t nb = (k + TREE_BUCKET - 1) / TREE_BUCKET;
    for (int b = threadIdx.x; b < nleaf; b += blockDim.x) {
        float4 lo, hi;
        box_empty(lo, hi);
        if (b < nb)
            for (int64_t t = (int64_t)b * TREE_BUCKET; t < k && t < (int64_t)(b + 1) * TREE_BUCKET; ++t)
                box_add(lo, hi, c32[(int)(sk[t] & 0xffffffffu)]);
        blo[nleaf + b] = lo;
        bhi[nleaf + b] = hi;
    }
    __syncthreads();
    for (int lev = h - 1; lev >= 0; --lev) {
        int first = 1 << lev;
        for (int nidx = first + threadIdx.x; nidx < 2 * first; nidx += blockDim.x) {
            float4 lo = blo[2 * nidx], hi = bhi[2 * nidx];
            box_union(lo, hi, blo[2 * nidx + 1], bhi[2 * nidx + 1]);
            blo[nidx] = lo;
            bhi[nidx] = hi;
        }
        __syncthreads();
    }
    for (int i = 1 + threadIdx.x; i < 2 * nleaf; i += blockDim.x) {
        node_lo[i] = blo[i];
        node_hi[i] = bhi[i];
    }
}

// Large k: sorted ids come from the device radix sort.
__global__ void __launch_bounds__(256) k_tree_buckets(const float4 *c32, const int32_t *sorted_id, int64_t k, int h,
                                                      float4 *cs, float4 *node_lo, float4 *node_hi)
{
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nleaf = (int64_t)1 << h;
    if (b >= nleaf)
        return;
    float4 lo, hi;
    box_empty(lo, hi);
    for (int64_t t = b * TREE_BUCKET; t < k && t < (b + 1) * TREE_BUCKET; ++t) {
        int id = sorted_id[t];
        float4 p = c32[id];
        box_add(lo, hi, p);
        p.w = __int_as_float(id);
        cs[t] = p;
    }
    node_lo[nleaf + b] = lo;
    node_hi[nleaf + b] = hi;
}

__global__ void __launch_bounds__(TREE_THREADS) k_tree_up(int h, float4 *node_lo, float4 *node_hi)
{
    for (int lev = h - 1; lev >= 0; --lev) {
        int64_t first = (int64_t)1 << lev;
        for (int64_t nidx = first + threadIdx.x; nidx < 2 * first; nidx += blockDim.x) {
            float4 lo = node_lo[2 * nidx], hi = node_hi[2 * nidx];
            box_union(lo, hi, node_lo[2 * nidx + 1], node_hi[2 * nidx + 1]);
            node_lo[nidx] = lo;
            node_hi[nidx] = hi;
        }
        // device-scope fence: the next level reads boxes other threads wrote
        __threadfence();
        __syncthreads();
    }
}

km_status build_centroid_tree(km_ctx *ctx, const double *c_in)
{
    hipStream_t st = ctx->stream;
    const int64_t k = ctx->k;
    unsigned g = (unsigned)((k + 255) / 256);
    if (ctx->d == 2)
        hipLaunchKernelGGL(k_centroid_prep<2>, dim3(g), dim3(256), 0, st, c_in, k, ctx->grid, ctx->c32,
                           ctx->ckey, ctx->cval, (unsigned *)ctx->cerr);
    else
        hipLaunchKernelGGL(k_centroid_prep<3>, dim3(g), dim3(256), 0, st, c_in, k, ctx->grid, ctx->c32,
                           ctx->ckey, ctx->cval, (unsigned *)ctx->cerr);
    if (ctx->cfg.algo != KM_INDEXED) // the brute path needs only fl32(c) and the norm bound
        return hip_ok(hipGetLastError(), "centroid prep launch") ? KM_OK : KM_ERR_HIP;
    if (k <= SMALL_K) {
        int P = 1;
        while (P < k)
            P <<= 1;
        size_t lds = (size_t)P * 8 + (size_t)4 * ((size_t)1 << ctx->tree_h) * sizeof(float4);
        hipLaunchKernelGGL(k_tree_small, dim3(1), dim3(TREE_THREADS), lds, st, ctx->c32, ctx->ckey, k, ctx->tree_h,
                           ctx->cs, ctx->node_lo, ctx->node_hi);
    } else {
        bool in_tmp = false;
        if (!hip_ok(radix_sort_u32(ctx->ckey, ctx->cval, ctx->ckey2, ctx->cval2, k, key_bits(ctx->d), ctx->rs_hist,
                                   ctx->scan_tmp, st, &in_tmp),
                    "centroid radix sort"))
            return KM_ERR_HIP;
        const int32_t *sid = in_tmp ? ctx->cval2 : ctx->cval;
        int64_t nleaf = (int64_t)1 << ctx->tree_h;
        hipLaunchKernelGGL(k_tree_buckets, dim3((unsigned)((nleaf + 255) / 256)), dim3(256), 0, st, ctx->c32, sid, k,
                           ctx->tree_h, ctx->cs, ctx->node_lo, ctx->node_hi);
        hipLaunchKernelGGL(k_tree_up, dim3(1), dim3(TREE_THREADS), 0, st, ctx->tree_h, ctx->node_lo, ctx->node_hi);
    }
    if (!hip_ok(hipGetLastError(), "centroid tree launch"))
        return KM_ERR_HIP;
    return KM_OK;
}

} // namespace ekm

namespace ekm {
// Allow the single-workgroup tree kernel its full LDS budget (up to 128 KB at
// k = SMALL_K).
hipError_t tree_setup()
{
    size_t need = (size_t)SMALL_K * 8 + (size_t)4 * (SMALL_K / TREE_BUCKET) * sizeof(float4);
    hipError_t e = hipFuncSetAttribute((const void *)k_tree_small, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)need);
    (void)hipGetLastError(); // a refusal shows up as a launch error of large trees instead
    (void)e;
    return hipSuccess;
}
int tree_small_k() { return SMALL_K; }
} // namespace ekm
