// Point index, built once per context (Algorithm 1 builds its point tree
// once, before the iteration loop; the node layout of the point index in the
// subsection on indexes over spatial vectors and centroids).
//
// GPU realisation: points are sorted along a Morton curve over the data
// bounding box and cut into group cells, the largest Morton cells (quadtree /
// octree cells) holding at most G * f points; each group cell is cut into
// leaves of f consecutive points (the last one shorter), so that a leaf fills
// a 64-lane wave.  (With KM_FLAG_CELL_LEAVES a leaf is instead the largest
// Morton cell holding at most f points: tighter boxes, fewer points per
// leaf.)  A leaf is a contiguous run of the sorted points, so a wave reads it
// with coalesced loads; each leaf
// keeps its exact FP32 bounding box (the box plays the role of the paper's
// ball pivot and radius) and the exact fixed-point sum of its points, so a
// leaf that falls wholly into one cluster updates that cluster's sum without
// reading its points (the paper's node-level sum-vector update).
//
// A context may hold several independent clouds (concatenated, cloud b owning
// points [pt_off[b], pt_off[b+1])): each gets its own Morton grid over its
// own bounding box, the sort orders points by (cloud, Morton key), and no
// leaf or group spans two clouds.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "ekm_internal.hpp"

namespace ekm {

// ------------------------------------------------------------ input scan
struct ScanOut {
    int32_t lo[3], hi[3]; // order-preserving integer images of float bounds
    int32_t nonfinite;
    int32_t neg_elsb; // max over nonzero coordinates of -(exponent of lowest set bit)
    int32_t emsb;     // max over nonzero coordinates of exponent of highest set bit
    int32_t any_nonzero;
};

// Order-preserving map float -> int32 (an involution on negative values).
__device__ inline int32_t ord_of(float f)
{
    int32_t i = __float_as_int(f);
    return i >= 0 ? i : (i ^ 0x7fffffff);
}
__host__ inline float float_of_ord(int32_t o)
{
    int32_t i = o >= 0 ? o : (o ^ 0x7fffffff);
    float f;
    __builtin_memcpy(&f, &i, 4);
    return f;
}

// Input scan, workgroup (b, y) over points of cloud b: the cloud's box goes
// to out[b], the non-finite flag and the exponent window (over all clouds)
// to out[B].
template <class T, int D>
__global__ void __launch_bounds__(256) k_scan_points(const T *x, const int64_t *pt_off, int B, ScanOut *outs)
{
    const int b = blockIdx.x;
    const int64_t p0 = pt_off[b], p1 = pt_off[b + 1];
    ScanOut *out = outs + b;
    ScanOut *glob = outs + B;
    float lo[D], hi[D];
    for (int i = 0; i < D; ++i) {
        lo[i] = INFINITY;
        hi[i] = -INFINITY;
    }
    int nonfin = 0, nelsb = -100000, emsb = -100000, anynz = 0;
    for (int64_t p = p0 + (int64_t)blockIdx.y * blockDim.x + threadIdx.x; p < p1; p += (int64_t)gridDim.y * blockDim.x) {
        for (int i = 0; i < D; ++i) {
            T v = x[p * D + i];
            if (!isfinite(v)) {
                nonfin = 1;
                continue;
            }
            float fv = (float)v;
            lo[i] = fminf(lo[i], fv);
            hi[i] = fmaxf(hi[i], fv);
            if (v != (T)0) {
                int el, em;
                if (sizeof(T) == 4)
                    bits_f32((float)v, el, em);
                else
                    bits_f64((double)v, el, em);
                nelsb = max(nelsb, -el);
                emsb = max(emsb, em);
                anynz = 1;
            }
        }
    }
    // the box is over the FP32 images of the coordinates, which is what
    // the Morton keys quantise; one lane per wave publishes the wave's result
    for (int i = 0; i < D; ++i) {
        lo[i] = wave_min_f32(lo[i]);
        hi[i] = -wave_min_f32(-hi[i]);
    }
    for (int o = 32; o >= 1; o >>= 1) {
        nonfin |= __shfl_xor(nonfin, o);
        nelsb = max(nelsb, __shfl_xor(nelsb, o));
        emsb = max(emsb, __shfl_xor(emsb, o));
        anynz |= __shfl_xor(anynz, o);
    }
    // then the workgroup's result, published by one thread (atomics on the
    // same words from every wave serialise)
    constexpr int NW = 256 / WAVE;
    __shared__ float slo[NW][D], shi[NW][D];
    __shared__ int sflag[NW][4];
    const int wv = threadIdx.x / WAVE;
    if (lane_id() == 0) {
        for (int i = 0; i < D; ++i) {
            slo[wv][i] = lo[i];
            shi[wv][i] = hi[i];
        }
        sflag[wv][0] = nonfin;
        sflag[wv][1] = nelsb;
        sflag[wv][2] = emsb;
        sflag[wv][3] = anynz;
    }
    __syncthreads();
    if (threadIdx.x != 0)
        return;
    for (int w = 1; w < NW; ++w) {
        for (int i = 0; i < D; ++i) {
            lo[i] = fminf(lo[i], slo[w][i]);
            hi[i] = fmaxf(hi[i], shi[w][i]);
        }
        nonfin |= sflag[w][0];
        nelsb = max(nelsb, sflag[w][1]);
        emsb = max(emsb, sflag[w][2]);
        anynz |= sflag[w][3];
    }
    for (int i = 0; i < D; ++i) {
        atomicMin(&out->lo[i], ord_of(lo[i]));
        atomicMax(&out->hi[i], ord_of(hi[i]));
    }
    if (nonfin)
        atomicOr(&glob->nonfinite, 1);
    if (anynz) {
        atomicMax(&glob->neg_elsb, nelsb);
        atomicMax(&glob->emsb, emsb);
        atomicOr(&glob->any_nonzero, 1);
    }
}

// ------------------------------------------------------------ keys, gather
// Morton key of every point on its cloud's grid (vals = the point index).
template <class T, int D>
__global__ void __launch_bounds__(256) k_point_keys(const T *x, int64_t n, const int64_t *pt_off, int B,
                                                    const Grid *grids, uint32_t *keys, int32_t *vals)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n)
        return;
    float q[D];
    for (int i = 0; i < D; ++i)
        q[i] = (float)x[p * D + i];
    keys[p] = morton_key<D>(q, grids[B == 1 ? 0 : cloud_of(pt_off, B, p)]);
    vals[p] = (int32_t)p;
}

// Cloud of every point, in the current order perm (the key of the stable
// sort by cloud that follows the sort by Morton key).
__global__ void __launch_bounds__(256) k_cloud_keys(const int32_t *perm, int64_t n, const int64_t *pt_off, int B,
                                                    uint32_t *keys)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        keys[i] = (uint32_t)cloud_of(pt_off, B, perm[i]);
}

// Morton keys in the final order (position i holds point perm[i], of the
// cloud that owns position i).
template <class T, int D>
__global__ void __launch_bounds__(256) k_keys_at(const T *x, const int32_t *perm, int64_t n, const int64_t *pt_off,
                                                 int B, const Grid *grids, uint32_t *keys)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t p = perm[i];
    float q[D];
    for (int d = 0; d < D; ++d)
        q[d] = (float)x[p * D + d];
    keys[i] = morton_key<D>(q, grids[cloud_of(pt_off, B, i)]);
}

template <class T, int D>
__global__ void __launch_bounds__(256) k_gather(const T *x, const int32_t *perm, int64_t n, T *xs)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n)
        return;
    int64_t src = perm[p];
    for (int i = 0; i < D; ++i)
        xs[(int64_t)i * n + p] = x[src * D + i];
}

// ------------------------------------------------------------ leaf cut
// Position i starts a new leaf iff the deepest Morton cell shared by points
// i-1 and i holds more than f points: then i-1 and i lie in different
// children of that cell, and their leaves (the largest cells with <= f
// points) differ.  Equal keys beyond f points are cut every f points.
//
// A cloud's first position always starts a leaf, and every search below
// stays inside the cloud of position i ([c_lo, c_hi)).
template <int D>
__global__ void __launch_bounds__(256) k_leaf_flags(const uint32_t *keys, int64_t n, int f, uint32_t *flag,
                                                    const int64_t *pt_off, int B)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int cl = B == 1 ? 0 : cloud_of(pt_off, B, i);
    const int64_t c_lo = pt_off[cl], c_hi = pt_off[cl + 1];
    if (i == c_lo) {
        flag[i] = 1;
        return;
    }
    const int KB = key_bits(D);
    uint32_t a = keys[i - 1], b = keys[i];
    uint32_t out;
    if (a == b) {
        int64_t lo = c_lo, hi = i; // first index with key == b
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (keys[mid] < b)
                lo = mid + 1;
            else
                hi = mid;
        }
        int64_t rs = lo;
        lo = i;
        hi = c_hi; // first index with key > b
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (keys[mid] <= b)
                lo = mid + 1;
            else
                hi = mid;
        }
        int64_t cntr = lo - rs;
        out = (cntr > f && ((i - rs) % f) == 0) ? 1u : 0u;
    } else {
        int lcp = __clz((int)(a ^ b)) - (32 - KB);
        int P = (lcp / D) * D; // bits of the deepest shared cell
        const uint32_t keymask = KB == 32 ? ~0u : ((1u << (KB & 31)) - 1u);
        uint32_t mask = P == 0 ? 0u : ((~0u) << (KB - P)) & keymask;
        uint32_t cell = b & mask;
        int64_t wlo = i - 1 - f < c_lo ? c_lo : i - 1 - f;
        int64_t lo = wlo, hi = i - 1; // first index in [wlo, i-1] inside the cell
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if ((keys[mid] & mask) < cell)
                lo = mid + 1;
            else
                hi = mid;
        }
        int64_t s = lo;
        int64_t whi = i + f + 1 > c_hi ? c_hi : i + f + 1;
        lo = i;
        hi = whi; // first index in [i, whi) past the cell
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if ((keys[mid] & mask) <= cell)
                lo = mid + 1;
            else
                hi = mid;
        }
        out = (lo - s > f) ? 1u : 0u;
    }
    flag[i] = out;
}

__global__ void __launch_bounds__(256) k_leaf_starts(const uint32_t *flag, const uint32_t *scan, int64_t n,
                                                     int32_t *leaf_start, int64_t L)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flag[i])
        leaf_start[scan[i]] = (int32_t)i;
    if (i == 0)
        leaf_start[L] = (int32_t)n;
}

// One wave per leaf: exact FP32 box and exact fixed-point coordinate sums.
template <int D>
__global__ void __launch_bounds__(256) k_leaf_info(const float *xs, int64_t n, const int32_t *leaf_start, int64_t L,
                                                   int S, float4 *box, int64_t *leaf_sum)
{
    int64_t l = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    if (l >= L)
        return; // whole wave leaves together
    int lane = lane_id();
    int32_t s = leaf_start[l], e = leaf_start[l + 1];
    bool valid = s + lane < e;
    float lo[4] = {0, 0, 0, 0}, hi[4] = {0, 0, 0, 0};
    for (int i = 0; i < D; ++i) {
        float v = valid ? xs[(int64_t)i * n + s + lane] : 0.0f;
        int64_t h, q;
        fix_split_f32(v, S, h, q);
        h = wave_sum_i64(valid ? h : 0);
        q = wave_sum_i64(valid ? q : 0);
        float mn = wave_min_f32(valid ? v : INFINITY);
        float mx = -wave_min_f32(valid ? -v : INFINITY);
        lo[i] = mn;
        hi[i] = mx;
        if (lane == 0) {
            leaf_sum[(l * D + i) * 2] = h;
            leaf_sum[(l * D + i) * 2 + 1] = q;
        }
    }
    if (lane == 0) {
        box[2 * l] = make_float4(lo[0], lo[1], lo[2], 0.0f);
        box[2 * l + 1] = make_float4(hi[0], hi[1], hi[2], 0.0f);
    }
}

// ------------------------------------------------------------ wave groups
// Leaves are grouped for the centroid-tree descent: a group is a run of at
// most G (<= GROUP_LEAVES) consecutive leaves inside one group cell, the
// largest Morton cell holding at most G * f points (the leaf rule at a
// coarser threshold).  Group boxes then stay inside one compact cell; runs
// of consecutive leaves across a Morton jump would give boxes spanning
// distant regions.  Every group-cell cut is a leaf cut (the threshold is a
// multiple of f), so cells are unions of whole leaves.

// cs[l] = 1 iff leaf l starts a group cell.
__global__ void __launch_bounds__(256) k_cell_starts(const uint32_t *pflag, const int32_t *leaf_start, int64_t L,
                                                     uint32_t *cs)
{
    int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l < L)
        cs[l] = pflag[leaf_start[l]];
}

// First leaf of each cell (cscan = exclusive scan of cs).
__global__ void __launch_bounds__(256) k_cell_first(const uint32_t *cs, const uint32_t *cscan, int64_t L,
                                                    int32_t *cell_first)
{
    int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l < L && cs[l])
        cell_first[cscan[l]] = (int32_t)l;
}

// ws[l] = 1 iff leaf l starts a group: its rank in its cell is a multiple of G.
__global__ void __launch_bounds__(256) k_group_starts(const uint32_t *cs, const uint32_t *cscan,
                                                      const int32_t *cell_first, int64_t L, int G, uint32_t *ws)
{
    int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= L)
        return;
    const int64_t cell = (int64_t)cscan[l] + cs[l] - 1;
    const int64_t rank = l - cell_first[cell];
    ws[l] = (rank % G) == 0 ? 1u : 0u;
}

// Cloud of every leaf (from its first point) and of every group (from its first leaf).
__global__ void __launch_bounds__(256) k_leaf_clouds(const int32_t *leaf_start, int64_t L, const int64_t *pt_off,
                                                     int B, int32_t *leaf_cloud)
{
    int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l < L)
        leaf_cloud[l] = B == 1 ? 0 : cloud_of(pt_off, B, leaf_start[l]);
}
__global__ void __launch_bounds__(256) k_group_clouds(const int32_t *group_leaf, int64_t ngroups,
                                                      const int32_t *leaf_cloud, int32_t *group_cloud)
{
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < ngroups)
        group_cloud[g] = leaf_cloud[group_leaf[g]];
}

__global__ void __launch_bounds__(256) k_group_first(const uint32_t *ws, const uint32_t *gscan, int64_t L,
                                                     int32_t *group_leaf, int64_t ngroups)
{
    int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l < L && ws[l])
        group_leaf[gscan[l]] = (int32_t)l;
    if (l == 0)
        group_leaf[ngroups] = (int32_t)L;
}

// One thread per group: union of its leaves' boxes.
__global__ void __launch_bounds__(256) k_group_boxes(const float4 *leaf_box, const int32_t *group_leaf,
                                                     int64_t ngroups, float4 *group_box)
{
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngroups)
        return;
    float4 lo = make_float4(INFINITY, INFINITY, INFINITY, 0.0f), hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.0f);
    for (int64_t l = group_leaf[g]; l < group_leaf[g + 1]; ++l) {
        float4 a = leaf_box[2 * l], b = leaf_box[2 * l + 1];
        lo.x = fminf(lo.x, a.x);
        lo.y = fminf(lo.y, a.y);
        lo.z = fminf(lo.z, a.z);
        hi.x = fmaxf(hi.x, b.x);
        hi.y = fmaxf(hi.y, b.y);
        hi.z = fmaxf(hi.z, b.z);
    }
    group_box[2 * g] = lo;
    group_box[2 * g + 1] = hi;
}

// ------------------------------------------------------------ driver
// Packed leaves.  cflag / cscan: group-cell starts over the sorted points and
// their exclusive scan; cell_first[c]: the first point of cell c.
__global__ void __launch_bounds__(256) k_cell_first_pt(const uint32_t *cflag, const uint32_t *cscan, int64_t n,
                                                       int32_t *cell_first)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && cflag[i])
        cell_first[cscan[i]] = (int32_t)i;
}

// lflag[i] = 1 iff point i starts a leaf: its rank in its group cell is a multiple of f.
__global__ void __launch_bounds__(256) k_packed_flags(const uint32_t *cflag, const uint32_t *cscan,
                                                      const int32_t *cell_first, int64_t n, int f, uint32_t *lflag)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int64_t c = (int64_t)cscan[i] + cflag[i] - 1;
    lflag[i] = ((i - cell_first[c]) % f) == 0 ? 1u : 0u;
}

// Group c = the leaves of group cell c (lscan: exclusive scan of the leaf starts).
__global__ void __launch_bounds__(256) k_packed_groups(const int32_t *cell_first, const uint32_t *lscan,
                                                       int64_t ncells, int64_t L, int32_t *group_leaf)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncells)
        group_leaf[c] = (int32_t)lscan[cell_first[c]];
    if (c == 0)
        group_leaf[ncells] = (int32_t)L;
}

static inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <class T, int D>
static km_status build_leaves_t(km_ctx *ctx, const T *x)
{
    hipStream_t st = ctx->stream;
    const int64_t n = ctx->n;
    const int B = ctx->B;
    const int64_t *pt_off = ctx->pt_off;
    // 1. input scan: each cloud's box, the non-finite flag and the exact-sum
    //    window over all clouds (slot B)
    std::vector<ScanOut> h0(B + 1);
    for (auto &o : h0) {
        for (int i = 0; i < 3; ++i) {
            o.lo[i] = 0x7fffffff;
            o.hi[i] = (int32_t)0x80000000;
        }
        o.nonfinite = 0;
        o.neg_elsb = -100000;
        o.emsb = -100000;
        o.any_nonzero = 0;
    }
    ScanOut *d0 = ctx_alloc<ScanOut>(ctx, B + 1);
    if (!d0) {
        set_error("kmeans_init: device allocation failed");
        return KM_ERR_OOM;
    }
    if (!hip_ok(hipMemcpyAsync(d0, h0.data(), (B + 1) * sizeof(ScanOut), hipMemcpyHostToDevice, st),
                "hipMemcpyAsync"))
        return KM_ERR_HIP;
    int64_t nmax = 0;
    for (int b = 0; b < B; ++b)
        nmax = std::max(nmax, ctx->h_pt_off[b + 1] - ctx->h_pt_off[b]);
    unsigned gy = nblocks(nmax, 256 * 4);
    gy = gy < 1 ? 1 : (gy > (B == 1 ? 1024u : 64u) ? (B == 1 ? 1024u : 64u) : gy);
    hipLaunchKernelGGL((k_scan_points<T, D>), dim3((unsigned)B, gy), dim3(256), 0, st, x, pt_off, B, d0);
    if (!hip_ok(hipMemcpyAsync(h0.data(), d0, (B + 1) * sizeof(ScanOut), hipMemcpyDeviceToHost, st),
                "hipMemcpyAsync") ||
        !hip_ok(hipStreamSynchronize(st), "hipStreamSynchronize"))
        return KM_ERR_HIP;
    const ScanOut &hg = h0[B];
    if (hg.nonfinite) {
        set_error("kmeans_init: points contain NaN or Inf");
        return KM_ERR_INVALID;
    }
    // exact-sum window
    int S = hg.any_nonzero ? hg.neg_elsb : 0;
    int logn = 0;
    while (((int64_t)1 << logn) < n)
        ++logn;
    int W = hg.any_nonzero ? hg.emsb + 1 + S + logn : 0;
    if (W > MAX_FIX_BITS) {
        set_error("kmeans_init: coordinates span " + std::to_string(W) +
                  " bits of fixed point; exact centroid sums support at most " + std::to_string(MAX_FIX_BITS));
        return KM_ERR_NOT_EXACT;
    }
    ctx->S = S;
    ctx->fix64 = (hg.any_nonzero ? hg.emsb + 1 + S : 0) <= FIX64_BITS ? 1 : 0;
    // each cloud's Morton grid over its own box
    ctx->h_grids.assign(B, Grid{});
    for (int b = 0; b < B; ++b)
        for (int i = 0; i < D; ++i) {
            float lo = float_of_ord(h0[b].lo[i]), hi = float_of_ord(h0[b].hi[i]);
            ctx->h_grids[b].lo[i] = lo;
            float ext = hi - lo;
            ctx->h_grids[b].scale[i] = ext > 0.0f ? (float)(1u << morton_bits(D)) / ext : 0.0f;
        }
    ctx->grid = ctx->h_grids[0];
    ctx->grids = ctx_alloc<Grid>(ctx, B);
    if (!ctx->grids) {
        set_error("kmeans_init: device allocation failed");
        return KM_ERR_OOM;
    }
    if (!hip_ok(hipMemcpyAsync(ctx->grids, ctx->h_grids.data(), B * sizeof(Grid), hipMemcpyHostToDevice, st),
                "hipMemcpyAsync"))
        return KM_ERR_HIP;
    // 2. sort by Morton key, then (several clouds) stably by cloud: the
    //    points are ordered by (cloud, Morton key)
    uint32_t *keys = ctx_alloc<uint32_t>(ctx, n), *keys2 = ctx_alloc<uint32_t>(ctx, n);
    int32_t *vals2 = ctx_alloc<int32_t>(ctx, n);
    ctx->perm = ctx_alloc<int32_t>(ctx, n);
    int64_t hist_len = (int64_t)radix_scratch_words(n);
    uint32_t *hist = ctx_alloc<uint32_t>(ctx, hist_len);
    uint32_t *scan_tmp = ctx_alloc<uint32_t>(ctx, scan_scratch_words(hist_len > n ? hist_len : n));
    if (!keys || !keys2 || !vals2 || !ctx->perm || !hist || !scan_tmp) {
        set_error("kmeans_init: device allocation failed");
        return KM_ERR_OOM;
    }
    hipLaunchKernelGGL((k_point_keys<T, D>), dim3(nblocks(n, 256)), dim3(256), 0, st, x, n, pt_off, B,
                       (const Grid *)ctx->grids, keys, ctx->perm);
    bool in_tmp = false;
    if (!hip_ok(radix_sort_u32(keys, ctx->perm, keys2, vals2, n, key_bits(D), hist, scan_tmp, st, &in_tmp),
                "radix sort"))
        return KM_ERR_HIP;
    uint32_t *skeys = in_tmp ? keys2 : keys;    // sorted keys
    uint32_t *flag = in_tmp ? keys : keys2;     // free buffer
    if (in_tmp &&
        !hip_ok(hipMemcpyAsync(ctx->perm, vals2, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st), "copy"))
        return KM_ERR_HIP;
    if (B > 1) {
        int cbits = 0;
        while ((1 << cbits) < B)
            ++cbits;
        hipLaunchKernelGGL(k_cloud_keys, dim3(nblocks(n, 256)), dim3(256), 0, st, ctx->perm, n, pt_off, B, skeys);
        in_tmp = false;
        if (!hip_ok(radix_sort_u32(skeys, ctx->perm, flag, vals2, n, cbits, hist, scan_tmp, st, &in_tmp),
                    "radix sort by cloud"))
            return KM_ERR_HIP;
        if (in_tmp &&
            !hip_ok(hipMemcpyAsync(ctx->perm, vals2, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st), "copy"))
            return KM_ERR_HIP;
        hipLaunchKernelGGL((k_keys_at<T, D>), dim3(nblocks(n, 256)), dim3(256), 0, st, x, ctx->perm, n, pt_off, B,
                           (const Grid *)ctx->grids, keys);
        skeys = keys;
        flag = keys2;
    }
    uint32_t *scan = (uint32_t *)vals2;         // free once perm is in place
    // 3. gather to SoA
    T *xs = ctx_alloc<T>(ctx, (size_t)n * D);
    if (!xs) {
        set_error("kmeans_init: device allocation failed");
        return KM_ERR_OOM;
    }
    ctx->xs = xs;
    hipLaunchKernelGGL((k_gather<T, D>), dim3(nblocks(n, 256)), dim3(256), 0, st, x, ctx->perm, n, xs);
    // 4. leaves
    const bool packed = sizeof(T) == 4 && ctx->cfg.algo == KM_INDEXED && !(ctx->cfg.flags & KM_FLAG_CELL_LEAVES);
    uint32_t last[2];
    int64_t ncells = 0;
    int32_t *cell_first = nullptr; // packed leaves: first point of each group cell (temporary)
    uint32_t *lflag = nullptr;
    struct FreeOnExit { // hipFree waits for the queued kernels that use the buffer
        void *p = nullptr;
        ~FreeOnExit()
        {
            if (p)
                (void)hipFree(p);
        }
    } tmp_guard;
    if (packed) {
        // group cells over the points, then leaves of f points inside each
        hipLaunchKernelGGL((k_leaf_flags<D>), dim3(nblocks(n, 256)), dim3(256), 0, st, skeys, n, ctx->G * ctx->f,
                           flag, pt_off, B);
        if (!hip_ok(hipMemcpyAsync(scan, flag, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st), "copy") ||
            !hip_ok(exclusive_scan_u32(scan, n, scan_tmp, st), "scan") ||
            !hip_ok(hipMemcpyAsync(&last[0], scan + n - 1, 4, hipMemcpyDeviceToHost, st), "copy") ||
            !hip_ok(hipMemcpyAsync(&last[1], flag + n - 1, 4, hipMemcpyDeviceToHost, st), "copy") ||
            !hip_ok(hipStreamSynchronize(st), "sync"))
            return KM_ERR_HIP;
        ncells = (int64_t)last[0] + last[1];
        if (hipMalloc((void **)&cell_first, (size_t)(ncells + n) * sizeof(int32_t)) != hipSuccess) {
            set_error("kmeans_init: device allocation failed");
            return KM_ERR_OOM;
        }
        tmp_guard.p = cell_first;
        lflag = (uint32_t *)(cell_first + ncells);
        hipLaunchKernelGGL(k_cell_first_pt, dim3(nblocks(n, 256)), dim3(256), 0, st, flag, scan, n, cell_first);
        hipLaunchKernelGGL(k_packed_flags, dim3(nblocks(n, 256)), dim3(256), 0, st, flag, scan,
                           (const int32_t *)cell_first, n, ctx->f, lflag);
        flag = lflag;
    } else {
        hipLaunchKernelGGL((k_leaf_flags<D>), dim3(nblocks(n, 256)), dim3(256), 0, st, skeys, n, ctx->f, flag, pt_off,
                           B);
    }
    if (!hip_ok(hipMemcpyAsync(scan, flag, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st), "copy") ||
        !hip_ok(exclusive_scan_u32(scan, n, scan_tmp, st), "scan"))
        return KM_ERR_HIP;
    if (!hip_ok(hipMemcpyAsync(&last[0], scan + n - 1, 4, hipMemcpyDeviceToHost, st), "copy") ||
        !hip_ok(hipMemcpyAsync(&last[1], flag + n - 1, 4, hipMemcpyDeviceToHost, st), "copy") ||
        !hip_ok(hipStreamSynchronize(st), "sync"))
        return KM_ERR_HIP;
    int64_t L = (int64_t)last[0] + last[1];
    ctx->L = L;
    // the rest of the workspace in one allocation, now that its sizes are
    // known (the leaf groups too with default leaves)
    ctx->groups_in_arena = packed;
    if (!ctx_arena(ctx, ctx_bytes_after_counts(ctx, L, ncells, packed))) {
        set_error("kmeans_init: device allocation failed");
        return KM_ERR_OOM;
    }
    ctx->leaf_start = ctx_alloc<int32_t>(ctx, L + 1);
    if (!ctx->leaf_start) {
        set_error("kmeans_init: device allocation failed");
        return KM_ERR_OOM;
    }
    hipLaunchKernelGGL(k_leaf_starts, dim3(nblocks(n, 256)), dim3(256), 0, st, flag, scan, n, ctx->leaf_start, L);
    if (sizeof(T) == 4 && ctx->cfg.algo == KM_INDEXED) {
        ctx->leaf_box = (float *)ctx_alloc<float4>(ctx, 2 * L);
        ctx->leaf_sum = ctx_alloc<int64_t>(ctx, (size_t)L * D * 2);
        ctx->leaf_cloud = ctx_alloc<int32_t>(ctx, L);
        if (!ctx->leaf_box || !ctx->leaf_sum || !ctx->leaf_cloud) {
            set_error("kmeans_init: device allocation failed");
            return KM_ERR_OOM;
        }
        hipLaunchKernelGGL((k_leaf_info<D>), dim3(nblocks(L * WAVE, 256)), dim3(256), 0, st, (const float *)xs, n,
                           ctx->leaf_start, L, S, (float4 *)ctx->leaf_box, ctx->leaf_sum);
        hipLaunchKernelGGL(k_leaf_clouds, dim3(nblocks(L, 256)), dim3(256), 0, st, (const int32_t *)ctx->leaf_start,
                           L, pt_off, B, ctx->leaf_cloud);
    }
    if (packed) { // one group per group cell
        ctx->ngroups = ncells;
        ctx->group_leaf = ctx_alloc_groups<int32_t>(ctx, ncells + 1);
        ctx->group_box = ctx_alloc_groups<float4>(ctx, 2 * ncells);
        ctx->group_cloud = ctx_alloc_groups<int32_t>(ctx, ncells);
        if (!ctx->group_leaf || !ctx->group_box || !ctx->group_cloud) {
            set_error("kmeans_init: device allocation failed");
            return KM_ERR_OOM;
        }
        hipLaunchKernelGGL(k_packed_groups, dim3(nblocks(ncells, 256)), dim3(256), 0, st, (const int32_t *)cell_first,
                           (const uint32_t *)scan, ncells, L, ctx->group_leaf);
        hipLaunchKernelGGL(k_group_boxes, dim3(nblocks(ncells, 256)), dim3(256), 0, st, (const float4 *)ctx->leaf_box,
                           (const int32_t *)ctx->group_leaf, ncells, ctx->group_box);
        hipLaunchKernelGGL(k_group_clouds, dim3(nblocks(ncells, 256)), dim3(256), 0, st,
                           (const int32_t *)ctx->group_leaf, ncells, (const int32_t *)ctx->leaf_cloud,
                           ctx->group_cloud);
        if (!hip_ok(hipStreamSynchronize(st), "sync"))
            return KM_ERR_HIP;
    } else if (sizeof(T) == 4 && ctx->cfg.algo == KM_INDEXED) {
        // wave groups (flag and scan are free again; the leaf-level arrays
        // live in scan, which holds n >= 4L words once L <= n/4, else in a
        // temporary): group cells are the leaf rule at G times the leaf size
        hipLaunchKernelGGL((k_leaf_flags<D>), dim3(nblocks(n, 256)), dim3(256), 0, st, skeys, n, ctx->G * ctx->f,
                           flag, pt_off, B);
        uint32_t *tmp = nullptr;
        uint32_t *lw = scan;
        if (4 * L > n) {
            if (hipMalloc((void **)&tmp, (size_t)4 * L * sizeof(uint32_t)) != hipSuccess) {
                set_error("kmeans_init: device allocation failed");
                return KM_ERR_OOM;
            }
            lw = tmp;
        }
        uint32_t *cs = lw, *cscan = lw + L, *ws = lw + 2 * L, *gscan = lw + 3 * L;
        int32_t *cell_first = (int32_t *)gscan; // used before gscan is written
        hipLaunchKernelGGL(k_cell_starts, dim3(nblocks(L, 256)), dim3(256), 0, st, flag, ctx->leaf_start, L, cs);
        bool ok = hip_ok(hipMemcpyAsync(cscan, cs, L * sizeof(uint32_t), hipMemcpyDeviceToDevice, st), "copy") &&
                  hip_ok(exclusive_scan_u32(cscan, L, scan_tmp, st), "scan");
        if (ok) {
            hipLaunchKernelGGL(k_cell_first, dim3(nblocks(L, 256)), dim3(256), 0, st, cs, cscan, L, cell_first);
            hipLaunchKernelGGL(k_group_starts, dim3(nblocks(L, 256)), dim3(256), 0, st, cs, cscan,
                               (const int32_t *)cell_first, L, ctx->G, ws);
            ok = hip_ok(hipMemcpyAsync(gscan, ws, L * sizeof(uint32_t), hipMemcpyDeviceToDevice, st), "copy") &&
                 hip_ok(exclusive_scan_u32(gscan, L, scan_tmp, st), "scan") &&
                 hip_ok(hipMemcpyAsync(&last[0], gscan + L - 1, 4, hipMemcpyDeviceToHost, st), "copy") &&
                 hip_ok(hipMemcpyAsync(&last[1], ws + L - 1, 4, hipMemcpyDeviceToHost, st), "copy") &&
                 hip_ok(hipStreamSynchronize(st), "sync");
        }
        if (ok) {
            ctx->ngroups = (int64_t)last[0] + last[1];
            ctx->group_leaf = ctx_alloc_groups<int32_t>(ctx, ctx->ngroups + 1);
            ctx->group_box = ctx_alloc_groups<float4>(ctx, 2 * ctx->ngroups);
            ctx->group_cloud = ctx_alloc_groups<int32_t>(ctx, ctx->ngroups);
            if (!ctx->group_leaf || !ctx->group_box || !ctx->group_cloud) {
                if (tmp)
                    (void)hipFree(tmp);
                set_error("kmeans_init: device allocation failed");
                return KM_ERR_OOM;
            }
            hipLaunchKernelGGL(k_group_first, dim3(nblocks(L, 256)), dim3(256), 0, st, ws, gscan, L, ctx->group_leaf,
                               ctx->ngroups);
            hipLaunchKernelGGL(k_group_boxes, dim3(nblocks(ctx->ngroups, 256)), dim3(256), 0, st,
                               (const float4 *)ctx->leaf_box, (const int32_t *)ctx->group_leaf, ctx->ngroups,
                               ctx->group_box);
            hipLaunchKernelGGL(k_group_clouds, dim3(nblocks(ctx->ngroups, 256)), dim3(256), 0, st,
                               (const int32_t *)ctx->group_leaf, ctx->ngroups, (const int32_t *)ctx->leaf_cloud,
                               ctx->group_cloud);
            ok = hip_ok(hipStreamSynchronize(st), "sync");
        }
        if (tmp)
            (void)hipFree(tmp);
        if (!ok)
            return KM_ERR_HIP;
    }
    // keep the sort scratch for the centroid sort of large k
    ctx->ckey = keys;
    ctx->ckey2 = keys2;
    ctx->cval2 = vals2;
    ctx->rs_hist = hist;
    ctx->rs_hist_len = hist_len;
    ctx->scan_tmp = scan_tmp;
    if (!hip_ok(hipGetLastError(), "leaf build launch"))
        return KM_ERR_HIP;
    return KM_OK;
}

size_t scan_record_bytes() { return sizeof(ScanOut); }

km_status build_leaves(km_ctx *ctx, const void *points)
{
    const bool f32 = ctx->cfg.point_dtype == KM_F32;
    if (ctx->d == 2)
        return f32 ? build_leaves_t<float, 2>(ctx, (const float *)points)
                   : build_leaves_t<double, 2>(ctx, (const double *)points);
    return f32 ? build_leaves_t<float, 3>(ctx, (const float *)points)
               : build_leaves_t<double, 3>(ctx, (const double *)points);
}

} // namespace ekm
