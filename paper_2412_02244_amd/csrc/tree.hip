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
// The sort runs at every TREE_RESORT-th step; in between, the tree is
// rebuilt over the order it had (any grouping of the centroids gives exact
// boxes, a stale order only looser ones).
//
// Also here: the inter bound of Eq. (3) for every centroid (the distance to
// its nearest other centroid), by a pair scan inside the small-k tree launch
// or by a search of the large-k tree.
#include "ekm_internal.hpp"

namespace ekm {

constexpr int SMALL_K = TREE_SMALL_K;
constexpr int TREE_THREADS = 1024;
constexpr int TREE_WAVES = TREE_THREADS / WAVE;

__device__ inline void f4_to3(const float4 v, float *o)
{
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
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

// Upper bound (FP32) on the drift ||c_j - c_prev_j|| of a centroid since the
// previous step (Algorithm 1 computes it with the refined centroids).
template <int D>
__device__ inline float drift_bound(const double *c, const double *cp)
{
    double s = 0.0;
    for (int i = 0; i < D; ++i) {
        const double t = c[i] - cp[i];
        s += t * t;
    }
    const double r = sqrt(s) * (1.0 + 0x1p-40);
    float f = (float)r;
    if ((double)f < r)
        f = nextafterf(f, INFINITY);
    return f;
}

// Inter bound of Eq. (3): the distance from a centroid to its nearest other
// centroid, found by a nearest-neighbour search of the centroid tree (the
// paper runs a 2-NN query per centroid, whose first hit is the centroid
// itself).  Returns the smallest FP32 squared distance from cj (tree
// position self) to any other centroid, or s0 if none is below s0.  A node
// whose box min-distance is not below the best so far is skipped (its
// members' FP32 distances are at least that min-distance).  The bucket of
// `self` is scanned first, for a good starting bound.  The walk is
// depth-first over the implicit 8-ary tree without a stack: after a node
// it moves to the next sibling, or up to the parent's next sibling, so all
// its state stays in registers.
//   cent(q): fl32 centroid at tree position q;  box(l, i, lo, hi): box of
//   node i of level l.
//   lev_size: node count of every level (a copy in LDS: the level is
//   thread-dependent, and indexing the kernel-argument copy with it would
//   move that copy to scratch memory); nlev: levels.
template <int D, class Cent, class Box>
__device__ float nn_search(int64_t self, const float *cj, float s0, const int64_t *lev_size, int nlev, int64_t k,
                           Cent cent, Box box)
{
    float best = s0;
    const int64_t b0 = self / TREE_BUCKET;
    for (int64_t q = b0 * TREE_BUCKET; q < k && q < (b0 + 1) * TREE_BUCKET; ++q)
        if (q != self) {
            float c[3];
            cent(q, c);
            best = fminf(best, sqdist32<D>(cj, c));
        }
    const int top = nlev - 1;
    if (top == 0)
        return best; // a single bucket: scanned above
    int lev = top - 1;
    int64_t idx = 0; // first child of the root
    while (true) {
        float lo[3], hi[3];
        box(lev, idx, lo, hi);
        const bool enter = box_mind<D>(lo, hi, cj) < best;
        if (enter && lev > 0) { // descend to the first child
            --lev;
            idx *= 8;
            continue;
        }
        if (enter && idx != b0) // a bucket: scan its centroids
            for (int64_t q = idx * TREE_BUCKET; q < k && q < (idx + 1) * TREE_BUCKET; ++q) {
                float c[3];
                cent(q, c);
                best = fminf(best, sqdist32<D>(cj, c));
            }
        // next sibling, or climb until a parent has one
        while (lev < top && ((idx & 7) == 7 || idx + 1 >= lev_size[lev])) {
            idx >>= 3;
            ++lev;
        }
        if (lev >= top)
            break;
        ++idx;
    }
    return best;
}

// FP32 squared-distance bound for the search of centroid j: with U an upper
// bound on the exact distance from c_j to its nearest other centroid, the
// FP32 distance between their fl32 copies is at most lo_inverse(U, 2e).
// Eq. (9): U = cb_j of the previous step + drift of c_j + the largest drift.
__device__ inline float nn_bound(bool have_prev, float cb_hi_prev, float drift_j, float drift_max, float e)
{
    if (!have_prev)
        return INFINITY;
    const float U = (cb_hi_prev + drift_j + drift_max) * MARGIN_UP * MARGIN_UP;
    return lo_inverse(U, 2.0f * e);
}

__device__ inline float err_of(float cmax) { return cmax * 0x1p-24f * (1.0f + 0x1p-20f) + 0x1p-100f; }

// ------------------------------------------------------------------ small k
// Inter bound of Eq. (3) for clouds of k <= SMALL_K: for every centroid, the
// smallest FP32 squared distance from fl32(c_j) to another fl32 centroid of
// its cloud, by scanning all pairs.  A workgroup of PAIR_WAVES waves, wave w
// taking items[w]: lane l holds centroid first + l of a chunk and scans one
// slice of the chunk's cloud.  The s slices of a chunk sit in consecutive
// waves of one workgroup, so their minima meet in LDS and the slice-0 wave
// writes the result (no atomics, nothing to clear beforehand).  The fl32
// copies are rounded here from the FP64 centroids, as the tree rounds them.
// The keep tests turn cb_s into a lower bound on the exact distance between
// the FP64 centroids.
//   pmin: LDS, PAIR_WAVES * WAVE floats.
template <int D>
__device__ void pair_block(const double *c_all, const PairItem *items, unsigned *cb_s, float *pmin)
{
    const int lane = lane_id(), wid = (int)threadIdx.x / WAVE;
    const PairItem it = items[wid];
    const int first = uniform_int(it.first), c0 = uniform_int(it.c0), c1 = uniform_int(it.c1);
    const int sl = uniform_int(it.sl);
    const int t = sl & 0xff, s = sl >> 8;
    const int j = first + lane;
    float b0 = INFINITY, b1 = INFINITY; // two chains: shorter dependences
    if (first >= 0) {
        float cj[3] = {0.0f, 0.0f, 0.0f};
        if (j < c1)
            for (int a = 0; a < D; ++a)
                cj[a] = (float)c_all[(int64_t)j * D + a];
        // the slice's centroids i = c0 + t + m s, 64 at a time: lane l loads
        // number m0 + l, then each is broadcast to the wave (readlane)
        const int M = (c1 - c0 - t + s - 1) / s;
        for (int m0 = 0; m0 < M; m0 += WAVE) {
            const int i_l = c0 + t + (m0 + lane) * s;
            float q[3] = {0.0f, 0.0f, 0.0f};
            if (m0 + lane < M)
                for (int a = 0; a < D; ++a)
                    q[a] = (float)c_all[(int64_t)i_l * D + a];
            const int cnt = M - m0 < WAVE ? M - m0 : WAVE;
            auto dist = [&](int u) {
                float p[3] = {0.0f, 0.0f, 0.0f};
                for (int a = 0; a < D; ++a)
                    p[a] = rl_f(q[a], u);
                const float sv = sqdist32<D>(cj, p);
                return c0 + t + (m0 + u) * s != j ? sv : INFINITY;
            };
            int u = 0;
            for (; u + 1 < cnt; u += 2) {
                b0 = fminf(b0, dist(u));
                b1 = fminf(b1, dist(u + 1));
            }
            if (u < cnt)
                b0 = fminf(b0, dist(u));
        }
    }
    pmin[wid * WAVE + lane] = fminf(b0, b1);
    __syncthreads();
    if (first >= 0 && t == 0 && j < c1) {
        float m = pmin[wid * WAVE + lane];
        for (int w = 1; w < s; ++w)
            m = fminf(m, pmin[(wid + w) * WAVE + lane]);
        cb_s[j] = __float_as_uint(m); // non-negative floats order like their bit patterns
    }
}

// The wave items of the pair scan over clouds [0, B) (c_off: B + 1 host
// offsets), PAIR_WAVES per workgroup; returns the workgroup count and, if
// items is given, fills it.  A chunk is up to 64 consecutive centroids of one
// cloud.  Its cloud is split into s slices, s the smallest power of two with
// s * PAIR_SCAN >= k_b (at most PAIR_WAVES), so a wave scans about
// PAIR_SCAN centroids; the s waves of a chunk start at a multiple of s and
// therefore share a workgroup.  Unused waves are idle (first = -1).
constexpr int PAIR_SCAN = 64;
int64_t pair_plan(const int64_t *c_off, int B, std::vector<PairItem> *items)
{
    int64_t pos = 0; // waves placed
    for (int b = 0; b < B; ++b) {
        const int64_t c0 = c_off[b], c1 = c_off[b + 1], kb = c1 - c0;
        int s = 1;
        while (s < PAIR_WAVES && (int64_t)s * PAIR_SCAN < kb)
            s *= 2;
        for (int64_t j = c0; j < c1; j += WAVE) {
            const int64_t at = (pos + s - 1) / s * s;
            if (items) {
                items->resize((size_t)at, PairItem{-1, 0, 0, 0});
                for (int t = 0; t < s; ++t)
                    items->push_back(PairItem{(int32_t)j, (int32_t)c0, (int32_t)c1, t | (s << 8)});
            }
            pos = at + s;
        }
    }
    const int64_t nblk = (pos + PAIR_WAVES - 1) / PAIR_WAVES;
    if (items)
        items->resize((size_t)(nblk * PAIR_WAVES), PairItem{-1, 0, 0, 0});
    return nblk;
}

// Everything in one workgroup, LDS-resident after one read of the centroids:
// prep, the tree order, the tree-ordered copy and every node box; global
// memory is only written (and, between re-sorts, the previous order read).
// The Morton sort (stable LSD radix sort, 8-bit digits, top 16 key bits)
// runs on every TREE_RESORT-th step of a context; in between, the previous
// step's order is kept and only the boxes are recomputed from the current
// centroids.  Any grouping of the centroids gives exact boxes, so the order
// only affects how tight the boxes are (centroids move little from step to
// step), never which centroids are candidates.
// One workgroup per cloud (blockIdx.x < nclouds): its centroids are [T.c0,
// T.c0 + T.k) of the concatenated arrays, with tree positions local to the
// cloud and global ids in cs[].w.  The workgroups after those run the pair
// scan of the inter bound (pair_block), which reads only the FP64 centroids,
// so both run side by side in one launch.
// At most 64 VGPRs (8 waves per SIMD): two tree workgroups per CU when a
// launch covers many clouds.
static_assert(TREE_WAVES == PAIR_WAVES, "a pair-scan workgroup is a tree workgroup");
template <int D>
__global__ void __launch_bounds__(TREE_THREADS, 8) k_tree_small(const double *c_all, const TreeArgs *trees,
                                                             const Grid *grids, float4 *c32, unsigned *cmax_bits,
                                                             unsigned *cb_s, double *c_prev_all, unsigned *drift_max,
                                                             const PairItem *pairs, int nclouds, int kcap,
                                                             const int32_t *ctl)
{
    if (ctl[CTL_STOP])
        return; // the run is over (the whole workgroup returns)
    extern __shared__ unsigned char smem[];
    if ((int)blockIdx.x >= nclouds) {
        pair_block<D>(c_all, pairs + (int64_t)(blockIdx.x - nclouds) * PAIR_WAVES, cb_s, (float *)smem);
        return;
    }
    const int have_prev = uniform_int(ctl[CTL_STEPS] > 0 ? 1 : 0);
    // the cloud's tree layout, read once into (scalar) registers: the
    // phases below use it after barriers, where a read through T would be
    // a memory round trip each time
    const TreeArgs &T = trees[blockIdx.x];
    const Grid g = grids[blockIdx.x];
    const int64_t c0 = T.c0, k = T.k;
    float4 *const cs = T.cs, *const node_lo = T.node_lo, *const node_hi = T.node_hi;
    const int nnodes = uniform_int((int)T.nnodes), nlev = uniform_int(T.nlev);
    int lev_off[TREE_MAX_LEVELS], lev_size[TREE_MAX_LEVELS];
#pragma unroll
    for (int l = 0; l < TREE_MAX_LEVELS; ++l) {
        lev_off[l] = uniform_int(l < nlev ? (int)T.lev_off[l] : 0);
        lev_size[l] = uniform_int(l < nlev ? (int)T.lev_size[l] : 0);
    }
    const double *c = c_all + c0 * D;
    const int resort = uniform_int(ctl[CTL_STEPS] % TREE_RESORT == 0 ? 1 : 0);
    // kcap: the largest cloud of the launch, rounded up (small_tree_lds)
    float4 *cq = (float4 *)smem;              // [kcap] fl32 centroids, caller order
    uint32_t *key = (uint32_t *)(cq + kcap);  // [kcap]
    uint32_t *id = key + kcap;                // [kcap]
    uint32_t *key2 = id + kcap;               // [kcap]
    uint32_t *id2 = key2 + kcap;              // [kcap]
    uint32_t *wcnt = id2 + kcap;              // [TREE_WAVES][256]
    uint32_t *base = wcnt + TREE_WAVES * 256; // [256]
    __shared__ float red[TREE_WAVES], dred[TREE_WAVES];
    const int tid = threadIdx.x, lane = lane_id(), wid = tid / WAVE;
    const int kk = (int)k;
    const int shift = key_bits(D) - 16; // sort on the top 16 bits
    float nb = 0.0f, dm = 0.0f;
    double *c_prev = c_prev_all + c0 * D;
    for (int j = tid; j < kk; j += TREE_THREADS) {
        float4 q4;
        uint32_t kb;
        nb = fmaxf(nb, centroid_prep_one<D>(c, j, g, q4, kb));
        // drift since the previous step (bounds of the previous step's
        // assignment carry over with it), then the centroid becomes the
        // previous one of the next step
        if (have_prev)
            dm = fmaxf(dm, drift_bound<D>(c + j * D, c_prev + j * D));
        for (int i = 0; i < D; ++i)
            c_prev[j * D + i] = c[j * D + i];
        cq[j] = q4;
        c32[c0 + j] = q4;
        key[j] = kb >> shift;
        // the order to keep: tree position j held centroid T.cs[j].w (a global id)
        id[j] = resort ? (uint32_t)j : (uint32_t)(__float_as_int(cs[j].w) - (int)c0);
    }
    nb = -wave_min_f32(-nb);
    dm = -wave_min_f32(-dm);
    if (lane == 0) {
        red[wid] = nb;
        dred[wid] = dm;
    }
    __syncthreads();
    if (tid == 0) {
        float m = 0.0f, d = 0.0f;
        for (int w = 0; w < TREE_WAVES; ++w) {
            m = fmaxf(m, red[w]);
            d = fmaxf(d, dred[w]);
        }
        atomicMax(cmax_bits, __float_as_uint(m)); // over all clouds (non-negative floats order like their bits)
        atomicMax(drift_max, __float_as_uint(d));
    }
    if (resort) {
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
    }
    __syncthreads();
    // sorted ids are back in `id`; node boxes go to LDS (over key2/id2,
    // free now: room for kcap / 4 float4, see small_tree_lds) and out
    float4 *nlo = (float4 *)key2, *nhi = nlo + nnodes;
    for (int t = tid; t < kk; t += TREE_THREADS) {
        int cid = (int)id[t];
        float4 p = cq[cid];
        p.w = __int_as_float((int)c0 + cid);
        cs[t] = p;
    }
    const int nb0 = lev_size[0];
    for (int b = tid; b < nb0; b += TREE_THREADS) {
        float4 lo, hi;
        box_empty(lo, hi);
        const int tl = ((b + 1) * TREE_BUCKET < kk ? (b + 1) * TREE_BUCKET : kk) - 1; // the bucket's last
        // all loads at once: indices past the bucket's end repeat its last
        // centroid, which leaves the box unchanged
        // (the centroids in two batches of 4: fewer registers, so that two
        // tree workgroups still fit a CU when many clouds are launched)
        uint32_t ids[TREE_BUCKET];
#pragma unroll
        for (int u = 0; u < TREE_BUCKET; ++u)
            ids[u] = id[b * TREE_BUCKET + u < tl ? b * TREE_BUCKET + u : tl];
#pragma unroll
        for (int h = 0; h < TREE_BUCKET; h += 4) {
            float4 p[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                p[u] = cq[ids[h + u]];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                box_add(lo, hi, p[u]);
        }
        nlo[b] = lo;
        nhi[b] = hi;
        node_lo[b] = lo;
        node_hi[b] = hi;
    }
    __syncthreads();
#pragma unroll // constant level indices: the layout stays in registers
    for (int l = 1; l < TREE_MAX_LEVELS; ++l) {
        if (l >= nlev)
            break;
        const int off = lev_off[l], poff = lev_off[l - 1], psz = lev_size[l - 1];
        for (int i = tid; i < lev_size[l]; i += TREE_THREADS) {
            float4 lo, hi;
            box_empty(lo, hi);
            const int cl = (8 * i + 8 < psz ? 8 * i + 8 : psz) - 1; // the node's last child
            // two batches of 4 children, each batch's loads at once (a
            // repeated last child leaves the box unchanged)
#pragma unroll
            for (int h = 0; h < 8; h += 4) {
                float4 clo[4], chi[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int ch = 8 * i + h + u < cl ? 8 * i + h + u : cl;
                    clo[u] = nlo[poff + ch];
                    chi[u] = nhi[poff + ch];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    box_union(lo, hi, clo[u], chi[u]);
            }
            nlo[off + i] = lo;
            nhi[off + i] = hi;
            node_lo[off + i] = lo;
            node_hi[off + i] = hi;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ large k
template <int D>
__global__ void __launch_bounds__(256) k_centroid_prep(const double *c, int64_t k, Grid g, float4 *c32,
                                                       uint32_t *keys, int32_t *vals, unsigned *cmax_bits,
                                                       double *c_prev, float *drift, unsigned *drift_max,
                                                       const int32_t *ctl)
{
    if (ctl[CTL_STOP])
        return;
    const int have_prev = ctl[CTL_STEPS] > 0;
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float nb = 0.0f, dj = 0.0f;
    if (j < k) {
        float4 q4;
        uint32_t kb;
        nb = centroid_prep_one<D>(c, j, g, q4, kb);
        c32[j] = q4;
        if (keys) {
            keys[j] = kb;
            vals[j] = (int32_t)j;
        }
        if (c_prev) {
            if (have_prev)
                dj = drift_bound<D>(c + j * D, c_prev + j * D);
            drift[j] = dj;
            for (int i = 0; i < D; ++i)
                c_prev[j * D + i] = c[j * D + i];
        }
    }
    // non-negative floats order like their bit patterns; the workgroup's
    // maxima first, then one atomic per word and workgroup (atomics on one
    // word from every wave serialise)
    __shared__ float wm[256 / WAVE], wd[256 / WAVE];
    const float m = -wave_min_f32(-nb);
    const float dm = -wave_min_f32(-dj);
    if (lane_id() == 0) {
        wm[threadIdx.x / WAVE] = m;
        wd[threadIdx.x / WAVE] = dm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float bm = wm[0], bd = wd[0];
        for (int w = 1; w < (int)(blockDim.x / WAVE); ++w) {
            bm = fmaxf(bm, wm[w]);
            bd = fmaxf(bd, wd[w]);
        }
        atomicMax(cmax_bits, __float_as_uint(bm));
        if (c_prev)
            atomicMax(drift_max, __float_as_uint(bd));
    }
}

// Inter bound of every centroid (large k): the smallest FP32 squared distance
// from fl32(c_j) to another fl32 centroid (Eq. (3)), found with the tree.
// One wave per 8 consecutive tree positions (a bucket; the last wave takes
// the last 8, overlapping its neighbour, which computes the same values);
// lane 8c + r works for centroid c of the 8 on slice r of the candidates.
//  1. every centroid bounds its answer: by its distances to the other 7 of
//     the wave, and from the previous step by Eq. (9) (nn_bound); S = the
//     largest of these bounds;
//  2. one descent keeps the nodes within some centroid's bound of it (box
//     min-distance at most that bound; first tested for the wave's bounding
//     box and S).  box_mind and bb_mind round like sqdist32 and are
//     monotone, so they never exceed the FP32 distance to a member of the
//     node: every node holding the nearest other centroid of one of the 8
//     stays;
//  3. the 8 lanes of a centroid scan the centroids of the surviving buckets,
//     each lane every eighth, and their minima combine.
// The minimum over those candidates is then the minimum over all centroids,
// bit for bit.  If the frontier of a level outgrows fr_cap (NN_FR, or a few
// entries with KM_FLAG_SMALL_LISTS to test this), every lane of the wave
// searches on its own instead (nn_search, the same result).
constexpr int NN_FR = 512; // frontier entries per wave and buffer
constexpr int NN_WAVES = 4;
constexpr int NN_GROUP = 8; // centroids per wave
template <int D>
__global__ void __launch_bounds__(NN_WAVES * WAVE) k_centroid_nn(TreeArgs T, int64_t k, const unsigned *cmax_bits,
                                                                const float *drift, const unsigned *drift_max,
                                                                unsigned *cb_s, float *cb_hi, int fr_cap,
                                                                const int32_t *ctl)
{
    static_assert(NN_GROUP * NN_GROUP == WAVE, "8 centroids x 8 slices per wave");
    if (ctl[CTL_STOP])
        return;
    const int have_prev = ctl[CTL_STEPS] > 0;
    __shared__ int64_t lev_size_sh[TREE_MAX_LEVELS], lev_off_sh[TREE_MAX_LEVELS];
    __shared__ int32_t fr[NN_WAVES][2][NN_FR]; // fr_cap <= NN_FR of each buffer in use
    if (threadIdx.x < TREE_MAX_LEVELS) {
        lev_size_sh[threadIdx.x] = T.lev_size[threadIdx.x];
        lev_off_sh[threadIdx.x] = T.lev_off[threadIdx.x];
    }
    __syncthreads();
    const int lane = lane_id(), wid = (int)threadIdx.x / WAVE;
    const int c = lane / NN_GROUP, r = lane % NN_GROUP;
    int64_t w0 = ((int64_t)blockIdx.x * NN_WAVES + wid) * NN_GROUP;
    if (w0 >= k)
        return; // a whole wave past the end (k >= 8 on this path)
    if (w0 + NN_GROUP > k)
        w0 = k - NN_GROUP;
    w0 = uniform_int((int)w0);
    const int64_t t = w0 + c; // this lane's centroid (tree position)
    const float e = err_of(__uint_as_float(*cmax_bits));
    const float4 p = T.cs[t];
    const int j = __float_as_int(p.w);
    float cj[3] = {p.x, p.y, p.z};
    // 1. bounds: lane (c, r) measures centroid c against centroid r
    float q[3];
    for (int a = 0; a < 3; ++a)
        q[a] = __shfl(cj[a], r * NN_GROUP); // centroid r sits in lanes 8r..8r+7
    float u = r != c ? sqdist32<D>(cj, q) : INFINITY;
    u = fminf(u, __shfl_xor(u, 1));
    u = fminf(u, __shfl_xor(u, 2));
    u = fminf(u, __shfl_xor(u, 4));
    const float s0 = nn_bound(have_prev != 0, have_prev ? cb_hi[j] : 0.0f, drift[j], __uint_as_float(*drift_max), e);
    const float bnd = fminf(u, s0);               // this centroid's bound
    const float S = -wave_min_f32(-bnd);          // the largest bound of the 8
    float blo[3], bhi[3];
    for (int a = 0; a < 3; ++a) {
        blo[a] = wave_min_f32(cj[a]);
        bhi[a] = -wave_min_f32(-cj[a]);
    }
    // a node can hold the nearest other centroid of centroid g only if its
    // box min-distance to c_g is at most g's bound (box_mind rounds like
    // sqdist32 and is monotone too)
    float gx[NN_GROUP][3], gb[NN_GROUP]; // the 8 centroids and their bounds, wave-uniform
    for (int g = 0; g < NN_GROUP; ++g) {
        for (int a = 0; a < 3; ++a)
            gx[g][a] = rl_f(cj[a], NN_GROUP * g);
        gb[g] = rl_f(bnd, NN_GROUP * g);
    }
    auto wanted = [&](const float *lo, const float *hi) {
        if (bb_mind<D>(blo, bhi, lo, hi) > S)
            return false;
        bool any = false;
        for (int g = 0; g < NN_GROUP; ++g)
            any = any || box_mind<D>(lo, hi, gx[g]) <= gb[g];
        return any;
    };
    // 2. descent from the root, keeping the wanted nodes
    int32_t *cur = fr[wid][0], *nxt = fr[wid][1];
    int ncur = 1;
    if (lane == 0)
        cur[0] = 0; // the root (level nlev - 1)
    bool overflow = false;
    for (int lev = T.nlev - 1; lev > 0 && !overflow; --lev) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int64_t csz = lev_size_sh[lev - 1], coff = lev_off_sh[lev - 1];
        int nnext = 0;
        for (int c0 = 0; c0 < 8 * ncur; c0 += WAVE) {
            const int ch = c0 + lane;
            int64_t child = -1;
            if (ch < 8 * ncur) {
                const int64_t nd = 8 * (int64_t)cur[ch >> 3] + (ch & 7);
                if (nd < csz) {
                    float lo[3], hi[3];
                    f4_to3(T.node_lo[coff + nd], lo);
                    f4_to3(T.node_hi[coff + nd], hi);
                    if (wanted(lo, hi))
                        child = nd;
                }
            }
            const uint64_t keep = __ballot(child >= 0);
            const int at = nnext + __popcll(keep & lanemask_lt());
            if (child >= 0 && at < fr_cap)
                nxt[at] = (int32_t)child;
            nnext += __popcll(keep);
        }
        nnext = uniform_int(nnext);
        if (nnext > fr_cap)
            overflow = true;
        int32_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
        ncur = nnext;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float sm;
    if (!overflow) {
        // 3. lane (c, r): candidates r, r + 8, ... of the surviving buckets
        float b0 = INFINITY, b1 = INFINITY;
        const int ncand = 8 * ncur;
        int m = r;
        for (; m + NN_GROUP < ncand; m += 2 * NN_GROUP) {
            const int64_t p0 = 8 * (int64_t)cur[m >> 3] + (m & 7);
            const int64_t p1 = 8 * (int64_t)cur[(m + NN_GROUP) >> 3] + ((m + NN_GROUP) & 7);
            if (p0 < k && p0 != t) {
                float x[3];
                f4_to3(T.cs[p0], x);
                b0 = fminf(b0, sqdist32<D>(cj, x));
            }
            if (p1 < k && p1 != t) {
                float x[3];
                f4_to3(T.cs[p1], x);
                b1 = fminf(b1, sqdist32<D>(cj, x));
            }
        }
        if (m < ncand) {
            const int64_t p0 = 8 * (int64_t)cur[m >> 3] + (m & 7);
            if (p0 < k && p0 != t) {
                float x[3];
                f4_to3(T.cs[p0], x);
                b0 = fminf(b0, sqdist32<D>(cj, x));
            }
        }
        sm = fminf(b0, b1);
        sm = fminf(sm, __shfl_xor(sm, 1));
        sm = fminf(sm, __shfl_xor(sm, 2));
        sm = fminf(sm, __shfl_xor(sm, 4));
    } else {
        auto cent = [&](int64_t qq, float *o) { f4_to3(T.cs[qq], o); };
        auto box = [&](int l, int64_t i, float *lo, float *hi) {
            const int64_t o = lev_off_sh[l] + i;
            f4_to3(T.node_lo[o], lo);
            f4_to3(T.node_hi[o], hi);
        };
        // bnd is attained (u) or bounds the answer (s0): the search returns
        // min(bnd, the minimum), which is the minimum
        sm = nn_search<D>(t, cj, bnd, lev_size_sh, T.nlev, k, cent, box);
    }
    if (r == 0) {
        cb_s[j] = __float_as_uint(sm);
        cb_hi[j] = dist_hi(sm, 2.0f * e); // the next step's search bound (Eq. (9))
    }
}

// Buckets of the large-k tree: tree position t holds centroid sorted_id[t],
// or, without a new sort (sorted_id null), the centroid it held in the last
// build (its id in cs[t].w; the context starts with the identity order).
__global__ void __launch_bounds__(256) k_tree_buckets(const float4 *c32, const int32_t *sorted_id, int64_t k,
                                                      TreeArgs T, const int32_t *ctl)
{
    if (ctl[CTL_STOP])
        return;
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= T.lev_size[0])
        return;
    float4 lo, hi;
    box_empty(lo, hi);
    // the bucket's ids, then its centroids, each batch of loads issued at
    // once (the stores below would otherwise order every load after them);
    // positions past the bucket's end repeat its last centroid, which
    // leaves the box unchanged, and are not written
    const int64_t t0 = b * TREE_BUCKET, tl = ((b + 1) * TREE_BUCKET < k ? (b + 1) * TREE_BUCKET : k) - 1;
    int ids[TREE_BUCKET];
#pragma unroll
    for (int u = 0; u < TREE_BUCKET; ++u) {
        const int64_t t = t0 + u < tl ? t0 + u : tl;
        ids[u] = sorted_id ? sorted_id[t] : __float_as_int(T.cs[t].w);
    }
    float4 p[TREE_BUCKET];
#pragma unroll
    for (int u = 0; u < TREE_BUCKET; ++u)
        p[u] = c32[ids[u]];
#pragma unroll
    for (int u = 0; u < TREE_BUCKET; ++u) {
        box_add(lo, hi, p[u]);
        if (t0 + u <= tl) {
            p[u].w = __int_as_float(ids[u]);
            T.cs[t0 + u] = p[u];
        }
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

// Every level from l0 up, in one workgroup: level l0 - 1 (at most
// TREE_UPPER_CAP nodes) is read once into LDS, and each level above is
// built there from its children and written out (one launch instead of
// one per level; the levels are stored one after the other, level 0 first).
constexpr int TREE_UPPER_CAP = 2048, TREE_UPPER_SPAN = 2560, TREE_UPPER_THREADS = 1024;
// the nodes from level l0 - 1 up: P <= TREE_UPPER_CAP, then at most
// ceil(P / 8) + ceil(P / 64) + ... <= P / 7 + one per level
static_assert(TREE_UPPER_SPAN >= TREE_UPPER_CAP + TREE_UPPER_CAP / 7 + TREE_MAX_LEVELS, "the levels fit the LDS");
__global__ void __launch_bounds__(TREE_UPPER_THREADS) k_tree_upper(TreeArgs T, int l0)
{
    __shared__ float4 blo[TREE_UPPER_SPAN], bhi[TREE_UPPER_SPAN];
    const int tid = threadIdx.x;
    const int64_t base = T.lev_off[l0 - 1];
    const int P = (int)T.lev_size[l0 - 1];
    for (int i = tid; i < P; i += TREE_UPPER_THREADS) {
        blo[i] = T.node_lo[base + i];
        bhi[i] = T.node_hi[base + i];
    }
    __syncthreads();
    for (int l = l0; l < T.nlev; ++l) {
        const int off = (int)(T.lev_off[l] - base), poff = (int)(T.lev_off[l - 1] - base);
        const int psz = (int)T.lev_size[l - 1], n = (int)T.lev_size[l];
        for (int i = tid; i < n; i += TREE_UPPER_THREADS) {
            float4 lo, hi;
            box_empty(lo, hi);
            for (int ch = 8 * i; ch < 8 * i + 8 && ch < psz; ++ch)
                box_union(lo, hi, blo[poff + ch], bhi[poff + ch]);
            blo[off + i] = lo;
            bhi[off + i] = hi;
            T.node_lo[base + off + i] = lo;
            T.node_hi[base + off + i] = hi;
        }
        __syncthreads();
    }
}

// LDS of the small-k tree launch for clouds of at most kcap centroids (a
// multiple of 64): fl32 copies, two key/id buffers, the per-wave digit
// counts and the digit bases.  The pair-scan workgroups use its first
// PAIR_WAVES * WAVE floats.
static size_t small_tree_lds(int kcap)
{
    return (size_t)kcap * 16 + (size_t)kcap * 16 + (size_t)TREE_WAVES * 256 * 4 + 256 * 4;
}
static_assert(PAIR_WAVES * WAVE * 4 <= TREE_WAVES * 256 * 4, "the pair minima fit the smallest tree LDS");

// kcap of a context: its largest cloud, rounded up to a multiple of 64, and
// large enough that every cloud's node boxes (32 bytes a node) fit in the
// key2/id2 region (8 kcap bytes).
int small_tree_cap(const int64_t *c_off, int B)
{
    int64_t m = 0, nodes = 0;
    for (int b = 0; b < B; ++b) {
        const int64_t kb = c_off[b + 1] - c_off[b];
        TreeArgs T;
        tree_layout(kb, T);
        m = kb > m ? kb : m;
        nodes = T.nnodes > nodes ? T.nnodes : nodes;
    }
    int64_t kcap = (m + 63) / 64 * 64;
    if (kcap < 64)
        kcap = 64;
    while (nodes * 32 > kcap * 8)
        kcap += 64;
    return (int)kcap;
}
static_assert(2 * (SMALL_K / TREE_BUCKET + SMALL_K / TREE_BUCKET / 7 + 8) * 16 <= SMALL_K * 8,
              "node boxes of the largest small tree fit in LDS");

// Every cloud's tree is built by one workgroup (k of each cloud at most SMALL_K).
bool small_trees(const km_ctx *ctx)
{
    for (int b = 0; b < ctx->B; ++b)
        if (ctx->h_c_off[b + 1] - ctx->h_c_off[b] > SMALL_K)
            return false;
    return true;
}

// resort: sort the large-k tree's centroids along the Morton curve (else
// keep the last build's order; any order gives exact boxes, a stale one
// only looser ones).  The small-k tree decides this on the device.
km_status build_centroid_tree(km_ctx *ctx, const double *c_in, bool resort)
{
    hipStream_t st = ctx->stream;
    const int64_t k = ctx->k;
    unsigned *cmax = (unsigned *)ctx->cerr;
    const int32_t *hp = ctx->ctl;
    if (ctx->cfg.algo == KM_INDEXED && small_trees(ctx)) {
        const unsigned nb = (unsigned)(ctx->B + ctx->npair_blocks);
        if (ctx->d == 2)
            hipLaunchKernelGGL(k_tree_small<2>, dim3(nb), dim3(TREE_THREADS), small_tree_lds(ctx->tree_kcap), st, c_in,
                               (const TreeArgs *)ctx->trees, (const Grid *)ctx->grids, ctx->c32, cmax, ctx->cb_s,
                               ctx->c_prev, ctx->drift_max, (const PairItem *)ctx->pair_items, ctx->B, ctx->tree_kcap, hp);
        else
            hipLaunchKernelGGL(k_tree_small<3>, dim3(nb), dim3(TREE_THREADS), small_tree_lds(ctx->tree_kcap), st, c_in,
                               (const TreeArgs *)ctx->trees, (const Grid *)ctx->grids, ctx->c32, cmax, ctx->cb_s,
                               ctx->c_prev, ctx->drift_max, (const PairItem *)ctx->pair_items, ctx->B, ctx->tree_kcap, hp);
        return hip_ok(hipGetLastError(), "centroid tree launch") ? KM_OK : KM_ERR_HIP;
    }
    unsigned g = (unsigned)((k + 255) / 256);
    const bool indexed = ctx->cfg.algo == KM_INDEXED;
    uint32_t *keys = indexed && resort ? ctx->ckey : nullptr;
    double *cprev = indexed ? ctx->c_prev : nullptr;
    if (ctx->d == 2)
        hipLaunchKernelGGL(k_centroid_prep<2>, dim3(g), dim3(256), 0, st, c_in, k, ctx->grid, ctx->c32, keys,
                           ctx->cval, cmax, cprev, ctx->drift, ctx->drift_max, hp);
    else
        hipLaunchKernelGGL(k_centroid_prep<3>, dim3(g), dim3(256), 0, st, c_in, k, ctx->grid, ctx->c32, keys,
                           ctx->cval, cmax, cprev, ctx->drift, ctx->drift_max, hp);
    if (!indexed) // the brute path needs only fl32(c) and the norm bound
        return hip_ok(hipGetLastError(), "centroid prep launch") ? KM_OK : KM_ERR_HIP;
    const int32_t *sid = nullptr;
    if (resort) {
        bool in_tmp = false;
        if (!hip_ok(radix_sort_u32(ctx->ckey, ctx->cval, ctx->ckey2, ctx->cval2, k, key_bits(ctx->d), ctx->rs_hist,
                                   ctx->scan_tmp, st, &in_tmp),
                    "centroid radix sort"))
            return KM_ERR_HIP;
        sid = in_tmp ? ctx->cval2 : ctx->cval;
    }
    const TreeArgs &T = ctx->tree;
    hipLaunchKernelGGL(k_tree_buckets, dim3((unsigned)((T.lev_size[0] + 255) / 256)), dim3(256), 0, st, ctx->c32,
                       sid, k, T, hp);
    // levels over large ones, one launch each; then every level above in one
    int l = 1;
    for (; l < T.nlev && T.lev_size[l - 1] > TREE_UPPER_CAP; ++l)
        hipLaunchKernelGGL(k_tree_level, dim3((unsigned)((T.lev_size[l] + 255) / 256)), dim3(256), 0, st, T, l);
    if (l < T.nlev)
        hipLaunchKernelGGL(k_tree_upper, dim3(1), dim3(TREE_UPPER_THREADS), 0, st, T, l);
    const unsigned gnn = (unsigned)((k + NN_WAVES * NN_GROUP - 1) / (NN_WAVES * NN_GROUP));
    if (ctx->d == 2)
        hipLaunchKernelGGL(k_centroid_nn<2>, dim3(gnn), dim3(NN_WAVES * WAVE), 0, st, T, k, (const unsigned *)cmax,
                           (const float *)ctx->drift, (const unsigned *)ctx->drift_max, ctx->cb_s, ctx->cb_hi,
                           ctx->small_lists ? 16 : NN_FR, hp);
    else
        hipLaunchKernelGGL(k_centroid_nn<3>, dim3(gnn), dim3(NN_WAVES * WAVE), 0, st, T, k, (const unsigned *)cmax,
                           (const float *)ctx->drift, (const unsigned *)ctx->drift_max, ctx->cb_s, ctx->cb_hi,
                           ctx->small_lists ? 16 : NN_FR, hp);
    return hip_ok(hipGetLastError(), "centroid tree launch") ? KM_OK : KM_ERR_HIP;
}

// Allow the single-workgroup tree kernel its LDS budget.
hipError_t tree_setup()
{
    int need = (int)small_tree_lds(SMALL_K);
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
