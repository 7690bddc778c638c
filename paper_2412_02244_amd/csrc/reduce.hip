// Centroid refinement (Algorithm 1: each centroid becomes the sum of its
// cluster divided by the cluster size), from the exact sums that the
// assignment kernels maintain.
//
// The sums are exact integers (fixed point), so their value does not depend
// on the order in which blocks added to them; each is rounded once to the
// nearest double and divided by the count in IEEE FP64.  An empty cluster
// keeps its previous centroid.  On the indexed path the sums persist from
// step to step (moves between clusters update them) and are only brought
// back to their normal limb form here; on the brute path every step sums
// afresh and they are cleared here.  The last block folds the per-block
// statistics and objective partials in a fixed order, so the reported
// counters and objective are deterministic.
#include "ekm_internal.hpp"

namespace ekm {

constexpr int FIN_THREADS = 256;

template <int D>
__global__ void __launch_bounds__(FIN_THREADS) k_finalize(const double *c_in, double *c_out, int64_t k, int64_t *acc,
                                                          int32_t *cnt, int S, int reset, int64_t nblk,
                                                          const int64_t *stat_part, int64_t nsse,
                                                          const double *sse_part, int64_t *stat_out, double *sse_out,
                                                          unsigned *cmax_bits, unsigned *drift_max,
                                                          int32_t *heavy_cnt, int64_t nclusterblocks, int32_t *ctl,
                                                          int64_t *stat_hist, int64_t hist_cap)
{
    // The cluster blocks run even when the run is over: every kernel of such
    // a step returned at once, so the sums are those of the last real step
    // and the centroids written are the same values again (the brute path's
    // cleared sums give c_out = c_in).  Only the statistics block, which
    // alone sets CTL_STOP, tests it, so no block races that write.
    if ((int64_t)blockIdx.x < nclusterblocks) {
        int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (j >= k)
            return;
        int32_t c = cnt[j];
        int64_t *aj = acc + j * D * 2;
        double out[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const __int128 V = ((__int128)aj[2 * i] << 32) + (__int128)aj[2 * i + 1];
            out[i] = c > 0 ? fix128_to_double(V, S) / (double)c // IEEE-correct FP64 division
                           : c_in[j * D + i];
            // normal form (hi, lo in [0, 2^32)) for the next step's updates, or cleared
            aj[2 * i] = reset ? 0 : (int64_t)(V >> 32);
            aj[2 * i + 1] = reset ? 0 : (int64_t)(V & (__int128)0xffffffff);
        }
#pragma unroll
        for (int i = 0; i < D; ++i)
            c_out[j * D + i] = out[i];
        if (reset)
            cnt[j] = 0;
        return;
    }
    // statistics block: each thread folds whole rows (NSTAT counters) of the
    // per-block partials, then a fixed-shape tree combines the threads
    if (ctl[CTL_STOP])
        return; // a step after the end of the run: nothing to record
    __shared__ long long red[NSTAT][FIN_THREADS];
    __shared__ double dred[FIN_THREADS];
    long long acc8[NSTAT];
    for (int q = 0; q < NSTAT; ++q)
        acc8[q] = 0;
    for (int64_t b = threadIdx.x; b < nblk; b += blockDim.x) {
        const longlong2 *row = (const longlong2 *)(stat_part + b * NSTAT);
#pragma unroll
        for (int q = 0; q < NSTAT / 2; ++q) {
            longlong2 v = row[q];
            acc8[2 * q] += v.x;
            acc8[2 * q + 1] += v.y;
        }
    }
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < nsse; b += blockDim.x)
        s += sse_part[b];
    for (int q = 0; q < NSTAT; ++q)
        red[q][threadIdx.x] = acc8[q];
    dred[threadIdx.x] = s;
    __syncthreads();
    for (int o = FIN_THREADS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            for (int q = 0; q < NSTAT; ++q)
                red[q][threadIdx.x] += red[q][threadIdx.x + o];
            dred[threadIdx.x] += dred[threadIdx.x + o];
        }
        __syncthreads();
    }
    const int it = ctl[CTL_RUN_ITERS]; // this step's index in the run
    if (threadIdx.x < NSTAT) {
        stat_out[threadIdx.x] = red[threadIdx.x][0];
        if (stat_hist && it < hist_cap)
            stat_hist[it * (NSTAT + 1) + threadIdx.x] = red[threadIdx.x][0];
    }
    if (threadIdx.x == 0) {
        if (stat_hist && it < hist_cap)
            stat_hist[it * (NSTAT + 1) + NSTAT] = __double_as_longlong(dred[0]);
        // loop control: the run ends after max_iter steps, or at the first
        // step t >= 2 whose assignment equals that of step t - 1
        ctl[CTL_RUN_ITERS] = it + 1;
        ctl[CTL_STEPS] += 1;
        if (it + 1 >= ctl[CTL_MAX_ITER] || (ctl[CTL_STABLE] && it >= 1 && red[ST_CHANGED][0] == 0))
            ctl[CTL_STOP] = 1;
        *sse_out = dred[0];
        *cmax_bits = 0u; // the next centroid tree recomputes the norm bound
        if (drift_max)
            *drift_max = 0u; // and the largest drift
        if (heavy_cnt)
            *heavy_cnt = 0; // the deferred-leaf list of the next step starts empty
    }
}

// Caller order and cloud-local centroid ids (position i of the Morton order
// belongs to the cloud whose point range holds i).
__global__ void __launch_bounds__(256) k_scatter_assign(const int32_t *a, const int32_t *perm, int64_t n,
                                                        const int64_t *pt_off, const int64_t *c_off, int B,
                                                        int32_t *out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[perm[i]] = B == 1 ? a[i] : a[i] - (int32_t)c_off[cloud_of(pt_off, B, i)];
}

int64_t assign_blocks(km_ctx *ctx);

km_status run_finalize(km_ctx *ctx, const double *c_in, double *c_out, int32_t *assign_out, bool with_sse)
{
    hipStream_t st = ctx->stream;
    int64_t ncb = (ctx->k + FIN_THREADS - 1) / FIN_THREADS;
    int64_t nblk = assign_blocks(ctx);
    const int reset = ctx->cfg.algo == KM_INDEXED ? 0 : 1;
    const int64_t nsse = with_sse ? ctx->nblk_sse : 0;
    if (ctx->d == 2)
        hipLaunchKernelGGL(k_finalize<2>, dim3((unsigned)(ncb + 1)), dim3(FIN_THREADS), 0, st, c_in, c_out, ctx->k,
                           ctx->acc, ctx->cnt, ctx->S, reset, nblk, ctx->stat_part, nsse, ctx->sse_part,
                           ctx->stat_out, ctx->sse_out, (unsigned *)ctx->cerr, ctx->drift_max, ctx->heavy_cnt, ncb,
                           ctx->ctl, ctx->stat_hist, ctx->hist_cap);
    else
        hipLaunchKernelGGL(k_finalize<3>, dim3((unsigned)(ncb + 1)), dim3(FIN_THREADS), 0, st, c_in, c_out, ctx->k,
                           ctx->acc, ctx->cnt, ctx->S, reset, nblk, ctx->stat_part, nsse, ctx->sse_part,
                           ctx->stat_out, ctx->sse_out, (unsigned *)ctx->cerr, ctx->drift_max, ctx->heavy_cnt, ncb,
                           ctx->ctl, ctx->stat_hist, ctx->hist_cap);
    if (!hip_ok(hipGetLastError(), "finalize launch"))
        return KM_ERR_HIP;
    return assign_out ? scatter_assignment(ctx, assign_out) : KM_OK;
}

// Loop control: a run of max_iter steps (stable: stop when the assignment
// is stable), or, with reset_run, the state outside runs (no limit); the
// context's step count is kept.
__global__ void k_set_ctl(int32_t *ctl, int32_t max_iter, int32_t stable)
{
    if (threadIdx.x == 0) {
        ctl[CTL_STOP] = max_iter > 0 ? 0 : 1;
        ctl[CTL_RUN_ITERS] = 0;
        ctl[CTL_MAX_ITER] = max_iter;
        ctl[CTL_STABLE] = stable;
    }
}

km_status set_ctl(km_ctx *ctx, int32_t max_iter, int32_t stable, int32_t reset_run)
{
    if (reset_run) {
        max_iter = 0x7fffffff;
        stable = 0;
    }
    hipLaunchKernelGGL(k_set_ctl, dim3(1), dim3(64), 0, ctx->stream, ctx->ctl, max_iter, stable);
    return hip_ok(hipGetLastError(), "loop control launch") ? KM_OK : KM_ERR_HIP;
}

// Current assignment (Morton order inside the context) -> caller order.
km_status scatter_assignment(km_ctx *ctx, int32_t *assign_out)
{
    hipLaunchKernelGGL(k_scatter_assign, dim3((unsigned)((ctx->n + 255) / 256)), dim3(256), 0, ctx->stream, ctx->a,
                       ctx->perm, ctx->n, (const int64_t *)ctx->pt_off, (const int64_t *)ctx->c_off, ctx->B,
                       assign_out);
    if (!hip_ok(hipGetLastError(), "scatter launch"))
        return KM_ERR_HIP;
    return KM_OK;
}

} // namespace ekm
