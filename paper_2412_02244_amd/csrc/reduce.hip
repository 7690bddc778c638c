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
// afresh and they are cleared here.  The workgroups after the cluster ones
// fold the per-block statistics and objective partials (fin_stats): exact
// integer counters, and the objective summed in a fixed order, so the
// reported counters and objective are deterministic.
#include "finalize.hpp"

namespace ekm {

template <int D>
__global__ void __launch_bounds__(FIN_THREADS) k_finalize(const double *c_in, double *c_out, int64_t k, int64_t *acc,
                                                          int32_t *cnt, int S, int reset, int64_t nclusterblocks,
                                                          FinStats F)
{
    // The cluster blocks run even when the run is over: every kernel of such
    // a step returned at once, so the sums are those of the last real step
    // and the centroids written are the same values again (the brute path's
    // cleared sums give c_out = c_in).  Only the statistics workgroups test
    // it, each before it takes its ticket, and only the last of them sets
    // it, so no workgroup races that write.
    if ((int64_t)blockIdx.x < nclusterblocks) {
        int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (j < k)
            fin_cluster<D>(j, c_in, c_out, acc, cnt, S, reset);
        return;
    }
    if (F.ctl[CTL_STOP])
        return; // a step after the end of the run: nothing to record (no workgroup takes a ticket)
    __shared__ FinShared fs;
    fin_stats(fs, F, (int64_t)blockIdx.x - nclusterblocks);
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

FinStats fin_stats_args(km_ctx *ctx, bool with_sse)
{
    FinStats F;
    F.nblk = assign_blocks(ctx);
    F.nheavy = ctx->cfg.algo == KM_INDEXED ? ctx->heavy_wgs : 0;
    F.stat_part = ctx->stat_part;
    F.nsse = with_sse ? ctx->nblk_sse : 0;
    F.sse_part = ctx->sse_part;
    F.stat_out = ctx->stat_out;
    F.sse_out = ctx->sse_out;
    F.cmax_bits = (unsigned *)ctx->cerr;
    F.drift_max = ctx->drift_max;
    F.heavy_cnt = ctx->heavy_cnt;
    F.ctl = ctx->ctl;
    F.stat_hist = ctx->stat_hist;
    F.hist_cap = ctx->hist_cap;
    F.nwg = fin_stat_wgs(F.nblk, fin_rows_per_wg(ctx->cfg.flags));
    F.wg_part = ctx->fin_part;
    F.ticket = ctx->fin_ticket;
    return F;
}

km_status run_finalize(km_ctx *ctx, const double *c_in, double *c_out, int32_t *assign_out, bool with_sse)
{
    hipStream_t st = ctx->stream;
    int64_t ncb = (ctx->k + FIN_THREADS - 1) / FIN_THREADS;
    const int reset = ctx->cfg.algo == KM_INDEXED ? 0 : 1;
    const FinStats F = fin_stats_args(ctx, with_sse);
    if (ctx->d == 2)
        hipLaunchKernelGGL(k_finalize<2>, dim3((unsigned)(ncb + F.nwg)), dim3(FIN_THREADS), 0, st, c_in, c_out,
                           ctx->k, ctx->acc, ctx->cnt, ctx->S, reset, ncb, F);
    else
        hipLaunchKernelGGL(k_finalize<3>, dim3((unsigned)(ncb + F.nwg)), dim3(FIN_THREADS), 0, st, c_in, c_out,
                           ctx->k, ctx->acc, ctx->cnt, ctx->S, reset, ncb, F);
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
