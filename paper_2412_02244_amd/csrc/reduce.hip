// Centroid refinement (Algorithm 1: each centroid becomes the sum of its
// cluster divided by the cluster size), finishing the exact sums that the
// assignment kernels accumulated.
//
// The paper keeps running sum vectors and updates them when points move;
// rounding would make such sums depend on the order of moves.  Here each
// iteration's sums are exact integers (fixed point, summed with integer
// atomics, so independent of block order), rounded once to the nearest
// double and divided by the count in IEEE FP64.  An empty cluster keeps its
// previous centroid.  The last block folds the per-block statistics in a
// fixed order, so the reported counters and objective are deterministic.
#include "ekm_internal.hpp"

namespace ekm {

constexpr int FIN_THREADS = 256;

template <int D>
__global__ void __launch_bounds__(FIN_THREADS) k_finalize(const double *c_in, double *c_out, int64_t k, int64_t *acc,
                                                          int32_t *cnt, int S, int64_t nblk, const int64_t *stat_part,
                                                          const double *sse_part, int64_t *stat_out, double *sse_out,
                                                          unsigned *cmax_bits, int32_t *heavy_cnt,
                                                          int64_t nclusterblocks)
{
    if ((int64_t)blockIdx.x < nclusterblocks) {
        int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (j >= k)
            return;
        int32_t c = cnt[j];
        int64_t *aj = acc + j * D * 2;
        double out[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            if (c > 0) {
                double sum = fix_to_double(aj[2 * i], aj[2 * i + 1], S);
                out[i] = sum / (double)c; // IEEE-correct FP64 division
            } else {
                out[i] = c_in[j * D + i];
            }
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            c_out[j * D + i] = out[i];
            aj[2 * i] = 0;
            aj[2 * i + 1] = 0;
        }
        cnt[j] = 0;
        return;
    }
    // statistics block: each thread folds whole rows (NSTAT counters) of the
    // per-block partials, then a fixed-shape tree combines the threads
    __shared__ long long red[NSTAT][FIN_THREADS];
    __shared__ double dred[FIN_THREADS];
    long long acc8[NSTAT];
    for (int q = 0; q < NSTAT; ++q)
        acc8[q] = 0;
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < nblk; b += blockDim.x) {
        const longlong2 *row = (const longlong2 *)(stat_part + b * NSTAT);
#pragma unroll
        for (int q = 0; q < NSTAT / 2; ++q) {
            longlong2 v = row[q];
            acc8[2 * q] += v.x;
            acc8[2 * q + 1] += v.y;
        }
        s += sse_part[b];
    }
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
    if (threadIdx.x < NSTAT)
        stat_out[threadIdx.x] = red[threadIdx.x][0];
    if (threadIdx.x == 0) {
        *sse_out = dred[0];
        *cmax_bits = 0u; // the next centroid tree recomputes the norm bound
        if (heavy_cnt)
            *heavy_cnt = 0; // the deferred-leaf list of the next step starts empty
    }
}

__global__ void __launch_bounds__(256) k_scatter_assign(const int32_t *a, const int32_t *perm, int64_t n,
                                                        int32_t *out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[perm[i]] = a[i];
}

int64_t assign_blocks(const km_ctx *ctx);

km_status run_finalize(km_ctx *ctx, const double *c_in, double *c_out, int32_t *assign_out)
{
    hipStream_t st = ctx->stream;
    int64_t ncb = (ctx->k + FIN_THREADS - 1) / FIN_THREADS;
    int64_t nblk = assign_blocks(ctx);
    if (ctx->d == 2)
        hipLaunchKernelGGL(k_finalize<2>, dim3((unsigned)(ncb + 1)), dim3(FIN_THREADS), 0, st, c_in, c_out, ctx->k,
                           ctx->acc, ctx->cnt, ctx->S, nblk, ctx->stat_part, ctx->sse_part, ctx->stat_out,
                           ctx->sse_out, (unsigned *)ctx->cerr, ctx->heavy_cnt, ncb);
    else
        hipLaunchKernelGGL(k_finalize<3>, dim3((unsigned)(ncb + 1)), dim3(FIN_THREADS), 0, st, c_in, c_out, ctx->k,
                           ctx->acc, ctx->cnt, ctx->S, nblk, ctx->stat_part, ctx->sse_part, ctx->stat_out,
                           ctx->sse_out, (unsigned *)ctx->cerr, ctx->heavy_cnt, ncb);
    if (!hip_ok(hipGetLastError(), "finalize launch"))
        return KM_ERR_HIP;
    return assign_out ? scatter_assignment(ctx, assign_out) : KM_OK;
}

// Current assignment (Morton order inside the context) -> caller order.
km_status scatter_assignment(km_ctx *ctx, int32_t *assign_out)
{
    hipLaunchKernelGGL(k_scatter_assign, dim3((unsigned)((ctx->n + 255) / 256)), dim3(256), 0, ctx->stream, ctx->a,
                       ctx->perm, ctx->n, assign_out);
    if (!hip_ok(hipGetLastError(), "scatter launch"))
        return KM_ERR_HIP;
    return KM_OK;
}

} // namespace ekm
