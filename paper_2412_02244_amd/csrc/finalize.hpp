// Centroid refinement and per-step statistics (the finalize kernel's two
// kinds of workgroup).
#pragma once

#include "ekm_internal.hpp"

namespace ekm {

constexpr int FIN_THREADS = 256;

struct FinShared {
    long long red[NSTAT][FIN_THREADS];
    double dred[FIN_THREADS];
};

// Cluster j: c_out[j] = RN(exact sum) / count (IEEE FP64 division), or
// c_in[j] for an empty cluster; the limbs go back to normal form (hi,
// lo in [0, 2^32)) for the next step's updates, or are cleared (reset).
template <int D>
__device__ inline void fin_cluster(int64_t j, const double *c_in, double *c_out, int64_t *acc, int32_t *cnt, int S,
                                   int reset)
{
    const int32_t c = cnt[j];
    int64_t *aj = acc + j * D * 2;
    double out[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const __int128 V = ((__int128)aj[2 * i] << 32) + (__int128)aj[2 * i + 1];
        out[i] = c > 0 ? fix128_to_double(V, S) / (double)c : c_in[j * D + i];
        aj[2 * i] = reset ? 0 : (int64_t)(V >> 32);
        aj[2 * i + 1] = reset ? 0 : (int64_t)(V & (__int128)0xffffffff);
    }
#pragma unroll
    for (int i = 0; i < D; ++i)
        c_out[j * D + i] = out[i];
    if (reset)
        cnt[j] = 0;
}

struct FinStats {
    int64_t nblk;               // rows of per-block counters
    const int64_t *stat_part;   // [nblk][NSTAT]
    int64_t nsse;               // objective partials (0: none)
    const double *sse_part;
    int64_t *stat_out;          // [NSTAT]
    double *sse_out;
    unsigned *cmax_bits;        // reset for the next step's centroid tree
    unsigned *drift_max;        // (may be null)
    int32_t *heavy_cnt;         // (may be null)
    int32_t *ctl;
    int64_t *stat_hist;         // (may be null)
    int64_t hist_cap;
};

// The step's statistics (a workgroup of FIN_THREADS threads): each thread
// folds whole rows of the per-block partials, then a fixed-shape tree
// combines the threads, so the totals do not depend on timing.  Also the
// loop control: the run ends after max_iter steps, or at the first step
// t >= 2 whose assignment equals that of step t - 1.
__device__ inline void fin_stats(FinShared &fs, const FinStats &F)
{
    long long acc8[NSTAT];
    for (int q = 0; q < NSTAT; ++q)
        acc8[q] = 0;
    for (int64_t b = threadIdx.x; b < F.nblk; b += FIN_THREADS) {
        const longlong2 *row = (const longlong2 *)(F.stat_part + b * NSTAT);
#pragma unroll
        for (int q = 0; q < NSTAT / 2; ++q) {
            longlong2 v = row[q];
            acc8[2 * q] += v.x;
            acc8[2 * q + 1] += v.y;
        }
    }
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < F.nsse; b += FIN_THREADS)
        s += F.sse_part[b];
    for (int q = 0; q < NSTAT; ++q)
        fs.red[q][threadIdx.x] = acc8[q];
    fs.dred[threadIdx.x] = s;
    __syncthreads();
    for (int o = FIN_THREADS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            for (int q = 0; q < NSTAT; ++q)
                fs.red[q][threadIdx.x] += fs.red[q][threadIdx.x + o];
            fs.dred[threadIdx.x] += fs.dred[threadIdx.x + o];
        }
        __syncthreads();
    }
    const int it = F.ctl[CTL_RUN_ITERS]; // this step's index in the run
    if (threadIdx.x < NSTAT) {
        F.stat_out[threadIdx.x] = fs.red[threadIdx.x][0];
        if (F.stat_hist && it < F.hist_cap)
            F.stat_hist[it * (NSTAT + 1) + threadIdx.x] = fs.red[threadIdx.x][0];
    }
    if (threadIdx.x == 0) {
        if (F.stat_hist && it < F.hist_cap)
            F.stat_hist[it * (NSTAT + 1) + NSTAT] = __double_as_longlong(fs.dred[0]);
        F.ctl[CTL_RUN_ITERS] = it + 1;
        F.ctl[CTL_STEPS] += 1;
        if (it + 1 >= F.ctl[CTL_MAX_ITER] || (F.ctl[CTL_STABLE] && it >= 1 && fs.red[ST_CHANGED][0] == 0))
            F.ctl[CTL_STOP] = 1;
        *F.sse_out = fs.dred[0];
        *F.cmax_bits = 0u; // the next centroid tree recomputes the norm bound
        if (F.drift_max)
            *F.drift_max = 0u; // and the largest drift
        if (F.heavy_cnt)
            *F.heavy_cnt = 0; // the deferred-leaf list of the next step starts empty
    }
}

} // namespace ekm
