// Centroid refinement and per-step statistics (the finalize kernel's two
// kinds of workgroup).
#pragma once

#include "ekm_internal.hpp"

namespace ekm {

constexpr int FIN_THREADS = 256;

struct FinShared {
    long long red[NSTAT][FIN_THREADS / WAVE]; // per-wave totals
    double dred[FIN_THREADS / WAVE];
    int last;
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

// Workgroups that fold the statistics rows: one per `rows` rows (8 per
// thread, or a few rows with KM_FLAG_SMALL_LISTS, which tests the
// hand-over), at most FIN_MAX_STAT_WG.  Below that a single workgroup
// folds them all: the hand-over costs more than it saves.
constexpr int FIN_MAX_STAT_WG = 256;
inline int fin_rows_per_wg(uint32_t flags) { return (flags & KM_FLAG_SMALL_LISTS) ? 8 : 8 * FIN_THREADS; }
inline int64_t fin_stat_wgs(int64_t nblk, int rows)
{
    const int64_t p = (nblk + rows - 1) / rows;
    return p < 1 ? 1 : (p > FIN_MAX_STAT_WG ? FIN_MAX_STAT_WG : p);
}

struct FinStats {
    int64_t nblk;               // rows of per-block counters
    int64_t nheavy;             // the last rows belong to the per-leaf pass: skipped when it had no leaf
    const int64_t *stat_part;   // [nblk][NSTAT]
    int64_t nsse;               // objective partials (0: none)
    const double *sse_part;
    int64_t nwg;                // folding workgroups (fin_stat_wgs)
    int64_t *wg_part;           // [nwg][NSTAT + 1]: each one's totals (the objective's bits last)
    int32_t *ticket;            // folding workgroups done this step (0 between steps)
    int64_t *stat_out;          // [NSTAT]
    double *sse_out;
    unsigned *cmax_bits;        // reset for the next step's centroid tree
    unsigned *drift_max;        // (may be null)
    int32_t *heavy_cnt;         // (may be null)
    int32_t *ctl;
    int64_t *stat_hist;         // (may be null)
    int64_t hist_cap;
};

// The step's statistics, folded by F.nwg workgroups of FIN_THREADS threads
// (w = 0 .. nwg - 1).  Workgroup w folds rows [w R, (w + 1) R) of the
// per-block partials (and the same share of the objective partials), each
// thread whole rows, then its threads are combined in a fixed order.  With
// several workgroups, each writes its totals, and the last one to finish
// (a ticket counter) adds them up in workgroup order.  Integer counters
// are exact in any order and the objective is summed in a fixed order, so
// the totals do not depend on timing.  The last workgroup also runs the
// loop control: the run ends after max_iter steps, or at the first step
// t >= 2 whose assignment equals that of step t - 1.
__device__ inline void fin_stats(FinShared &fs, const FinStats &F, int64_t w)
{
    // the per-leaf pass writes its rows only when it had leaves (the count
    // is read before the last workgroup clears it)
    const int64_t nrows = F.heavy_cnt && *F.heavy_cnt == 0 ? F.nblk - F.nheavy : F.nblk;
    const int64_t R = (nrows + F.nwg - 1) / F.nwg, Rs = (F.nsse + F.nwg - 1) / F.nwg;
    const int64_t r1 = (w + 1) * R < nrows ? (w + 1) * R : nrows;
    const int64_t s1 = (w + 1) * Rs < F.nsse ? (w + 1) * Rs : F.nsse;
    long long acc8[NSTAT];
    for (int q = 0; q < NSTAT; ++q)
        acc8[q] = 0;
#pragma unroll 4 // independent rows: several in flight at once
    for (int64_t b = w * R + threadIdx.x; b < r1; b += FIN_THREADS) {
        const longlong2 *row = (const longlong2 *)(F.stat_part + b * NSTAT);
#pragma unroll
        for (int q = 0; q < NSTAT / 2; ++q) {
            longlong2 v = row[q];
            acc8[2 * q] += v.x;
            acc8[2 * q + 1] += v.y;
        }
    }
    double s = 0.0;
    for (int64_t b = w * Rs + threadIdx.x; b < s1; b += FIN_THREADS)
        s += F.sse_part[b];
    // each wave sums its lanes (a fixed order), then thread q adds the wave
    // totals of value q in wave order
    const int wv = (int)threadIdx.x / WAVE;
    for (int q = 0; q < NSTAT; ++q) {
        const int64_t v = wave_sum_i64(acc8[q]);
        if (lane_id() == 0)
            fs.red[q][wv] = v;
    }
    const double dv = wave_sum_f64(s);
    if (lane_id() == 0)
        fs.dred[wv] = dv;
    __syncthreads();
    if (threadIdx.x < NSTAT) {
        long long t = fs.red[threadIdx.x][0];
        for (int u = 1; u < FIN_THREADS / WAVE; ++u)
            t += fs.red[threadIdx.x][u];
        fs.red[threadIdx.x][0] = t;
    } else if (threadIdx.x == NSTAT) {
        double d = fs.dred[0];
        for (int u = 1; u < FIN_THREADS / WAVE; ++u)
            d += fs.dred[u];
        fs.dred[0] = d;
    }
    __syncthreads();
    if (F.nwg > 1) {
        // hand this workgroup's totals over; the last workgroup folds them
        if (threadIdx.x < NSTAT)
            F.wg_part[w * (NSTAT + 1) + threadIdx.x] = fs.red[threadIdx.x][0];
        if (threadIdx.x == NSTAT)
            F.wg_part[w * (NSTAT + 1) + NSTAT] = __double_as_longlong(fs.dred[0]);
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0)
            fs.last = atomicAdd(F.ticket, 1) == (int)F.nwg - 1;
        __syncthreads();
        if (!fs.last)
            return;
        __threadfence();
        if (threadIdx.x <= NSTAT) {
            const int q = threadIdx.x;
            long long t = 0;
            double d = 0.0;
            for (int64_t u = 0; u < F.nwg; ++u) {
                const long long v = __atomic_load_n(F.wg_part + u * (NSTAT + 1) + q, __ATOMIC_RELAXED);
                if (q < NSTAT)
                    t += v;
                else
                    d += __longlong_as_double(v);
            }
            if (q < NSTAT)
                fs.red[q][0] = t;
            else
                fs.dred[0] = d;
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
        if (F.nwg > 1)
            *F.ticket = 0;
    }
}

} // namespace ekm
